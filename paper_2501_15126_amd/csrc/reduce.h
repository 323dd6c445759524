// reduce.h -- launcher of the precompiled fixed-order final reduction.
#pragma once

#include <hip/hip_runtime.h>

namespace permx {

// out[0] + out[1] = double-double sum of partials[2b] + partials[2b+1],
// b = 0..count-1, in an order fixed by b; count_out[0] = sum of counts[b].
// Asynchronous on `stream`.
hipError_t launch_final_reduce(const double *partials, const unsigned long long *counts, long long count,
                               double *out, unsigned long long *count_out, hipStream_t stream);

// Exact mode: out[0..1] = column sums of count (residue, sum |term|) pairs,
// in an order fixed by the index.
hipError_t launch_final_reduce_x(const double *xparts, long long count, double *out, hipStream_t stream);

}  // namespace permx
