// reduce.h -- launchers of the precompiled fixed-order final reduction.
#pragma once

#include <hip/hip_runtime.h>

namespace permx {

// First-stage workgroups (slices) for `count` partials; the caller's stage
// buffer holds 6 doubles per slice.
long long final_reduce_slices(long long count);

// out[0] + out[1] = double-double sum of partials[2b] + partials[2b+1],
// b = 0..count-1, in an order fixed by count; out[2] holds the bits of the
// sum of counts[b]; with xparts (exact mode), out[3] and out[4] are the sums
// of xparts[2b] and xparts[2b+1] (residues: exact integer sums).  Two
// launches on `stream` (slices, then their sum), asynchronous.
hipError_t launch_final_reduce(const double *partials, const unsigned long long *counts, const double *xparts,
                               long long count, double *stage, double *out, hipStream_t stream);

}  // namespace permx
