// batch.h -- precompiled (non-generated) kernels for many matrices at once.
//
// Per-matrix hipRTC compilation costs 0.1-1.5 s, far more than the GPU time
// of a small permanent, so batches and served requests use kernels compiled
// once into the library, templated on the number of 4-row groups NG of x.
// The matrix arrives as data: after Alg. 4 ordering each flipped column j is
// stored as dense 4-row groups 0..top[j]; a Gray step adds whole groups
// (entries the column lacks add 0) and refreshes the cached suffix products
// of groups top[j]..0.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch_types.h"

namespace permx {

// Launches the batch kernel for items [0, nitems) whose matrices all have ng
// groups.  Item i writes its double-double partial to partials[2*items[i].out].
hipError_t launch_batch_items(int ng, const BatchItem *items, int64_t nitems, const BatchMat *mats,
                              const double *vals, const int32_t *tops, double *partials, hipStream_t stream);

// out[i] = (4 (n mod 2) - 2) * (partials of d[i], added in order in
// double-double), i = 0..count-1.
hipError_t launch_batch_finish(const FinishDesc *d, int count, const double *partials, double *out,
                               hipStream_t stream);

// Resources of the compiled batch kernel for ng groups (VGPRs, scratch).
int batch_kernel_attributes(int ng, int *vgprs, int *scratch);

}  // namespace permx
