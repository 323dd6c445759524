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

// Launches the batch kernel for waves [0, nwaves) described by ranges[0,
// nranges) (sorted by wave0, each non-empty, ranges[0].wave0 = 0) whose
// matrices all have ng groups and the same zero_skip and exact flags;
// blk_first[b] is the range holding wave 4b.
hipError_t launch_batch_ranges(int ng, bool zero_skip, bool exact, const BatchRange *ranges, int nranges,
                               const int32_t *blk_first, int64_t nwaves, const BatchMat *mats, const double *vals,
                               const int32_t *tops, double *partials, hipStream_t stream);

// out[kPartStride i ..] = the sum of the partials of d[i] (double-double term
// sum, residue, sum of |term|), added in an order fixed by the partials'
// count, i = 0..count-1.
hipError_t launch_batch_finish(const FinishDesc *d, int count, const double *partials, double *out,
                               hipStream_t stream);

// Resources of the compiled batch kernel for ng groups (VGPRs, scratch); the
// exact-mode zero-skip instance when exact, else the plain one.
int batch_kernel_attributes(int ng, bool exact, int *vgprs, int *scratch);

}  // namespace permx
