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

// The waves of one launch: ranges[0, nranges) (sorted by wave0, each
// non-empty, ranges[0].wave0 = 0), blk_first[b] = the range holding wave 4b,
// matrices, their column data and tops, and the partials written.
struct BatchLaunchArgs {
    const BatchRange *ranges = nullptr;
    int nranges = 0;
    const int32_t *blk_first = nullptr;
    int64_t nwaves = 0;
    const BatchMat *mats = nullptr;
    const double *vals = nullptr;
    const int32_t *tops = nullptr;
    double *partials = nullptr;
};

// Launches the batch kernel instance (ng groups, zero_skip, exact) for waves
// [0, nwaves) with `block` threads (64, 128 or 256) per workgroup: one wave per
// work item, or, with a counter, `grid` workgroups of the persistent form
// taking items from *counter (which must start at 0).
hipError_t launch_batch_ranges(int ng, bool zero_skip, bool exact, const BatchLaunchArgs &a, int block,
                               unsigned long long *counter, int grid, hipStream_t stream);

// Workgroups of `block` threads of the persistent instance resident on the
// current device at once (occupancy API times compute units); -1 on error.
int batch_resident_blocks(int ng, bool zero_skip, bool exact, int block);

// c[0 .. n-1] = 0 with a kernel (graph-capturable).
hipError_t launch_counters_reset(unsigned long long *c, int n, hipStream_t stream);

// out[kPartStride i ..] = the sum of the partials of d[i] (double-double term
// sum, residue, sum of |term|), added in an order fixed by the partials'
// count, i = 0..count-1.
hipError_t launch_batch_finish(const FinishDesc *d, int count, const double *partials, double *out,
                               hipStream_t stream);

// The allocation-free entry point's device region: kNoallocScratchBytes
// bytes per device, a file-scope device array of batch.hip.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
constexpr int kNoallocMaxDevices = 64;

// *ptr = the current device's address of that region (looked up once per
// device with hipGetSymbolAddress, then kept).  Not thread-safe on the first
// call for a device: callers hold the library lock.
hipError_t batch_scratch_address(void **ptr);

// Resources of the compiled batch kernel instance (VGPRs, scratch).
int batch_kernel_attributes(int ng, bool zero_skip, bool exact, int *vgprs, int *scratch);

}  // namespace permx
