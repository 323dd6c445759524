// batch.hip -- precompiled Gray-code kernels for batches of matrices.
//
// Same method and schedule as the generated single-matrix kernel (Alg. 1;
// power-of-two aligned chunks, Theorem 1 / Lemma 2), with the matrix as
// data instead of code:
//  * x has 4*NG rows (NG a template parameter; rows past n are constant 1.0)
//    held in registers with compile-time indices only;
//  * after Alg. 4 ordering, column j touches 4-row groups 0..top[j]; its
//    entries are stored as dense groups so a step adds whole groups with a
//    +-1 multiplier (a missing entry adds 0.0, which leaves x unchanged);
//  * S[g] = product of x over groups >= g is cached; a step refreshes groups
//    top[j]..1 and accumulates fma(+-G_0, S[1], acc) (the cached-product idea
//    of Sec. V with fixed 4-row groups);
//  * each wave takes 64 consecutive chunks of one matrix (a work item) and
//    writes one partial; a second kernel adds each matrix's partials in a
//    fixed order, so a matrix's result does not depend on the rest of the
//    batch, nor on which wave ran which item;
//  * launch forms: one wave per item, or persistent (a grid of resident
//    waves taking items from an atomic counter).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "batch.h"
#include "batch_lane.h"

namespace permx {

namespace {

using namespace batch_detail;

// NG = 8 compiles to 130 VGPRs (3 waves per SIMD); held to 128 it runs 4
// waves per SIMD at the cost of a few spilled values, measured 6 % faster on
// the batch workload.  The other instances keep the compiler's choice.
template <int NG>
constexpr int batch_waves_per_eu() {
    return NG == 8 ? 4 : 1;
}

// The work of wave w of a launch (wave-uniform w): the 64 chunks of item
// item0 + (w - wave0) of its range's matrix, one per lane, and the wave's
// partial (double-double term sum, then in exact mode the residue and the
// sum of |term|) at partials[kPartStride (out0 + w - wave0) ..].
template <int NG, bool ZS, bool EX>
__device__ __forceinline__ void wave_item(long long w, const BatchRange *__restrict__ ranges, int nranges,
                                          const int32_t *__restrict__ blk_first, const BatchMat *__restrict__ mats,
                                          const double *__restrict__ vals, const int32_t *__restrict__ tops_all,
                                          double *__restrict__ partials) {
    // blk_first[b] holds the range of wave 4b; ranges are non-empty, so wave w
    // is at most three ranges further
    int r = blk_first[w >> 2];
    while (r + 1 < nranges && (long long)ranges[r + 1].wave0 <= w) ++r;
    const BatchRange rg = ranges[r];
    const u64 k = (u64)(w - (long long)rg.wave0);
    const BatchMat md = mats[rg.mat];
    const int lane = threadIdx.x & 63;
    const u64 chunk0 = (rg.item0 + k) * 64;
    const u64 m0 = chunk0 + (u64)lane;
    const bool active = m0 < md.nchunks;
    const u64 m = active ? m0 : chunk0;  // inactive lanes replay a valid chunk and add nothing
    double xo[2] = {0.0, 0.0};
    dd cs = batch_lane<NG, ZS, EX>(md, vals, tops_all, m, xo);
    if (!active) {
        cs.h = 0.0;
        cs.l = 0.0;
        xo[0] = 0.0;
        xo[1] = 0.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        dd o;
        o.h = __shfl_xor(cs.h, off, 64);
        o.l = __shfl_xor(cs.l, off, 64);
        cs = dd_add(cs, o);
        if constexpr (EX) {
            // residues: exact integer sums (64 lanes: below 2^30)
            xo[0] += __shfl_xor(xo[0], off, 64);
            xo[1] += __shfl_xor(xo[1], off, 64);
        }
    }
    if (lane == 0) {
        const u64 out = rg.out0 + k;
        partials[kPartStride * out] = cs.h;
        partials[kPartStride * out + 1] = cs.l;
        partials[kPartStride * out + 2] = EX ? reduce_mod(xo[0], md.pmod, md.pinv) : 0.0;
        partials[kPartStride * out + 3] = xo[1];
    }
}

// One wave per work item: wave w = blockIdx.x * (waves per block) + its index
// in the block.
template <int NG, bool ZS, bool EX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(batch_waves_per_eu<NG>()))) batch_kernel(const BatchRange *__restrict__ ranges, int nranges,
                                                    const int32_t *__restrict__ blk_first, long long nwaves,
                                                    const BatchMat *__restrict__ mats,
                                                    const double *__restrict__ vals,
                                                    const int32_t *__restrict__ tops_all,
                                                    double *__restrict__ partials) {
    // the wave's index is uniform: readfirstlane lets the compiler keep the
    // range, the matrix descriptor and the column data in scalar registers
    const long long w = (long long)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= nwaves) return;  // the whole wave leaves together
    wave_item<NG, ZS, EX>(w, ranges, nranges, blk_first, mats, vals, tops_all, partials);
}

// Persistent form: a grid of at most the resident waves; each wave takes the
// next work item from a counter (one atomic add per item) until none is
// left, so every wave reaches the exit.  Results do not depend on which
// wave ran an item (each item writes its own partial).
template <int NG, bool ZS, bool EX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(batch_waves_per_eu<NG>()))) batch_persistent(const BatchRange *__restrict__ ranges, int nranges,
                                                    const int32_t *__restrict__ blk_first, long long nwaves,
                                                    const BatchMat *__restrict__ mats,
                                                    const double *__restrict__ vals,
                                                    const int32_t *__restrict__ tops_all,
                                                    double *__restrict__ partials,
                                                    unsigned long long *__restrict__ counter) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned long long got = 0;
        if (lane == 0) got = atomicAdd(counter, 1ull);
        // the item index is the same in every lane: both halves to scalars
        const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)got);
        const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(got >> 32));
        const long long w = (long long)(((unsigned long long)hi << 32) | lo);
        if (w >= nwaves) break;
        wave_item<NG, ZS, EX>(w, ranges, nranges, blk_first, mats, vals, tops_all, partials);
    }
}

// Clears the persistent kernels' item counters (a kernel, not a memset, so
// that it can sit in a captured graph).
__global__ void batch_counters_reset(unsigned long long *__restrict__ c, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0ull;
}

// One workgroup per matrix: thread t adds partials t, t + 256, ... and a
// fixed binary tree in LDS combines the 256 sums, so the order depends only
// on the number of partials.  Residues (each below 2^23 + 2, at most 2^22 of
// them) add exactly.
__global__ void __launch_bounds__(256) batch_finish(const FinishDesc *__restrict__ d,
                                                    const double *__restrict__ partials, double *__restrict__ out) {
    __shared__ double sh[4 * 256];
    const FinishDesc fd = d[blockIdx.x];
    const int t = threadIdx.x;
    dd acc;
    acc.h = 0.0;
    acc.l = 0.0;
    double r = 0.0, a = 0.0;
    for (u64 k = t; k < fd.count; k += 256) {
        const double *q = partials + kPartStride * (fd.part + k);
        dd v;
        v.h = q[0];
        v.l = q[1];
        acc = dd_add(acc, v);
        r += q[2];
        a += q[3];
    }
    sh[4 * t] = acc.h;
    sh[4 * t + 1] = acc.l;
    sh[4 * t + 2] = r;
    sh[4 * t + 3] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            dd x, y;
            x.h = sh[4 * t];
            x.l = sh[4 * t + 1];
            y.h = sh[4 * (t + s)];
            y.l = sh[4 * (t + s) + 1];
            x = dd_add(x, y);
            sh[4 * t] = x.h;
            sh[4 * t + 1] = x.l;
            sh[4 * t + 2] += sh[4 * (t + s) + 2];
            sh[4 * t + 3] += sh[4 * (t + s) + 3];
        }
        __syncthreads();
    }
    if (t == 0) {
        double *o = out + kPartStride * (u64)blockIdx.x;
        o[0] = sh[0];
        o[1] = sh[1];
        o[2] = fd.exact ? reduce_mod(sh[2], fd.pmod, fd.pinv) : 0.0;
        o[3] = sh[3];
    }
}

template <int NG, bool ZS, bool EX>
hipError_t launch_one(const BatchLaunchArgs &a, int block, unsigned long long *counter, int grid,
                      hipStream_t stream) {
    if (counter) {
        hipLaunchKernelGGL((batch_persistent<NG, ZS, EX>), dim3((unsigned)grid), dim3((unsigned)block), 0, stream,
                           a.ranges, a.nranges, a.blk_first, (long long)a.nwaves, a.mats, a.vals, a.tops, a.partials,
                           counter);
    } else {
        const int wpb = block / 64;
        const unsigned blocks = (unsigned)((a.nwaves + wpb - 1) / wpb);
        hipLaunchKernelGGL((batch_kernel<NG, ZS, EX>), dim3(blocks), dim3((unsigned)block), 0, stream, a.ranges,
                           a.nranges, a.blk_first, (long long)a.nwaves, a.mats, a.vals, a.tops, a.partials);
    }
    return hipGetLastError();
}

template <int NG>
hipError_t launch_t(bool zs, bool ex, const BatchLaunchArgs &a, int block, unsigned long long *counter, int grid,
                    hipStream_t stream) {
    if (zs && ex) return launch_one<NG, true, true>(a, block, counter, grid, stream);
    if (zs) return launch_one<NG, true, false>(a, block, counter, grid, stream);
    if (ex) return launch_one<NG, false, true>(a, block, counter, grid, stream);
    return launch_one<NG, false, false>(a, block, counter, grid, stream);
}

template <int NG>
const void *kernel_of(bool zs, bool ex, bool persistent) {
    if (persistent) {
        if (zs && ex) return reinterpret_cast<const void *>(&batch_persistent<NG, true, true>);
        if (zs) return reinterpret_cast<const void *>(&batch_persistent<NG, true, false>);
        if (ex) return reinterpret_cast<const void *>(&batch_persistent<NG, false, true>);
        return reinterpret_cast<const void *>(&batch_persistent<NG, false, false>);
    }
    if (zs && ex) return reinterpret_cast<const void *>(&batch_kernel<NG, true, true>);
    if (zs) return reinterpret_cast<const void *>(&batch_kernel<NG, true, false>);
    if (ex) return reinterpret_cast<const void *>(&batch_kernel<NG, false, true>);
    return reinterpret_cast<const void *>(&batch_kernel<NG, false, false>);
}

template <int NG>
void attrs_t(bool zs, bool ex, int *vgprs, int *scratch) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, kernel_of<NG>(zs, ex, false)) == hipSuccess) {
        *vgprs = a.numRegs;
        *scratch = (int)a.localSizeBytes;
    }
}

#define PERM_NG_TABLE(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

}  // namespace

hipError_t launch_batch_ranges(int ng, bool zero_skip, bool exact, const BatchLaunchArgs &a, int block,
                               unsigned long long *counter, int grid, hipStream_t stream) {
    if (a.nwaves <= 0) return hipSuccess;
    if (a.nranges <= 0 || a.nwaves > 0x7fffffffLL || (block != 64 && block != 128 && block != 256) ||
        (counter && grid <= 0))
        return hipErrorInvalidValue;
#define PERM_CASE(NGV) \
    case NGV:          \
        return launch_t<NGV>(zero_skip, exact, a, block, counter, grid, stream);
    switch (ng) {
        PERM_NG_TABLE(PERM_CASE)
        default:
            return hipErrorInvalidValue;
    }
#undef PERM_CASE
}

int batch_resident_blocks(int ng, bool zero_skip, bool exact, int block) {
    const void *f = nullptr;
#define PERM_CASE(NGV)                                     \
    case NGV:                                              \
        f = kernel_of<NGV>(zero_skip, exact, true);        \
        break;
    switch (ng) {
        PERM_NG_TABLE(PERM_CASE)
        default:
            return -1;
    }
#undef PERM_CASE
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, block, 0) != hipSuccess) return -1;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    return std::max(1, per_cu) * cus;
}

hipError_t launch_counters_reset(unsigned long long *c, int n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_counters_reset, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, c, n);
    return hipGetLastError();
}

hipError_t launch_batch_finish(const FinishDesc *d, int count, const double *partials, double *out,
                               hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_finish, dim3(count), dim3(256), 0, stream, d, partials, out);
    return hipGetLastError();
}

// Device memory of the allocation-free batch entry point: the staged
// matrices, the wave partials and the per-matrix sums live here instead of
// in buffers the library allocates.  Each device the library runs on holds
// its own copy, at its own address, until the process ends.  Host code never
// names the array itself (its host-side symbol is not a device address); it
// uses the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

hipError_t batch_scratch_address(void **ptr) {
    static void *addr[kNoallocMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoallocMaxDevices) return hipErrorInvalidDevice;
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

int batch_kernel_attributes(int ng, bool zero_skip, bool exact, int *vgprs, int *scratch) {
    *vgprs = -1;
    *scratch = -1;
#define PERM_CASE(NGV)                                  \
    case NGV:                                           \
        attrs_t<NGV>(zero_skip, exact, vgprs, scratch); \
        return 0;
    switch (ng) {
        PERM_NG_TABLE(PERM_CASE)
        default:
            return -1;
    }
#undef PERM_CASE
}

}  // namespace permx
