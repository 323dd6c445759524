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
//  * each wave takes 64 consecutive chunks of one matrix and writes one
//    double-double partial; a second kernel adds each matrix's partials in a
//    fixed order, so a matrix's result does not depend on the rest of the batch.
#include <hip/hip_runtime.h>

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

template <int NG, bool ZS, bool EX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(batch_waves_per_eu<NG>()))) batch_kernel(const BatchRange *__restrict__ ranges, int nranges,
                                                    const int32_t *__restrict__ blk_first, long long nwaves,
                                                    const BatchMat *__restrict__ mats,
                                                    const double *__restrict__ vals,
                                                    const int32_t *__restrict__ tops_all,
                                                    double *__restrict__ partials) {
    // the wave's index is uniform: readfirstlane lets the compiler keep the
    // range, the matrix descriptor and the column data in scalar registers
    const long long w = (long long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= nwaves) return;  // the whole wave leaves together
    // blk_first holds the range of the workgroup's first wave; ranges are
    // non-empty, so the other three waves are at most three ranges further
    int r = blk_first[blockIdx.x];
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
void launch_one(unsigned blocks, const BatchRange *ranges, int nranges, const int32_t *blk_first, int64_t nwaves,
                const BatchMat *mats, const double *vals, const int32_t *tops, double *partials, hipStream_t stream) {
    hipLaunchKernelGGL((batch_kernel<NG, ZS, EX>), dim3(blocks), dim3(256), 0, stream, ranges, nranges, blk_first,
                       (long long)nwaves, mats, vals, tops, partials);
}

template <int NG>
hipError_t launch_t(bool zs, bool ex, const BatchRange *ranges, int nranges, const int32_t *blk_first,
                    int64_t nwaves, const BatchMat *mats, const double *vals, const int32_t *tops, double *partials,
                    hipStream_t stream) {
    const unsigned blocks = (unsigned)((nwaves + 3) / 4);
    if (zs && ex)
        launch_one<NG, true, true>(blocks, ranges, nranges, blk_first, nwaves, mats, vals, tops, partials, stream);
    else if (zs)
        launch_one<NG, true, false>(blocks, ranges, nranges, blk_first, nwaves, mats, vals, tops, partials, stream);
    else if (ex)
        launch_one<NG, false, true>(blocks, ranges, nranges, blk_first, nwaves, mats, vals, tops, partials, stream);
    else
        launch_one<NG, false, false>(blocks, ranges, nranges, blk_first, nwaves, mats, vals, tops, partials, stream);
    return hipGetLastError();
}

template <int NG>
void attrs_t(bool ex, int *vgprs, int *scratch) {
    hipFuncAttributes a;
    const void *f = ex ? reinterpret_cast<const void *>(&batch_kernel<NG, true, true>)
                       : reinterpret_cast<const void *>(&batch_kernel<NG, false, false>);
    if (hipFuncGetAttributes(&a, f) == hipSuccess) {
        *vgprs = a.numRegs;
        *scratch = (int)a.localSizeBytes;
    }
}

#define PERM_NG_TABLE(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

}  // namespace

hipError_t launch_batch_ranges(int ng, bool zero_skip, bool exact, const BatchRange *ranges, int nranges,
                               const int32_t *blk_first, int64_t nwaves, const BatchMat *mats, const double *vals,
                               const int32_t *tops, double *partials, hipStream_t stream) {
    if (nwaves <= 0) return hipSuccess;
    if (nranges <= 0 || (nwaves + 3) / 4 > 0x7fffffff) return hipErrorInvalidValue;
#define PERM_CASE(NGV) \
    case NGV:          \
        return launch_t<NGV>(zero_skip, exact, ranges, nranges, blk_first, nwaves, mats, vals, tops, partials, stream);
    switch (ng) {
        PERM_NG_TABLE(PERM_CASE)
        default:
            return hipErrorInvalidValue;
    }
#undef PERM_CASE
}

hipError_t launch_batch_finish(const FinishDesc *d, int count, const double *partials, double *out,
                               hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_finish, dim3(count), dim3(256), 0, stream, d, partials, out);
    return hipGetLastError();
}

int batch_kernel_attributes(int ng, bool exact, int *vgprs, int *scratch) {
    *vgprs = -1;
    *scratch = -1;
#define PERM_CASE(NGV)                       \
    case NGV:                                \
        attrs_t<NGV>(exact, vgprs, scratch); \
        return 0;
    switch (ng) {
        PERM_NG_TABLE(PERM_CASE)
        default:
            return -1;
    }
#undef PERM_CASE
}

}  // namespace permx
