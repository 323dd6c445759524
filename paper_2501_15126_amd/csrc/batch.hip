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

template <int NG>
__global__ void __launch_bounds__(256) batch_kernel(const BatchItem *__restrict__ items, long long nitems,
                                                    const BatchMat *__restrict__ mats,
                                                    const double *__restrict__ vals,
                                                    const int32_t *__restrict__ tops_all,
                                                    double *__restrict__ partials) {
    // the wave's index is uniform: readfirstlane lets the compiler keep the
    // item, the matrix descriptor and the column data in scalar registers
    const long long item = (long long)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (item >= nitems) return;  // the whole wave leaves together
    const BatchItem it = items[item];
    const BatchMat md = mats[it.mat];
    const int lane = threadIdx.x & 63;
    const u64 m0 = it.chunk0 + (u64)lane;
    const bool active = m0 < md.nchunks;
    const u64 m = active ? m0 : it.chunk0;  // inactive lanes replay a valid chunk and add nothing
    dd cs = batch_lane<NG>(md, vals, tops_all, m);
    if (!active) {
        cs.h = 0.0;
        cs.l = 0.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        dd o;
        o.h = __shfl_xor(cs.h, off, 64);
        o.l = __shfl_xor(cs.l, off, 64);
        cs = dd_add(cs, o);
    }
    if (lane == 0) {
        partials[2 * it.out] = cs.h;
        partials[2 * it.out + 1] = cs.l;
    }
}

__global__ void __launch_bounds__(256) batch_finish(const FinishDesc *__restrict__ d, int count,
                                                    const double *__restrict__ partials, double *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    dd acc;
    acc.h = 0.0;
    acc.l = 0.0;
    const uint64_t p0 = d[i].part;
    for (uint64_t k = 0; k < d[i].count; ++k) {
        dd v;
        v.h = partials[2 * (p0 + k)];
        v.l = partials[2 * (p0 + k) + 1];
        acc = dd_add(acc, v);
    }
    const double f = (d[i].n % 2 == 1) ? 2.0 : -2.0;  // 4 (n mod 2) - 2
    out[i] = (acc.h + acc.l) * f;
}

template <int NG>
hipError_t launch_t(const BatchItem *items, int64_t nitems, const BatchMat *mats, const double *vals,
                    const int32_t *tops, double *partials, hipStream_t stream) {
    const unsigned blocks = (unsigned)((nitems + 3) / 4);
    hipLaunchKernelGGL((batch_kernel<NG>), dim3(blocks), dim3(256), 0, stream, items, (long long)nitems, mats,
                       vals, tops, partials);
    return hipGetLastError();
}

template <int NG>
void attrs_t(int *vgprs, int *scratch) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, reinterpret_cast<const void *>(&batch_kernel<NG>)) == hipSuccess) {
        *vgprs = a.numRegs;
        *scratch = (int)a.localSizeBytes;
    }
}

#define PERM_NG_TABLE(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

}  // namespace

hipError_t launch_batch_items(int ng, const BatchItem *items, int64_t nitems, const BatchMat *mats,
                              const double *vals, const int32_t *tops, double *partials, hipStream_t stream) {
    if (nitems <= 0) return hipSuccess;
#define PERM_CASE(NGV) \
    case NGV:          \
        return launch_t<NGV>(items, nitems, mats, vals, tops, partials, stream);
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
    hipLaunchKernelGGL(batch_finish, dim3((count + 255) / 256), dim3(256), 0, stream, d, count, partials, out);
    return hipGetLastError();
}

int batch_kernel_attributes(int ng, int *vgprs, int *scratch) {
    *vgprs = -1;
    *scratch = -1;
#define PERM_CASE(NGV)                  \
    case NGV:                           \
        attrs_t<NGV>(vgprs, scratch);   \
        return 0;
    switch (ng) {
        PERM_NG_TABLE(PERM_CASE)
        default:
            return -1;
    }
#undef PERM_CASE
}

}  // namespace permx
