// reduce.hip -- fixed-order double-double sum of per-workgroup partials.
//
// The paper adds per-thread partial permanents into a global variable
// (Sec. II-A) in no stated order.  Here every workgroup of the Gray kernel
// writes one double-double partial (and its evaluated-term count, and in the
// exact mode its residue and |term| sums), and two kernels sum them in an
// order fixed by the partials' count: contiguous slices, each summed by one
// workgroup in a fixed order, then the slices' sums by one workgroup.  The
// result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "reduce.h"

namespace {

struct dd {
    double h, l;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    dd r;
    r.h = s;
    r.l = (a - (s - bb)) + (b - bb);
    return r;
}

__device__ __forceinline__ dd dd_add(dd x, dd y) {
    const dd s = two_sum(x.h, y.h);
    const double e = s.l + (x.l + y.l);
    dd r;
    r.h = s.h + e;
    r.l = e - (r.h - s.h);
    return r;
}

constexpr int kThreads = 256;      // threads per workgroup of both stages
constexpr long long kSlice = 2048;  // partials per first-stage workgroup (at most)
constexpr int kMaxSlices = 1024;    // first-stage workgroups (more partials make the slices longer)

// Stage 1: workgroup s sums partials [s L, (s+1) L) (L from the count):
// thread t takes partials s L + t, s L + t + 256, ... in order, with the
// loads of four issued before their additions, and a fixed binary tree in
// LDS combines the 256 sums.  Its results (double-double sum, evaluated-term
// count, exact mode's residue and |term| sums) go to stage[6 s ..].
__global__ void __launch_bounds__(kThreads) reduce_stage1(const double *__restrict__ partials,
                                                          const unsigned long long *__restrict__ counts,
                                                          const double *__restrict__ xparts, long long count,
                                                          long long slice, double *__restrict__ stage) {
    __shared__ double sh[4 * kThreads];
    __shared__ unsigned long long shc[kThreads];
    const int t = threadIdx.x;
    const long long b0 = (long long)blockIdx.x * slice;
    const long long b1 = b0 + slice < count ? b0 + slice : count;
    dd acc;
    acc.h = 0.0;
    acc.l = 0.0;
    unsigned long long c = 0;
    double r = 0.0, a = 0.0;
    constexpr int kBatch = 4;
    long long b = b0 + t;
    for (; b + (kBatch - 1) * (long long)kThreads < b1; b += kBatch * (long long)kThreads) {
        dd v[kBatch];
        unsigned long long cc[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const long long q = b + (long long)i * kThreads;
            v[i].h = partials[2 * q];
            v[i].l = partials[2 * q + 1];
            cc[i] = counts[q];
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            acc = dd_add(acc, v[i]);
            c += cc[i];
        }
        if (xparts) {
#pragma unroll
            for (int i = 0; i < kBatch; ++i) {
                const long long q = b + (long long)i * kThreads;
                r += xparts[2 * q];
                a += xparts[2 * q + 1];
            }
        }
    }
    for (; b < b1; b += kThreads) {
        dd v;
        v.h = partials[2 * b];
        v.l = partials[2 * b + 1];
        acc = dd_add(acc, v);
        c += counts[b];
        if (xparts) {
            r += xparts[2 * b];
            a += xparts[2 * b + 1];
        }
    }
    sh[4 * t] = acc.h;
    sh[4 * t + 1] = acc.l;
    sh[4 * t + 2] = r;
    sh[4 * t + 3] = a;
    shc[t] = c;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
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
            shc[t] += shc[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        double *o = stage + 6 * (long long)blockIdx.x;
        o[0] = sh[0];
        o[1] = sh[1];
        unsigned long long *oc = reinterpret_cast<unsigned long long *>(o + 2);
        oc[0] = shc[0];
        o[3] = sh[2];
        o[4] = sh[3];
    }
}

// Stage 2: one workgroup adds the nslices stage-1 results in index order
// (thread t takes t, t + 256, ...; then the same fixed tree): out[0..1]
// double-double sum, out[2] the evaluated-term count (its bits), out[3..4]
// the residue and |term| sums.
__global__ void __launch_bounds__(kThreads) reduce_stage2(const double *__restrict__ stage, int nslices,
                                                          double *__restrict__ out) {
    __shared__ double sh[4 * kThreads];
    __shared__ unsigned long long shc[kThreads];
    const int t = threadIdx.x;
    dd acc;
    acc.h = 0.0;
    acc.l = 0.0;
    unsigned long long c = 0;
    double r = 0.0, a = 0.0;
    for (int s = t; s < nslices; s += kThreads) {
        const double *q = stage + 6 * (long long)s;
        dd v;
        v.h = q[0];
        v.l = q[1];
        acc = dd_add(acc, v);
        c += reinterpret_cast<const unsigned long long *>(q + 2)[0];
        r += q[3];
        a += q[4];
    }
    sh[4 * t] = acc.h;
    sh[4 * t + 1] = acc.l;
    sh[4 * t + 2] = r;
    sh[4 * t + 3] = a;
    shc[t] = c;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
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
            shc[t] += shc[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = sh[0];
        out[1] = sh[1];
        reinterpret_cast<unsigned long long *>(out + 2)[0] = shc[0];
        out[3] = sh[2];
        out[4] = sh[3];
    }
}

}  // namespace

namespace permx {

long long final_reduce_slices(long long count) {
    if (count <= 0) return 1;
    long long ns = (count + kSlice - 1) / kSlice;
    return ns < kMaxSlices ? ns : kMaxSlices;
}

hipError_t launch_final_reduce(const double *partials, const unsigned long long *counts, const double *xparts,
                               long long count, double *stage, double *out, hipStream_t stream) {
    const long long ns = final_reduce_slices(count);
    const long long slice = count > 0 ? (count + ns - 1) / ns : 1;
    hipLaunchKernelGGL(reduce_stage1, dim3((unsigned)ns), dim3(kThreads), 0, stream, partials, counts, xparts, count,
                       slice, stage);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_stage2, dim3(1), dim3(kThreads), 0, stream, stage, (int)ns, out);
    return hipGetLastError();
}

}  // namespace permx
