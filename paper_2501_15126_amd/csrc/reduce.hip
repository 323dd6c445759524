// reduce.hip -- fixed-order double-double sum of per-workgroup partials.
//
// The paper adds per-thread partial permanents into a global variable
// (Sec. II-A) in no stated order.  Here every workgroup of the Gray kernel
// writes one double-double partial, and this single-workgroup kernel sums
// them in an order fixed by the partial's index (and adds the workgroups'
// evaluated-term counts): thread t accumulates
// partials t, t + 1024, t + 2048, ... and the 1024 results are combined by a
// fixed binary tree in LDS.  The result does not depend on scheduling.
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

constexpr int kThreads = 1024;

__global__ void __launch_bounds__(kThreads) final_reduce(const double *__restrict__ partials,
                                                          const unsigned long long *__restrict__ counts,
                                                          long long count, double *__restrict__ out,
                                                          unsigned long long *__restrict__ count_out) {
    __shared__ double sh[2 * kThreads];
    __shared__ unsigned long long shc[kThreads];
    const int t = threadIdx.x;
    dd acc;
    acc.h = 0.0;
    acc.l = 0.0;
    unsigned long long c = 0;
    // the same order of additions as a plain strided loop, with the loads of
    // eight partials issued before the first of their additions waits
    constexpr int kBatch = 8;
    long long b = t;
    for (; b + (kBatch - 1) * (long long)kThreads < count; b += kBatch * (long long)kThreads) {
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
    }
    for (; b < count; b += kThreads) {
        dd v;
        v.h = partials[2 * b];
        v.l = partials[2 * b + 1];
        acc = dd_add(acc, v);
        c += counts[b];
    }
    sh[2 * t] = acc.h;
    sh[2 * t + 1] = acc.l;
    shc[t] = c;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            dd a, b;
            a.h = sh[2 * t];
            a.l = sh[2 * t + 1];
            b.h = sh[2 * (t + s)];
            b.l = sh[2 * (t + s) + 1];
            a = dd_add(a, b);
            sh[2 * t] = a.h;
            sh[2 * t + 1] = a.l;
            shc[t] += shc[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = sh[0];
        out[1] = sh[1];
        count_out[0] = shc[0];
    }
}

// Exact mode: per-workgroup (residue, sum |term|) pairs summed column by
// column in the same fixed order.  Residues are integers below 2^23 + 2 in
// magnitude, so their sum over at most 2^23 workgroups is exact.
__global__ void __launch_bounds__(kThreads) final_reduce_x(const double *__restrict__ xparts, long long count,
                                                            double *__restrict__ out) {
    __shared__ double sh[2 * kThreads];
    const int t = threadIdx.x;
    double r = 0.0, a = 0.0;
    for (long long b = t; b < count; b += kThreads) {
        r += xparts[2 * b];
        a += xparts[2 * b + 1];
    }
    sh[2 * t] = r;
    sh[2 * t + 1] = a;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            sh[2 * t] += sh[2 * (t + s)];
            sh[2 * t + 1] += sh[2 * (t + s) + 1];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = sh[0];
        out[1] = sh[1];
    }
}

}  // namespace

namespace permx {

hipError_t launch_final_reduce_x(const double *xparts, long long count, double *out, hipStream_t stream) {
    hipLaunchKernelGGL(final_reduce_x, dim3(1), dim3(kThreads), 0, stream, xparts, count, out);
    return hipGetLastError();
}

hipError_t launch_final_reduce(const double *partials, const unsigned long long *counts, long long count,
                               double *out, unsigned long long *count_out, hipStream_t stream) {
    hipLaunchKernelGGL(final_reduce, dim3(1), dim3(kThreads), 0, stream, partials, counts, count, out, count_out);
    return hipGetLastError();
}

}  // namespace permx
