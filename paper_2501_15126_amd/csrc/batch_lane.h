// batch_lane.h -- per-lane arithmetic of the batch kernels (see batch.hip).
// Kept in a header of its own so that the same code can be compiled for the
// host in tests of its logic.
#pragma once

#include "batch_types.h"

namespace permx {
namespace batch_detail {

typedef unsigned long long u64;
typedef unsigned int u32;

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

template <int NG>
struct LaneState {
    double x[4 * NG];
    double S[NG + 1];  // S[g] = product of x over groups >= g (g >= 1); S[NG] = 1
    double acc0, acc1;
};

// x[group G] += s * c[group G], then S[G] = prod(group G) * S[G+1].
template <int NG, int G>
__device__ __forceinline__ void group_fma(LaneState<NG> &st, const double *__restrict__ c, double s) {
    if constexpr (G < NG) {
#pragma unroll
        for (int i = 0; i < 4; ++i) st.x[4 * G + i] = fma(s, c[4 * G + i], st.x[4 * G + i]);
        if constexpr (G >= 1) {
            const double p = (st.x[4 * G] * st.x[4 * G + 1]) * (st.x[4 * G + 2] * st.x[4 * G + 3]);
            if constexpr (G + 1 < NG)
                st.S[G] = p * st.S[G + 1];
            else
                st.S[G] = p;
        }
    }
}

// Groups top..G (highest first, since S[g] needs S[g+1]) as nested
// structured conditionals on the wave-uniform `top`.
template <int NG, int G>
__device__ __forceinline__ void groups_from_top(LaneState<NG> &st, const double *__restrict__ c, int top,
                                                double s) {
    if constexpr (G < NG) {
        if (top >= G) {
            groups_from_top<NG, G + 1>(st, c, top, s);
            group_fma<NG, G>(st, c, s);
        }
    }
}

template <int NG>
__device__ __forceinline__ double group0_product(const LaneState<NG> &st) {
    return (st.x[0] * st.x[1]) * (st.x[2] * st.x[3]);
}

template <int NG>
__device__ __forceinline__ double suffix1(const LaneState<NG> &st) {
    if constexpr (NG > 1)
        return st.S[1];
    else
        return 1.0;
}

// One Gray step: column (groups 0..top at c, unsigned) flipped with direction
// s (+-1 per lane), cached products refreshed, term (-1)^l added with weight w.
// The column's group 0 values (and, if G1, group 1 values) are passed in v01,
// already loaded, so that their scalar loads need not wait behind the others.
template <int NG, bool G1>
__device__ __forceinline__ void gray_step(LaneState<NG> &st, const double *__restrict__ c, const double *v01,
                                          int top, double s, double w, bool negterm, double &acc) {
    if constexpr (G1 && NG >= 2) {
        if (top >= 1) {
            groups_from_top<NG, 2>(st, c, top, s);
#pragma unroll
            for (int i = 0; i < 4; ++i) st.x[4 + i] = fma(s, v01[4 + i], st.x[4 + i]);
            const double p = (st.x[4] * st.x[5]) * (st.x[6] * st.x[7]);
            if constexpr (NG > 2)
                st.S[1] = p * st.S[2];
            else
                st.S[1] = p;
        }
    } else {
        groups_from_top<NG, 1>(st, c, top, s);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) st.x[i] = fma(s, v01[i], st.x[i]);
    const double g0 = group0_product(st) * w;
    acc = fma(negterm ? -g0 : g0, suffix1(st), acc);
}

// S[g] for a wave-uniform g in 1..NG (S[NG] = 1) without register indexing.
template <int NG>
__device__ __forceinline__ double suffix_at(const LaneState<NG> &st, int g) {
    double r = 1.0;
#pragma unroll
    for (int i = 1; i < NG; ++i) r = (g == i) ? st.S[i] : r;
    return r;
}

// The Gray-term sum of chunk m of matrix md (one lane's work): Alg. 1 over
// Gray indices [m 2^kappa, (m+1) 2^kappa).  Local step l flips column ctz(l)
// in every lane (Theorem 1); its direction is bit ctz(l)+1 of l except at
// l = 2^(kappa-1), where it is the parity of m (Lemma 2's divergent step).
// ZS: the matrix uses zero-aware skipping (md.zero_skip), a separate kernel
// instance.  Only whole chunks are skipped: a per-position interval test (as
// in the generated kernel) cost more than it saved on the serving mix, where
// the 64 lanes of a wave rarely agree on a zero.
template <int NG, bool ZS>
__device__ __forceinline__ dd batch_lane(const BatchMat &md, const double *__restrict__ vals,
                                         const int32_t *__restrict__ tops_all, const u64 m) {
    const int kappa = md.kappa;
    const int n = md.n;
    const double *__restrict__ cv = vals + md.col_off;  // [j][NG][4]
    const int32_t *__restrict__ tops = tops_all + md.top_off;
    constexpr int CS = NG * 4;  // doubles per column

    LaneState<NG> st;
    // x(Gray_{m 2^kappa}): Alg. 1's initialisation plus the columns set in the code
#pragma unroll
    for (int r = 0; r < 4 * NG; ++r) st.x[r] = vals[md.base_off + r];
    const u64 g0 = m << kappa;
    const u64 G = g0 ^ (g0 >> 1);
    for (int j = (kappa >= 1 ? kappa - 1 : 0); j < n - 1; ++j) {
        const double b = (double)((G >> j) & 1ull);
        const double *c = cv + (size_t)j * CS;
#pragma unroll
        for (int r = 0; r < 4 * NG; ++r) st.x[r] = fma(b, c[r], st.x[r]);
    }
    st.S[NG] = 1.0;
#pragma unroll
    for (int g = NG - 1; g >= 1; --g)
        st.S[g] = ((st.x[4 * g] * st.x[4 * g + 1]) * (st.x[4 * g + 2] * st.x[4 * g + 3])) * st.S[g + 1];
    st.acc0 = group0_product(st) * suffix1(st);  // term m 2^kappa (even index: +)
    st.acc1 = 0.0;

    if (kappa >= 1) {
        const double lsgn = (m & 1ull) ? -1.0 : 1.0;
        const u32 DELTA = 1u << kappa;
        const int t0 = tops[0];
        bool live = true;
        // exact zero-aware skip: rows above every group the chunk's columns
        // touch stay constant; a zero product there in all lanes zeroes every term
        if (ZS && md.chunk_top + 1 < NG) live = !__all(suffix_at(st, md.chunk_top + 1) == 0.0);
        if (live) {
            // column 0's groups 0 and 1 stay in scalar registers for the whole chunk
            constexpr int NV = NG >= 2 ? 8 : 4;
            double c0[8];
#pragma unroll
            for (int i = 0; i < NV; ++i) c0[i] = cv[i];
            for (u32 base = 0; base < DELTA; base += 2) {
                // step base + 2 flips column ctz(base + 2) >= 1; at base + 2 =
                // 2^kappa (not a step of this chunk) the weight is 0 and the
                // update is 0.  Its top and group 0 are read together, so that
                // one wait covers both loads.
                const u32 ell = base + 2;
                const bool in = ell < DELTA;
                const int jj = in ? __builtin_ctz(ell) : 0;
                const double *cj = cv + (size_t)jj * CS;
                const int tj = tops[jj];
                double vj[8];  // groups 0 (read) and 1 (not used by this step)
#pragma unroll
                for (int i = 0; i < 4; ++i) vj[i] = cj[i];
                // step base + 1: column 0, direction bit 1 of the local index
                const double s0 = (kappa == 1) ? lsgn : (((base >> 1) & 1u) ? -1.0 : 1.0);
                gray_step<NG, true>(st, cv, c0, t0, s0, 1.0, true, st.acc0);
                const double sd = in ? ((jj == kappa - 1) ? lsgn : (((ell >> (jj + 1)) & 1u) ? -1.0 : 1.0)) : 0.0;
                gray_step<NG, false>(st, cj, vj, tj, sd, in ? 1.0 : 0.0, false, st.acc1);
            }
        }
    }
    return two_sum(st.acc0, st.acc1);
}

}  // namespace batch_detail
}  // namespace permx
