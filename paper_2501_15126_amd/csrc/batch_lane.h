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

// q r reduced modulo the prime p (pinv = 1/p): with |q| <= 2^20 and |r| <
// 2^23 + 2 the product is exact and rint(t / p) is within one of its
// quotient, so the remainder is exact and lies in (-p/2 - 2, p/2 + 2).  The
// same reduction brings any exact integer below 2^53 into that range.
__device__ __forceinline__ double reduce_mod(double t, double pmod, double pinv) {
    return fma(-rint(t * pinv), pmod, t);
}

// EX: exact mode (integer-valued matrix on y = 2x): R[g] holds S[g] modulo
// the prime, racc the term sum modulo the prime (reduced at least every 1023
// terms), accA the sum of |term| of the error bound.
template <int NG, bool EX>
struct LaneState {
    double x[4 * NG];
    double S[NG + 1];  // S[g] = product of x over groups >= g (g >= 1); S[NG] = 1
    double R[EX ? NG + 1 : 1];
    double acc0, acc1;
    double racc, accA;
    double pmod, pinv;
};

// x[group G] += s * c[group G], then S[G] = prod(group G) * S[G+1] (and R[G]).
template <int NG, bool EX, int G>
__device__ __forceinline__ void group_fma(LaneState<NG, EX> &st, const double *__restrict__ c, double s) {
    if constexpr (G < NG) {
#pragma unroll
        for (int i = 0; i < 4; ++i) st.x[4 * G + i] = fma(s, c[4 * G + i], st.x[4 * G + i]);
        if constexpr (G >= 1) {
            const double p = (st.x[4 * G] * st.x[4 * G + 1]) * (st.x[4 * G + 2] * st.x[4 * G + 3]);
            if constexpr (G + 1 < NG) {
                st.S[G] = p * st.S[G + 1];
                if constexpr (EX) st.R[G] = reduce_mod(p * st.R[G + 1], st.pmod, st.pinv);
            } else {
                st.S[G] = p;
                if constexpr (EX) st.R[G] = p;
            }
        }
    }
}

// Groups top..G (highest first, since S[g] needs S[g+1]) as nested
// structured conditionals on the wave-uniform `top`.
template <int NG, bool EX, int G>
__device__ __forceinline__ void groups_from_top(LaneState<NG, EX> &st, const double *__restrict__ c, int top,
                                                double s) {
    if constexpr (G < NG) {
        if (top >= G) {
            groups_from_top<NG, EX, G + 1>(st, c, top, s);
            group_fma<NG, EX, G>(st, c, s);
        }
    }
}

template <int NG, bool EX>
__device__ __forceinline__ double group0_product(const LaneState<NG, EX> &st) {
    return (st.x[0] * st.x[1]) * (st.x[2] * st.x[3]);
}

template <int NG, bool EX>
__device__ __forceinline__ double suffix1(const LaneState<NG, EX> &st) {
    if constexpr (NG > 1)
        return st.S[1];
    else
        return 1.0;
}

template <int NG, bool EX>
__device__ __forceinline__ double rsuffix1(const LaneState<NG, EX> &st) {
    if constexpr (NG > 1 && EX)
        return st.R[1];
    else
        return 1.0;
}

// acc += (+-) g0 S[1]; in exact mode also the residue and |term|.
template <int NG, bool EX>
__device__ __forceinline__ void add_term(LaneState<NG, EX> &st, double g0, bool negterm, double &acc) {
    const double sg0 = negterm ? -g0 : g0;
    acc = fma(sg0, suffix1(st), acc);
    if constexpr (EX) {
        st.racc = fma(sg0, rsuffix1(st), st.racc);
        st.accA = fma(fabs(g0), fabs(suffix1(st)), st.accA);
    }
}

// One Gray step: column (groups 0..top at c, unsigned) flipped with direction
// s (+-1 per lane), cached products refreshed, term (-1)^l added with weight w.
// The column's group 0 values (and, if G1, group 1 values) are passed in v01,
// already loaded, so that their scalar loads need not wait behind the others.
template <int NG, bool EX, bool G1>
__device__ __forceinline__ void gray_step(LaneState<NG, EX> &st, const double *__restrict__ c, const double *v01,
                                          int top, double s, double w, bool negterm, double &acc) {
    if constexpr (G1 && NG >= 2) {
        if (top >= 1) {
            groups_from_top<NG, EX, 2>(st, c, top, s);
#pragma unroll
            for (int i = 0; i < 4; ++i) st.x[4 + i] = fma(s, v01[4 + i], st.x[4 + i]);
            const double p = (st.x[4] * st.x[5]) * (st.x[6] * st.x[7]);
            if constexpr (NG > 2) {
                st.S[1] = p * st.S[2];
                if constexpr (EX) st.R[1] = reduce_mod(p * st.R[2], st.pmod, st.pinv);
            } else {
                st.S[1] = p;
                if constexpr (EX) st.R[1] = p;
            }
        }
    } else {
        groups_from_top<NG, EX, 1>(st, c, top, s);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) st.x[i] = fma(s, v01[i], st.x[i]);
    add_term(st, group0_product(st) * w, negterm, acc);
}

// S[g] for a wave-uniform g in 1..NG (S[NG] = 1) without register indexing.
template <int NG, bool EX>
__device__ __forceinline__ double suffix_at(const LaneState<NG, EX> &st, int g) {
    double r = 1.0;
#pragma unroll
    for (int i = 1; i < NG; ++i) r = (g == i) ? st.S[i] : r;
    return r;
}

// The steps base + 1 .. base + 2 of the chunk loop for base in [b0, b1).
template <int NG, bool EX>
__device__ __forceinline__ void chunk_steps(LaneState<NG, EX> &st, const double *__restrict__ cv,
                                            const int32_t *__restrict__ tops, const double *c0, int t0, int kappa,
                                            double lsgn, u32 b0, u32 b1) {
    constexpr int CS = NG * 4;  // doubles per column
    const u32 DELTA = 1u << kappa;
    for (u32 base = b0; base < b1; base += 2) {
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
        gray_step<NG, EX, true>(st, cv, c0, t0, s0, 1.0, true, st.acc0);
        const double sd = in ? ((jj == kappa - 1) ? lsgn : (((ell >> (jj + 1)) & 1u) ? -1.0 : 1.0)) : 0.0;
        gray_step<NG, EX, false>(st, cj, vj, tj, sd, in ? 1.0 : 0.0, false, st.acc1);
    }
}

// The Gray-term sum of chunk m of matrix md (one lane's work): Alg. 1 over
// Gray indices [m 2^kappa, (m+1) 2^kappa).  Local step l flips column ctz(l)
// in every lane (Theorem 1); its direction is bit ctz(l)+1 of l except at
// l = 2^(kappa-1), where it is the parity of m (Lemma 2's divergent step).
// ZS: the matrix uses zero-aware skipping (md.zero_skip), a separate kernel
// instance.  Only whole chunks are skipped: a per-position interval test (as
// in the generated kernel) cost more than it saved on the serving mix, where
// the 64 lanes of a wave rarely agree on a zero.
// EX: exact mode; xo receives the lane's residue (in (-p/2 - 2, p/2 + 2)) and
// its sum of |term|.
template <int NG, bool ZS, bool EX>
__device__ __forceinline__ dd batch_lane(const BatchMat &md, const double *__restrict__ vals,
                                         const int32_t *__restrict__ tops_all, const u64 m, double *xo) {
    const int kappa = md.kappa;
    const int n = md.n;
    const double *__restrict__ cv = vals + md.col_off;  // [j][NG][4]
    const int32_t *__restrict__ tops = tops_all + md.top_off;
    constexpr int CS = NG * 4;  // doubles per column

    LaneState<NG, EX> st;
    if constexpr (EX) {
        st.pmod = md.pmod;
        st.pinv = md.pinv;
    }
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
    if constexpr (EX) st.R[NG] = 1.0;
#pragma unroll
    for (int g = NG - 1; g >= 1; --g) {
        const double p = (st.x[4 * g] * st.x[4 * g + 1]) * (st.x[4 * g + 2] * st.x[4 * g + 3]);
        st.S[g] = p * st.S[g + 1];
        if constexpr (EX) st.R[g] = (g == NG - 1) ? p : reduce_mod(p * st.R[g + 1], st.pmod, st.pinv);
    }
    // term m 2^kappa (even index: +)
    st.acc0 = 0.0;
    st.acc1 = 0.0;
    st.racc = 0.0;
    st.accA = 0.0;
    add_term(st, group0_product(st), false, st.acc0);

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
            if constexpr (EX) {
                // 512 steps (at most 2^43 each) between reductions of racc
                for (u32 b0 = 0; b0 < DELTA; b0 += 512u) {
                    chunk_steps(st, cv, tops, c0, t0, kappa, lsgn, b0, DELTA - b0 > 512u ? b0 + 512u : DELTA);
                    st.racc = reduce_mod(st.racc, st.pmod, st.pinv);
                }
            } else {
                chunk_steps(st, cv, tops, c0, t0, kappa, lsgn, 0u, DELTA);
            }
        }
    }
    if constexpr (EX) {
        xo[0] = reduce_mod(st.racc, st.pmod, st.pinv);
        xo[1] = st.accA;
    } else {
        (void)xo;
    }
    return two_sum(st.acc0, st.acc1);
}

}  // namespace batch_detail
}  // namespace permx
