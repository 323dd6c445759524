// exact.cpp -- certificate and integer recovery for integer-valued matrices
// (see exact.h).
#include "exact.h"

#include <cmath>

namespace permx {

const double kExactPrimes[kExactMaxPasses] = {16777213.0, 16777199.0, 16777183.0};

namespace {

typedef __int128 i128;

int64_t mod_pos(int64_t a, int64_t m) {
    a %= m;
    return a < 0 ? a + m : a;
}

int64_t mulmod(int64_t a, int64_t b, int64_t m) { return (int64_t)((i128)a * b % m); }

int64_t powmod(int64_t b, int64_t e, int64_t m) {
    int64_t r = 1 % m;
    b = mod_pos(b, m);
    while (e > 0) {
        if (e & 1) r = mulmod(r, b, m);
        b = mulmod(b, b, m);
        e >>= 1;
    }
    return r;
}

// inverse modulo a prime (Fermat)
int64_t invmod(int64_t a, int64_t p) { return powmod(a, p - 2, p); }

}  // namespace

// Error of the FP64 term sum, in y units, from A = sum |computed term| and
// the chunk length:
//  * a term is a product of n exact integers formed with at most n - 1
//    rounded multiplications, so it is off by at most gamma_{n-1} |t| <=
//    gamma_{n+1} |computed t| (gamma_k = k u / (1 - k u), u = 2^-53);
//  * each accumulation (one FMA) rounds once, by at most u' = u / (1 - u)
//    times the magnitude of its result; an accumulator takes at most
//    N = 2^chunk_log2 terms, so each of its partial sums is at most its own
//    share of A (times 1 + N u' for the errors before it), and all its
//    roundings together at most N u' (1 + N u') times that share;
//  * the lane, wave, workgroup and final double-double combinations add at
//    most a few u^2 of their operands per level, far below 1e-24 A;
//  * A itself is a sum of non-negative values, computed with a relative
//    error far below 1e-6.
double exact_term_bound(int n, int chunk_log2, double abs_sum) {
    const double u = std::ldexp(1.0, -53);
    const double up = u / (1.0 - u);
    const double g = (n + 1) * u / (1.0 - (n + 1) * u);
    const double N = std::ldexp(1.0, chunk_log2);
    return abs_sum * ((g + N * up * (1.0 + N * up)) * (1.0 + 1e-6) + 1e-24);
}

ExactOutcome exact_recover(int n, const ExactSums &s) {
    ExactOutcome o;
    const double f = (n % 2 == 1) ? 2.0 : -2.0;  // 4 (n mod 2) - 2
    // perm = f 2^-n T, T the integer term sum in y units
    o.estimate = std::ldexp((s.hi + s.lo) * f, -n);
    o.err_bound = std::ldexp(exact_term_bound(n, s.chunk_log2, s.abs_sum), 1 - n);
    o.value = o.estimate;
    const long double est = std::ldexp(((long double)s.hi + (long double)s.lo) * (long double)f, -n);
    // the bound, plus the long double rounding of est and of the candidate below
    const long double E = (long double)o.err_bound + fabsl(est) * 0x1p-61L;
    if (!std::isfinite((double)est) || !std::isfinite((double)E) || !(fabsl(est) < 0x1p100L) || !(E < 0x1p100L))
        return o;
    // perm modulo M = product of the primes used: perm = (-1)^(n-1) 2^(1-n) T,
    // combined over the primes by the Chinese remainder theorem
    i128 r = 0, M = 1;
    for (int i = 0; i < s.passes; ++i) {
        const int64_t p = (int64_t)kExactPrimes[i];
        const int64_t t = mod_pos((int64_t)s.resid[i], p);
        int64_t pm = mulmod(t, invmod(powmod(2, n - 1, p), p), p);
        if (n % 2 == 0) pm = mod_pos(-pm, p);
        const int64_t k = mulmod(mod_pos(pm - (int64_t)(r % p), p), invmod((int64_t)(M % p), p), p);
        r += M * k;
        M *= p;
    }
    // the representative of r modulo M nearest the estimate
    const long double q = roundl((est - (long double)r) / (long double)M);
    const i128 c = r + (i128)q * M;
    const long double d = fabsl((long double)c - est);
    // c is the permanent when it lies within the bound and no other
    // representative does
    o.certified = d <= E && (long double)M - d > E;
    if (o.certified) {
        o.value = (double)c;
        return o;
    }
    // exactness is required while |perm| may be below 2^53; another prime
    // helps only if the enlarged modulus can exceed twice the bound
    o.more = d <= E && s.passes < kExactMaxPasses && fabsl(est) - E < 0x1p53L &&
             2 * E < (long double)M * (long double)kExactPrimes[s.passes];
    return o;
}

}  // namespace permx
