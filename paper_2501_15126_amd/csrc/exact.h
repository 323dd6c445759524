// exact.h -- exact permanents of integer-valued matrices.
//
// For an integer-valued matrix, y_i = 2 x_i is an integer at every Gray index
// (Alg. 1's initialisation gives x_i = a_{i,n-1} - (sum_j a_ij)/2, and every
// step adds or subtracts whole entries), so the kernels of this library run
// such a matrix on y (all values doubled, an exact scaling) and each term is
// an integer.  The integer term sum T = sum_g (-1)^g prod_i y_i equals
// (-1)^(n-1) 2^(n-1) perm(A) (Sec. II, Alg. 1 and its final factor).
//
// Besides the FP64 sum, each kernel computes, in FP64 modular arithmetic, the
// term sum modulo one prime p < 2^24 (a kernel argument) and A = sum |term|,
// which with the chunk length bounds the FP64 result's rounding error
// rigorously (exact_term_bound).  The host then takes
// the integer congruent to the residue that lies nearest the FP64 estimate;
// that integer is the permanent whenever the error bound is below half the
// modulus.  When it is not, the same kernel runs again with the next prime
// and the residues are combined by the Chinese remainder theorem.
#pragma once

#include <cstdint>

namespace permx {

// Primes below 2^24: residues and their products with a bounded sub-product
// stay exact in FP64.
constexpr int kExactMaxPasses = 3;
extern const double kExactPrimes[kExactMaxPasses];

// Largest bound on the magnitude of one exactly formed sub-product of y
// values (a product of several rows' y): a sub-product times a residue stays
// below 2^44, and 1023 such terms fit one residue accumulator (< 2^53).
constexpr double kExactPartMax = 1048576.0;  // 2^20

// What the kernels return for one permanent, over all passes so far.
struct ExactSums {
    double hi = 0.0, lo = 0.0;  // FP64 term sum (y units), double-double
    double abs_sum = 0.0;       // sum of |term| over the evaluated terms
    int chunk_log2 = 0;         // no accumulator takes more than 2^chunk_log2 terms
    int passes = 0;             // residues available (primes kExactPrimes[0 .. passes-1])
    double resid[kExactMaxPasses] = {0.0, 0.0, 0.0};  // term sum mod prime i (any representative)
};

struct ExactOutcome {
    double value = 0.0;      // the permanent: the exact integer when certified, else the estimate
    double estimate = 0.0;   // the FP64 estimate (4 (n mod 2) - 2) 2^-n (hi + lo)
    double err_bound = 0.0;  // rigorous bound on |estimate - perm|
    bool certified = false;  // value is the exact permanent
    bool more = false;       // another pass (next prime) could certify it, and exactness is required
};

// Recovers the permanent of an n x n integer-valued matrix from the sums of
// one or more passes.  Exactness is required (more = true) while the
// permanent could be below 2^53 in magnitude.
ExactOutcome exact_recover(int n, const ExactSums &s);

// Rigorous bound on |FP64 term sum - exact term sum| (y units) from A and
// the longest accumulation (exposed for tests).
double exact_term_bound(int n, int chunk_log2, double abs_sum);

}  // namespace permx
