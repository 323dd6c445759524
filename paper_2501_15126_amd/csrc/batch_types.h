// batch_types.h -- plain data shared by the batch kernels and their host code.
#pragma once

#include <cstdint>

namespace permx {

// Descriptor of one matrix of a batch (device-resident).
struct BatchMat {
    int32_t n, ng, kappa;           // size, 4-row groups of x, chunk log2
    int32_t zero_skip, chunk_top;   // zero-aware skipping on; highest group any in-chunk column touches
    int32_t exact;                  // exact mode: values are 2a (x holds y = 2x), residues modulo pmod
    uint64_t nchunks;               // 2^(n-1-kappa)
    uint64_t col_off;               // doubles: column groups [j][g][4]
    uint64_t base_off;              // doubles: x at Gray index 0, 4*ng values (padding rows 1.0)
    uint64_t top_off;               // int32: top group of each flipped column
    double pmod, pinv;              // exact mode: the prime of this pass and its reciprocal
};

// Consecutive waves of one launch that work on one matrix: wave w of the
// launch, wave0 <= w < the next range's wave0, takes the 64 chunks of item
// item0 + (w - wave0) (chunks 64 item .. 64 item + 63) and writes its
// partial to partials[kPartStride (out0 + w - wave0) ..]: the double-double
// term sum, then (exact mode) the residue and the sum of |term|.
struct BatchRange {
    int32_t mat;
    int32_t pad;
    uint64_t wave0;
    uint64_t item0;
    uint64_t out0;
};

// A matrix's final sum: partials part .. part+count-1 added in an order fixed
// by their index, written as kPartStride doubles (double-double term sum,
// residue, sum of |term|; the host applies the final factor 4 (n mod 2) - 2).
struct FinishDesc {
    uint64_t part;
    uint64_t count;
    int32_t n;
    int32_t exact;
    double pmod, pinv;
};

constexpr int kPartStride = 4;  // doubles per wave partial and per finished matrix

constexpr int kBatchMaxNG = 16;  // x of up to 64 rows
// A batch launch covers whole matrices: n <= 44 keeps one at 2^43 Gray steps
// (about 13 s of the device), with at most 2^22 waves; larger n goes through
// the single-matrix path, whose launches are sliced.
constexpr int kBatchMaxN = 44;
constexpr int kBatchStreams = 4;  // kernel instances ng run on stream ng % kBatchStreams

}  // namespace permx
