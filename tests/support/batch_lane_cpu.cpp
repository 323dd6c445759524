// Host build of the batch kernels' per-lane code (tests only): runs
// batch_lane<NG, ZS, EX>() for one chunk on the CPU with the data
// perm_batch_describe returns (exact mode: with the prime pmod).
#include "batch_types.h"
#include "batch_lane.h"

using namespace permx;
using namespace permx::batch_detail;

template <int NG>
static dd run(const BatchMat &md, const double *vals, const int32_t *tops, u64 m, double *xo) {
    if (md.exact)
        return md.zero_skip ? batch_lane<NG, true, true>(md, vals, tops, m, xo)
                            : batch_lane<NG, false, true>(md, vals, tops, m, xo);
    return md.zero_skip ? batch_lane<NG, true, false>(md, vals, tops, m, xo)
                        : batch_lane<NG, false, false>(md, vals, tops, m, xo);
}

// out[0..3] = the chunk's term sum (hi, lo), then (exact mode) its residue
// modulo pmod and its sum of |term|.
extern "C" int cpu_batch_lane(const int32_t *desc, const double *vals, size_t nvals, const int32_t *tops, u64 m,
                              double pmod, double *out) {
    BatchMat md{};
    md.n = desc[0];
    md.ng = desc[1];
    md.kappa = desc[2];
    md.zero_skip = desc[3];
    md.chunk_top = desc[4];
    md.exact = desc[6];
    md.nchunks = 1ull << (md.n - 1 - md.kappa);
    md.col_off = 0;
    md.base_off = nvals - 4 * (size_t)md.ng;
    md.top_off = 0;
    md.pmod = pmod;
    md.pinv = pmod > 0.0 ? 1.0 / pmod : 0.0;
    double xo[2] = {0.0, 0.0};
    dd r;
    switch (md.ng) {
#define C(NGV) \
    case NGV:  \
        r = run<NGV>(md, vals, tops, m, xo); \
        break;
        C(1) C(2) C(3) C(4) C(5) C(6) C(7) C(8) C(9) C(10) C(11) C(12) C(13) C(14) C(15) C(16)
#undef C
        default:
            return -1;
    }
    out[0] = r.h;
    out[1] = r.l;
    out[2] = xo[0];
    out[3] = xo[1];
    return 0;
}
