// Host build of the batch kernels' per-lane code (tests only): runs
// batch_lane<NG>() for one chunk on the CPU with the data perm_batch_describe
// returns.
#include "batch_types.h"
#include "batch_lane.h"

using namespace permx;
using namespace permx::batch_detail;

template <int NG>
static dd run(const BatchMat &md, const double *vals, const int32_t *tops, u64 m) {
    return md.zero_skip ? batch_lane<NG, true>(md, vals, tops, m) : batch_lane<NG, false>(md, vals, tops, m);
}

extern "C" int cpu_batch_lane(const int32_t *desc, const double *vals, size_t nvals, const int32_t *tops, u64 m,
                              double *out) {
    BatchMat md{};
    md.n = desc[0];
    md.ng = desc[1];
    md.kappa = desc[2];
    md.zero_skip = desc[3];
    md.chunk_top = desc[4];
    md.nchunks = 1ull << (md.n - 1 - md.kappa);
    md.col_off = 0;
    md.base_off = nvals - 4 * (size_t)md.ng;
    md.top_off = 0;
    dd r;
    switch (md.ng) {
#define C(NGV) \
    case NGV:  \
        r = run<NGV>(md, vals, tops, m); \
        break;
        C(1) C(2) C(3) C(4) C(5) C(6) C(7) C(8) C(9) C(10) C(11) C(12) C(13) C(14) C(15) C(16)
#undef C
        default:
            return -1;
    }
    out[0] = r.h;
    out[1] = r.l;
    return 0;
}
