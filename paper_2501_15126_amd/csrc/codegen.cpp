// codegen.cpp -- emits the matrix-specific gfx950 kernel (HIP C++ for hipRTC).
//
// What the generated kernel computes: the Gray-term sum of Alg. 1 over the
// chunks [chunk_begin, chunk_end), chunk m covering Gray indices
// [m 2^kappa, (m+1) 2^kappa), one chunk per lane.  For each workgroup it
// writes the double-double sum of its lanes' chunks to partials[2b], [2b+1].
//
// How (the paper's ideas, rebuilt for a 64-wide wavefront):
//  * x lives in named variables, one per row, so the compiler keeps it in
//    VGPRs; the matrix values are exact hex-float literals in the code
//    (Sec. III-B, Listings 2-3: per-column inclusion/exclusion updates).
//  * Chunks are power-of-two sized and aligned, so at local step l every lane
//    flips the same column ctz(l) (Theorem 1) with the same direction, except
//    at l = 2^(kappa-1) where the direction is the parity of the chunk index
//    (Lemma 2, first case); that one step uses a per-lane +-1 multiplier.  The
//    step that would differ in column (l = 2^kappa, Lemma 2's second case) is
//    the next chunk's start and is never executed inside a chunk.
//  * The loop body is a static unrolled block of 2^u steps whose columns and
//    signs are compile-time constants, followed by one wave-uniform dynamic
//    step whose column ctz(l) selects a row of a constant table of entries.
//  * Products are cached by level (a generalisation of Sec. V's cached
//    global product, Listings 4-5): rows are grouped by the first flipped
//    column that touches them, S_l = product of x over levels >= l is kept,
//    and a flip of column j recomputes only the levels up to the highest
//    level column j touches.  With one level this is the plain full product.
//  * Zero-aware pruning (exact): intervals of Gray indices whose terms all
//    have an exactly-zero factor in every lane are skipped.  A block of steps
//    that only some lanes of a wave need is not evaluated in place: each
//    needing lane queues the block's start state in LDS and takes the skip
//    path; after the walks, the workgroup evaluates all queued blocks, one per
//    thread, in a fixed order (so the sum stays deterministic).
//  * Rows >= k (HYBRID) live in global memory, [row][lane] so that a wave's
//    accesses are contiguous (Sec. V), or in LDS with the same layout per
//    workgroup (the shared-memory tier the paper leaves to future work), and
//    their product is recomputed only when a column that touches them flips.
#include <cmath>
#include <cstdio>
#include <map>
#include <set>
#include <unordered_map>
#include <unordered_set>
#include <sstream>

#include "perm_internal.h"

namespace permx {

const char *const kGrayKernelName = "perm_gray";

namespace {

std::string lit(double v) {
    char b[64];
    snprintf(b, sizeof b, "%a", v);  // exact binary64 value as a hex-float literal
    return b;
}

enum class Sign { Plus, Minus, Uniform, Lane };

struct Gen {
    const Plan &p;
    std::ostringstream os;
    int tmp = 0;
    std::vector<std::vector<int>> level_rows;

    explicit Gen(const Plan &plan) : p(plan) {
        level_rows.assign(p.nlevels, {});
        for (int r = 0; r < p.n; ++r) level_rows[p.row_level[r]].push_back(r);
    }

    // Block queue: per wave kQueueSlots slots of the start state of a block
    // pair (rows of levels <= qtop, then S_{qtop+1}, then the direction of
    // the middle step), stored [field][slot].
    bool use_queue = false;
    int qslots = 0;
    int qtop = 0;
    std::vector<int> qrows;
    // (exact mode: then R_{qtop+1}, the residue of S_{qtop+1})
    int qfields() const { return (int)qrows.size() + 2 + (p.exact ? 1 : 0); }

    // Exact mode with pruned blocks: the walk between evaluated blocks keeps
    // only the FP64 products S_l (its zero tests need nothing else); the
    // residues R_l are formed again from x where a term is evaluated (at an
    // evaluated or queued block, and under a wave-uniform branch for a
    // nonzero walk term).  walk_s_only marks code emitted for the walk.
    bool lazy_r = false;
    bool walk_s_only = false;
    // Nested accumulation (FP64 kernels with column-0 pairing): instead of
    // the cached products S_l = P_l S_{l+1} the kernel keeps each level's
    // own product P_l and one accumulator c_l per level, holding the sum of
    // the terms since level l+1 last changed as a coefficient of
    // P_{l+1} ... P_{L-1} (c_0: the pairs' brackets).  A step whose highest
    // level is t first moves c_0 .. c_{t-1} up through the products they
    // multiply (c_l += c_{l-1} P_l, old P_l), then changes x and the touched
    // P_l, then starts c_0 with its term: t operations where the cached
    // products need t multiplies and an accumulate.  cz[l] marks an
    // accumulator whose sum has moved up (its register is stale and its next
    // fill is a multiply, not an FMA).  The loop's last (dynamic) step moves
    // everything up to T, the highest level any step of the loop reaches, so
    // c_1 .. c_{T-1} are empty at the loop's end and are taken as empty at
    // its top (their registers hold 0 on entry).
    bool horner = false;
    // Exact mode in nested form: beside c_l, r_l (the sum's residue modulo
    // the prime, reduced at every move) and a_l (the sum of |term| for the
    // error bound), moved up through RP_l (P_l's residue) and |P_l|.
    bool hx = false;
    // r_l's moves since its last reduction (0: reduced).  A move adds less
    // than (2^23 + 2)^2 < 2^46.01, so after at most kMaxDeferred of them
    // |r_l| < 2^50.1 and the next FMA into it stays exact; r_l is reduced
    // before it multiplies (then every product is below 2^46.01).
    std::vector<int> rdef;
    static constexpr int kMaxDeferred = 16;
    long acc_written = 0;  // accumulator operations as written (per chunk; the error bound's length)
    long body_acc = 0;     // of those, one loop iteration's
    double acc_chunk = 0;  // all of one chunk
    std::vector<char> cz;
    int loop_top = 0;  // T

    // Bracket tracking (nested accumulation): with two entries in column 0
    // the pair's bracket a_r x_s + a_s x_r + a_r a_s is affine in x, so it is
    // kept in `dp` and moved by every step that touches row r or s (one add
    // of the column's constant change); the level-0 rows' own x are never
    // needed (with one entry the bracket is a constant).
    bool dtrack = false;
    int dyn_dslot = -1;  // slot of the bracket's change in the dynamic table

    // Copies over the walk's first m columns (its most frequent flips:
    // columns 1..m with pairing, else 0..m-1; m = copy_cols): row r (at a
    // level >= 1 with pairing) is kept once per subset sigma of Tr[r], the
    // copied columns touching it (x<r> for none, x<r>_<sigma> with
    // those columns' entries added), level l once per subset of Tl[l] (P<l>,
    // P<l>_<sigma>), the bracket once per subset of T0 (dp, dp_<sigma>).  ts
    // is the set of those columns in x where a step is emitted (none at
    // every chunk start, loop top and dynamic step); a flip of copied column
    // c only toggles bit c - cbase of ts, and every other flip moves every copy.
    int cm = 0;
    int cbase = 1;  // the first copied column (the walk's first: 1 with pairing, else 0)
    int lv0 = 1;    // the lowest level whose product a step forms (0: nested, no pairing)
    unsigned ts = 0u, T0 = 0u;
    // Levels whose rows changed since their products were last formed (the
    // nested-accumulation kernels form only those again).
    std::vector<char> dirty;
    void touch_row(int r) {
        if (horner && r < p.n && (p.row_level[r] >= 1 || !p.pair0)) dirty[p.row_level[r]] = 1;
    }
    std::vector<unsigned> Tr, Tl;
    static std::string sub(const std::string &base, unsigned sigma) {
        return sigma ? base + "_" + std::to_string(sigma) : base;
    }
    // every subset of T (the empty one first)
    static std::vector<unsigned> subsets(unsigned T) {
        std::vector<unsigned> v;
        for (unsigned sg = 0;; sg = (sg - T) & T) {  // next subset in increasing order
            v.push_back(sg);
            if (sg == T) break;
        }
        return v;
    }
    std::string xv(int r, unsigned sigma) const { return sub(xname(r), sigma & Tr[r]); }
    std::string pname(int l) const { return sub("P" + std::to_string(l), ts & Tl[l]); }
    std::string dname() const { return sub("dp", ts & T0); }

    // ---- FP64 operations of the step loop (nested-accumulation kernels) ----
    // Each FP64 operation the loop emits is noted with its operands: a value
    // is named by its operation and its operands' values, and it varies in
    // the loop when an operand does (every name the loop assigns varies at
    // its top).  An operation on values that do not vary is hoisted out of
    // the loop by the compiler and one that this iteration already computed
    // is reused, so only the others are counted.  Without a loop (one pass
    // per chunk) every distinct operation is counted.
    bool track = false, counting = false, all_vary = false;
    double loop_ops = -1, loop_flops = -1;  // per Gray term, when counted
    double loop_terms = 0;                  // Gray terms per iteration
    uint64_t loop_iters = 0;
    int sign_fmas = 0;                      // table-entry FMAs per iteration
    // values are numbered: a value's key is its operation and its operands'
    // numbers (a name the loop does not assign is a value of its own)
    std::unordered_map<std::string, int> interned;
    std::unordered_map<std::string, std::pair<int, bool>> vid;  // name -> (value, varies)
    std::unordered_set<int> seen;
    std::unordered_set<std::string> assigned;
    double cnt_ops = 0, cnt_flops = 0;
    double hoist_ops = 0, hoist_flops = 0;  // the loop's invariant operations (once per chunk)
    int intern(const std::string &key) { return interned.emplace(key, (int)interned.size()).first->second; }
    std::pair<int, bool> val(const std::string &name) {
        auto it = vid.find(name);
        return it != vid.end() ? it->second : std::make_pair(intern("=" + name), false);
    }
    // +1 or -1 if the value is that constant (a literal, or its sign), else 0
    std::map<std::string, int> unit;
    int unit_of(const std::string &name) const {
        auto it = unit.find(name);
        if (it != unit.end()) return it->second;
        std::string t = name;
        while (t.size() > 2 && t.front() == '(' && t.back() == ')') t = t.substr(1, t.size() - 2);
        if (t == "0x1p+0") return 1;
        if (t == "-0x1p+0") return -1;
        return 0;
    }
    void note(const std::string &lhs, const char *op, std::initializer_list<std::string> args, int flops,
              bool free = false) {
        if (!track) return;
        // a product with a factor +-1 is a sign (folded into its use), an
        // FMA with one a plain add
        const std::vector<std::string> av(args);
        const std::string sop(op);
        if (sop == "mul" && av.size() == 2 && (unit_of(av[0]) || unit_of(av[1]))) {
            const int u0 = unit_of(av[0]), u1 = unit_of(av[1]);
            const std::string &other = u0 ? av[1] : av[0];
            const int sgn = u0 ? u0 : u1;
            const auto v = val(other);
            vid[lhs] = {intern(std::string(sgn > 0 ? "id(" : "neg(") + std::to_string(v.first) + ")"), v.second};
            unit[lhs] = unit_of(other) * sgn;
            assigned.insert(lhs);
            return;
        }
        if (sop == "fma" && (unit_of(av[0]) || unit_of(av[1]))) flops = 1;
        if (sop == "neg" || sop == "id") unit[lhs] = (sop == "neg" ? -1 : 1) * unit_of(av[0]);
        else unit.erase(lhs);
        std::string key = std::string(op) + "(";
        bool vary = all_vary;
        for (const std::string &a : args) {
            const auto v = val(a);
            key += std::to_string(v.first) + ",";
            vary = vary || v.second;
        }
        key += ")";
        const int id = intern(key);
        if (counting && seen.insert(id).second && !free) {
            // varying: every iteration; not varying: once, before the loop
            (vary ? cnt_ops : hoist_ops) += 1;
            (vary ? cnt_flops : hoist_flops) += flops;
        }
        vid[lhs] = {id, vary};
        assigned.insert(lhs);
    }
    // a value that costs no operation of its own (a sign folded into its use)
    void derive(const std::string &lhs, const char *op, std::initializer_list<std::string> args) {
        note(lhs, op, args, 0, true);
    }
    void alias(const std::string &lhs, const std::string &rhs) {
        if (!track) return;
        vid[lhs] = val(rhs);
        if (unit_of(rhs)) unit[lhs] = unit_of(rhs); else unit.erase(lhs);
        assigned.insert(lhs);
    }
    void varies(const std::string &name) {
        if (!track) return;
        unit.erase(name);
        vid[name] = {intern("(" + name + ")"), true};
        assigned.insert(name);
    }

    // Coefficients of x_r and x_s in the bracket and the bracket at x.
    void bracket_coeffs(double &cr, double &cs) const {
        const Ccs &B = p.B;
        const int q0 = B.colptr[0];
        const double ar = B.val[B.rowidx[q0] == p.pair_r ? q0 : q0 + 1];
        const double as = B.val[B.rowidx[q0] == p.pair_s ? q0 : q0 + 1];
        cr = as;  // d/dx_r
        cs = ar;  // d/dx_s
    }
    // Change of the bracket when column j's entries are added to x.
    double bracket_delta(int j) const {
        const Ccs &B = p.B;
        double cr, cs, dr = 0.0, ds = 0.0;
        bracket_coeffs(cr, cs);
        for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) {
            if (B.rowidx[q] == p.pair_r) dr = B.val[q];
            if (B.rowidx[q] == p.pair_s) ds = B.val[q];
        }
        return std::fma(cr, dr, cs * ds);
    }
    bool touches_level0(int j) const {
        const Ccs &B = p.B;
        for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q)
            if (p.row_level[B.rowidx[q]] == 0) return true;
        return false;
    }

    // c_0 .. c_{t-1} into c_t through the current products.
    void flush_to(int t, const char *I) {
        for (int l = 1; l <= t; ++l) {
            const std::string cl = "c" + std::to_string(l), cb = "c" + std::to_string(l - 1);
            if (cz[l]) {
                os << I << cl << " = " << cb << " * " << pname(l) << ";\n";
                note(cl, "mul", {cb, pname(l)}, 1);
            } else {
                os << I << cl << " = fma(" << cb << ", " << pname(l) << ", " << cl << ");\n";
                note(cl, "fma", {cb, pname(l), cl}, 2);
            }
            ++acc_written;
            if (hx) {
                const std::string al = "a" + std::to_string(l), ab = "a" + std::to_string(l - 1);
                const std::string rl = "r" + std::to_string(l), rb = "r" + std::to_string(l - 1);
                if (l - 1 >= 1 && rdef[l - 1] > 0) settle_residue(l - 1, I);  // reduced before it multiplies
                const std::string rp = "R" + pname(l), t = fresh();
                int k;
                if (cz[l]) {
                    os << I << al << " = " << ab << " * fabs(" << pname(l) << ");\n";
                    note(al, "mula", {ab, pname(l)}, 1);
                    os << I << "const double " << t << " = " << rb << " * " << rp << ";\n";
                    note(t, "mul", {rb, rp}, 1);
                    k = 1;
                } else {
                    os << I << al << " = fma(" << ab << ", fabs(" << pname(l) << "), " << al << ");\n";
                    note(al, "fmaa", {ab, pname(l), al}, 2);
                    os << I << "const double " << t << " = fma(" << rb << ", " << rp << ", " << rl << ");\n";
                    note(t, "fma", {rb, rp, rl}, 2);
                    k = rdef[l] + 1;
                }
                // |r_{l-1}|, |RP_l| < 2^23 + 2 and at most kMaxDeferred
                // earlier moves in r_l: the product and the sum are exact; the
                // reduction waits until r_l multiplies or the count is reached
                if (k > kMaxDeferred) {
                    const std::string red = reduce_expr(t, I);
                    os << I << rl << " = " << red << ";\n";
                    note(rl, "red", {t}, 1);
                    k = 0;
                } else {
                    os << I << rl << " = " << t << ";\n";
                    alias(rl, t);
                }
                rdef[l] = k;
            }
            cz[l] = 0;
            if (l >= 2) cz[l - 1] = 1;
        }
    }

    std::string fresh() { return "t" + std::to_string(tmp++); }
    std::string xname(int r) const { return "x" + std::to_string(r); }
    std::string cold_addr(int r) const {
        if (p.cold_lds) return "xl[" + std::to_string((r - p.k) * p.block) + " + threadIdx.x]";
        return "xg[(u64)" + std::to_string(r - p.k) + " * xs + lid]";
    }

    // Pairwise (tree) product of the named values; returns the result name.
    std::string product(std::vector<std::string> vals, const char *ind) {
        if (vals.empty()) return "1.0";
        while (vals.size() > 1) {
            std::vector<std::string> next;
            for (size_t i = 0; i + 1 < vals.size(); i += 2) {
                std::string t = fresh();
                os << ind << "const double " << t << " = " << vals[i] << " * " << vals[i + 1] << ";\n";
                note(t, "mul", {vals[i], vals[i + 1]}, 1);
                next.push_back(t);
            }
            if (vals.size() % 2) next.push_back(vals.back());
            vals.swap(next);
        }
        return vals[0];
    }

    // Name of row r's current x value; a cold row not in `cur` is loaded
    // from global memory (or LDS).
    std::string value_of(int r, std::map<int, std::string> &cur, const char *ind) {
        if (r < p.k) return xname(r);
        auto it = cur.find(r);
        if (it != cur.end()) return it->second;
        std::string t = fresh();
        os << ind << "const double " << t << " = " << cold_addr(r) << ";\n";
        cur[r] = t;
        return t;
    }

    // Names of the current x values of level l's rows.
    std::vector<std::string> level_values(int l, std::map<int, std::string> &cur, const char *ind) {
        std::vector<std::string> v;
        for (int r : level_rows[l]) v.push_back(value_of(r, cur, ind));
        return v;
    }

    // The same in copy sigma (columns <= m in sigma added).
    std::vector<std::string> level_values_in(int l, unsigned sigma, std::map<int, std::string> &cur,
                                             const char *ind) {
        std::vector<std::string> v;
        for (int r : level_rows[l]) v.push_back(Tr[r] & sigma ? xv(r, sigma) : value_of(r, cur, ind));
        return v;
    }

    // ---- exact mode (integer-valued matrices, x holds y = 2x) ----
    // The products of level l's sub-products (each an exact integer of at
    // most 2^20 in magnitude); `weight` (0 or 1) joins the first.
    std::vector<std::string> part_products(int l, std::map<int, std::string> &cur, const char *I,
                                           const char *weight = nullptr) {
        std::vector<std::string> qs;
        const auto &parts = p.level_parts[l];
        for (size_t pi = 0; pi < parts.size(); ++pi) {
            std::vector<std::string> v;
            for (int r : parts[pi]) v.push_back(value_of(r, cur, I));
            if (pi == 0 && weight) v.push_back(weight);
            qs.push_back(product(v, I));
        }
        return qs;
    }

    // q * r reduced modulo the prime: |q| <= 2^20 and |r| < 2^23 + 2, so the
    // product is exact (< 2^44) and rint(t / p) is within one of its quotient;
    // the result lies in (-p/2 - 2, p/2 + 2).
    std::string mulmod(const std::string &q, const std::string &r, const char *I) {
        const std::string t = fresh(), m = fresh();
        os << I << "const double " << t << " = " << q << " * " << r << ";\n";
        note(t, "mul", {q, r}, 1);
        const std::string red = reduce_expr(t, I);  // emits the quotient first
        os << I << "const double " << m << " = " << red << ";\n";
        note(m, "red", {t}, 1);
        return m;
    }
    // r_l brought back to (-p/2 - 2, p/2 + 2)
    void settle_residue(int l, const char *I) {
        const std::string rl = "r" + std::to_string(l);
        const std::string red = reduce_expr(rl, I);
        os << I << rl << " = " << red << ";\n";
        note(rl, "red", {rl}, 1);
        rdef[l] = 0;
    }
    // every r_l reduced (where the generated code joins: the loop's top and
    // end, the chunk's end)
    void settle_residues(const char *I) {
        for (int l = 1; l < (int)rdef.size(); ++l)
            if (rdef[l] > 0) settle_residue(l, I);
    }
    // t reduced modulo the prime (an exact remainder for exact t below 2^53;
    // the quotient's multiply is an FP64 operation of its own)
    std::string reduce_expr(const std::string &t, const char *I) {
        const std::string q = fresh();
        os << I << "const double " << q << " = rint(" << t << " * pinv);\n";
        note(q, "quot", {t}, 1);
        return "fma(-" + q + ", pmod, " + t + ")";
    }
    // RP_l of copy sigma: the residue of level l's product, from its exact
    // sub-products (each at most 2^20 in magnitude)
    void level_residue(int l, unsigned sigma, std::map<int, std::string> &cur, const char *I, bool decl = false) {
        std::vector<std::string> qs;
        for (const auto &part : p.level_parts[l]) {
            std::vector<std::string> v;
            for (int r : part) v.push_back(cm && (Tr[r] & sigma) ? xv(r, sigma) : value_of(r, cur, I));
            qs.push_back(product(v, I));
        }
        const std::string res = residue_chain(qs, 0, "", I);
        const std::string name = "R" + sub("P" + std::to_string(l), sigma);
        os << I << (decl ? "double " : "") << name << " = " << res << ";\n";
        alias(name, res);
    }

    // residue of sub-products qs[from..] times `r` (r empty: no factor)
    std::string residue_chain(const std::vector<std::string> &qs, size_t from, std::string r, const char *I) {
        for (size_t i = qs.size(); i-- > from;) r = r.empty() ? qs[i] : mulmod(qs[i], r, I);
        return r;
    }

    // racc back to (-p/2 - 2, p/2 + 2): after at most 1023 terms of at most
    // 2^20 (2^23 + 2) each it is below 2^53, where rint(racc / p) is exact
    // enough for an exact remainder.
    void reduce_racc(const char *I) {
        if (p.exact && !hx) os << I << "racc = fma(-rint(racc * pinv), pmod, racc);\n";
    }

    // x updates of one Gray step flipping column j in direction sg; updated
    // cold rows are recorded in `cur`.
    void update(int j, Sign sg, std::map<int, std::string> &cur, const char *I) {
        const Ccs &B = p.B;
        if (dtrack && touches_level0(j)) {
            for (unsigned sgm : subsets(T0)) emit_add(sub("dp", sgm), lit(bracket_delta(j)), sg, I);
        }
        for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) {
            const int r = B.rowidx[q];
            if (horner && p.pair0 && p.row_level[r] == 0) continue;  // level 0 lives in the bracket
            touch_row(r);
            const std::string a = lit(B.val[q]);
            if (cm && Tr[r])
                for (unsigned sgm : subsets(Tr[r]))
                    if (sgm) emit_add(xv(r, sgm), a, sg, I);
            std::string target;
            if (r < p.k) {
                target = xname(r);
            } else {
                target = fresh();
                os << I << "double " << target << " = " << cold_addr(r) << ";\n";
                cur[r] = target;
            }
            emit_add(target, a, sg, I);
            if (r >= p.k) os << I << cold_addr(r) << " = " << target << ";\n";
        }
    }

    // target += a in direction sg
    void emit_add(const std::string &target, const std::string &a, Sign sg, const char *I) {
        if (sg == Sign::Plus)
            os << I << target << " += " << a << ";\n";
        else if (sg == Sign::Minus)
            os << I << target << " -= " << a << ";\n";
        else if (sg == Sign::Uniform)
            os << I << target << " += (neg ? -(" << a << ") : (" << a << "));\n";
        else
            os << I << target << " = fma(lsgn, " << a << ", " << target << ");\n";
        note(target, sg == Sign::Plus ? "add" : sg == Sign::Minus ? "sub" : sg == Sign::Uniform ? "addu" : "addl",
             {target, a, sg == Sign::Uniform ? "neg" : "lsgn"}, 1);
    }

    // Recompute the cached product of level l: S_l = prod(level l) * S_{l+1}.
    void refresh_level(int l, std::map<int, std::string> &cur, const char *I) {
        if (p.exact && !horner) {
            // S_l = P_l * S_{l+1} in FP64; R_l = P_l R_{l+1} modulo the prime
            const std::vector<std::string> qs = part_products(l, cur, I);
            const std::string pl = product(qs, I);
            const bool top = l + 1 >= p.nlevels;
            os << I << "S" << l << " = " << pl;
            if (!top) os << " * S" << l + 1;
            os << ";\n";
            if (walk_s_only) return;  // residues are formed again where a term is evaluated
            const std::string r = residue_chain(qs, 0, top ? "" : "R" + std::to_string(l + 1), I);
            os << I << "R" << l << " = " << r << ";\n";
            return;
        }
        if (horner && !dirty[l]) return;  // its products are current
        if (horner) dirty[l] = 0;
        std::vector<std::string> v = level_values(l, cur, I);
        if (horner) {
            const std::string pr = product(v, I);
            os << I << "P" << l << " = " << pr << ";\n";
            alias("P" + std::to_string(l), pr);
            if (hx) level_residue(l, 0u, cur, I);
            if (cm)
                for (unsigned sgm : subsets(Tl[l])) {
                    if (!sgm) continue;
                    const std::string pi = product(level_values_in(l, sgm, cur, I), I);
                    os << I << sub("P" + std::to_string(l), sgm) << " = " << pi << ";\n";
                    alias(sub("P" + std::to_string(l), sgm), pi);
                    if (hx) level_residue(l, sgm, cur, I);
                }
            return;
        }
        if (l + 1 < p.nlevels) v.push_back("S" + std::to_string(l + 1));
        std::string prod = product(v, I);
        os << I << "S" << l << " = " << prod << ";\n";
    }

    // R_l for l = rtop down to lo, from the current x (exact mode).  Levels
    // above rtop hold rows that no column of the chunk flips: their residues,
    // formed at the chunk start, stay valid for the whole chunk.
    int rtop = 0;
    void recompute_residues(int lo, std::map<int, std::string> &cur, const char *I) {
        for (int l = std::min(rtop, p.nlevels - 1); l >= lo; --l) {
            const std::vector<std::string> qs = part_products(l, cur, I);
            const std::string r = residue_chain(qs, 0, l + 1 < p.nlevels ? "R" + std::to_string(l + 1) : "", I);
            os << I << "R" << l << " = " << r << ";\n";
        }
    }

    // One Gray step: flip column j with the given direction, refresh the
    // cached products it invalidates and accumulate the term with sign
    // term_sign into accumulator acc.
    void step(int j, Sign sg, int term_sign, int acc, const char *ind) {
        std::map<int, std::string> cur;
        os << ind << "{  // column " << j
           << (sg == Sign::Plus ? " +" : sg == Sign::Minus ? " -" : sg == Sign::Uniform ? " uniform sign" : " lane sign")
           << "\n";
        std::string in = std::string(ind) + "  ";
        const char *I = in.c_str();
        if (horner) flush_to(p.col_top[j], I);
        if (cm && j >= cbase && j < cbase + cm) {
            // column j in (Plus) or out (Minus): other copies become current
            const unsigned bit = 1u << (j - cbase);
            if ((sg == Sign::Plus) != !(ts & bit) || (sg != Sign::Plus && sg != Sign::Minus))
                os << "#error copies of x out of step\n";  // a generator fault: fail to compile
            ts ^= bit;
        } else {
            update(j, sg, cur, I);
            for (int l = p.col_top[j]; l >= lv0; --l) refresh_level(l, cur, I);
        }
        accumulate(term_sign, acc, cur, I, nullptr, horner && p.col_top[j] >= 1);
        os << ind << "}\n";
    }

    // acc += term_sign * (product of level 0) * S_1   (one FMA)
    void accumulate(int term_sign, int acc, std::map<int, std::string> &cur, const char *I,
                    const char *weight = nullptr, bool fresh_run = false) {
        if (p.pair0) {
            // the pair (-1)^i S_1 (P(x) - P(x + a)) over column 0's rows: one
            // row r gives -a_r; two rows r, s give -(a_r x_s + a_s x_r + a_r a_s)
            const Ccs &B = p.B;
            const int q0 = B.colptr[0];
            std::string d;
            if (B.colptr[1] - q0 == 1) {
                d = "(" + lit(B.val[q0]) + ")";
            } else if (dtrack) {
                d = dname();
            } else {
                // r in the inner FMA, t in the outer (the plan puts there the
                // row that more often changes)
                const int r = p.pair_r, t = p.pair_s;
                const double ar = B.val[B.rowidx[q0] == r ? q0 : q0 + 1];
                const double at = B.val[B.rowidx[q0] == t ? q0 : q0 + 1];
                d = fresh();
                os << I << "const double " << d << " = fma(" << lit(ar) << ", " << xname(t) << ", fma(" << lit(at)
                   << ", " << xname(r) << ", " << lit(ar * at) << "));\n";
            }
            if (weight) {
                const std::string dw = fresh();
                os << I << "const double " << dw << " = " << d << " * " << weight << ";\n";
                note(dw, "mul", {d, weight}, 1);
                d = dw;
            }
            // term_sign * (-d) * S_1; exact mode: d is an integer (y units,
            // within the sub-product bound), so its residue is d R_1
            const char *sg = term_sign < 0 ? "" : "-";
            if (horner) {
                // the pair's bracket starts c_0 (after a flush) or adds to it
                if (fresh_run) {
                    os << I << "c0 = " << sg << d << ";\n";
                    derive("c0", *sg ? "neg" : "id", {d});  // a sign the consumer folds in
                } else {
                    os << I << "c0 = c0 + " << sg << d << ";\n";
                    note("c0", *sg ? "subc" : "addc", {"c0", d}, 1);
                    ++acc_written;
                }
                if (hx) {
                    // exact mode: d is an integer of at most 2^20 (y units), its
                    // own residue; r_0 is brought back to range after each add
                    if (fresh_run) {
                        os << I << "a0 = fabs(" << d << ");\n";
                        derive("a0", "abs", {d});
                        os << I << "r0 = " << sg << d << ";\n";
                        derive("r0", *sg ? "neg" : "id", {d});
                    } else {
                        os << I << "a0 = a0 + fabs(" << d << ");\n";
                        note("a0", "adda", {"a0", d}, 1);
                        const std::string t = fresh();
                        os << I << "const double " << t << " = r0 + " << sg << d << ";\n";
                        note(t, *sg ? "subc" : "addc", {"r0", d}, 1);
                        const std::string red = reduce_expr(t, I);
                        os << I << "r0 = " << red << ";\n";
                        note("r0", "red", {t}, 1);
                    }
                }
                return;
            }
            os << I << "acc" << acc << " = fma(" << sg << d << ", S1, acc" << acc << ");\n";
            if (p.exact) {
                os << I << "racc = fma(" << sg << d << ", R1, racc);\n";
                os << I << "accA = fma(fabs(" << d << "), fabs(S1), accA);\n";
            }
            return;
        }
        if (p.exact) {
            // the term is pr * last (exact inside the FMA); its residue is the
            // first sub-product times the residue of the rest; A (the error
            // bound's sum) takes |term|
            const std::vector<std::string> qs = part_products(0, cur, I, weight);
            const char *sg = term_sign < 0 ? "-" : "";
            std::string pr, last, rest;
            if (p.nlevels > 1 && walk_s_only) {
                // a walk term: its residue only where some lane's term is
                // nonzero, from residues formed again from x (reduced at once,
                // so any number of walk terms keeps racc exact)
                pr = product(qs, I);
                os << I << "acc" << acc << " = fma(" << sg << pr << ", S1, acc" << acc << ");\n";
                os << I << "accA = fma(fabs(" << pr << "), fabs(S1), accA);\n";
                os << I << "if (__any(" << pr << " != 0.0 && S1 != 0.0)) {\n";
                const std::string in2 = std::string(I) + "  ";
                recompute_residues(1, cur, in2.c_str());
                rest = residue_chain(qs, 1, "R1", in2.c_str());
                os << in2 << "racc = fma(" << sg << qs[0] << ", " << rest << ", racc);\n";
                os << in2 << "racc = fma(-rint(racc * pinv), pmod, racc);\n";
                os << I << "}\n";
                return;
            }
            if (p.nlevels > 1) {
                pr = product(qs, I);
                last = "S1";
                rest = residue_chain(qs, 1, "R1", I);
            } else {
                std::vector<std::string> head(qs.begin(), qs.end() - 1);
                pr = product(head, I);
                last = qs.back();
                rest = qs.size() > 1 ? residue_chain(qs, 1, "", I) : "1.0";
            }
            os << I << "acc" << acc << " = fma(" << sg << pr << ", " << last << ", acc" << acc << ");\n";
            os << I << "racc = fma(" << sg << qs[0] << ", " << rest << ", racc);\n";
            os << I << "accA = fma(fabs(" << pr << "), fabs(" << last << "), accA);\n";
            return;
        }
        if (horner) {
            // nested accumulation without pairing: the term's level-0 factor
            // is P_0 (its current copy), which starts c_0 or adds to it
            std::string d = pname(0);
            if (weight) {
                const std::string dw = fresh();
                os << I << "const double " << dw << " = " << d << " * " << weight << ";\n";
                note(dw, "mul", {d, weight}, 1);
                d = dw;
            }
            const char *sg = term_sign < 0 ? "-" : "";
            if (fresh_run) {
                os << I << "c0 = " << sg << d << ";\n";
                derive("c0", *sg ? "neg" : "id", {d});
            } else {
                os << I << "c0 = c0 + " << sg << d << ";\n";
                note("c0", *sg ? "subc" : "addc", {"c0", d}, 1);
            }
            return;
        }
        std::vector<std::string> v = level_values(0, cur, I);
        if (weight) v.push_back(weight);
        std::string last;
        if (p.nlevels > 1) {
            last = "S1";
        } else {
            last = v.back();
            v.pop_back();
        }
        std::string pr = product(v, I);
        os << I << "acc" << acc << " = fma(" << (term_sign < 0 ? "-" : "") << pr << ", " << last << ", acc" << acc
           << ");\n";
    }

    // Rows that the dynamic columns u+1 .. kappa-1 touch, and the table of
    // their entries: row (jj - (u+1)) holds column jj's value for each of
    // those rows (0 where the column has no entry); row kappa - u - 1 (jj =
    // kappa, "no column") is all zeros.  Emitted as a __constant__ array, so a
    // wave-uniform jj reads it with scalar loads.
    std::vector<int> dyn_rows;
    int dyn_lo = 0, dyn_hi = -1;  // columns in the table

    void build_dyn_table(int lo, int hi) {
        const Ccs &B = p.B;
        dyn_lo = lo;
        dyn_hi = hi;
        std::vector<char> used(p.n, 0);
        dyn_dslot = -1;
        bool dtouch = false;
        for (int j = lo; j <= hi; ++j) {
            for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) used[B.rowidx[q]] = 1;
            dtouch = dtouch || touches_level0(j);
        }
        dyn_rows.clear();
        for (int r = 0; r < p.n; ++r)
            if (used[r] && !(horner && p.pair0 && p.row_level[r] == 0)) dyn_rows.push_back(r);
        // with bracket tracking, one more slot per column: the bracket's change
        if (dtrack && dtouch) dyn_dslot = (int)dyn_rows.size();
        const size_t R = dyn_rows.size() + (dyn_dslot >= 0 ? 1 : 0);
        if (R == 0) return;
        std::vector<double> tab((size_t)(hi - lo + 2) * R, 0.0);
        std::vector<int> slot(p.n, -1);
        for (size_t i = 0; i < dyn_rows.size(); ++i) slot[dyn_rows[i]] = (int)i;
        for (int j = lo; j <= hi; ++j) {
            for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q)
                if (slot[B.rowidx[q]] >= 0) tab[(size_t)(j - lo) * R + slot[B.rowidx[q]]] = B.val[q];
            if (dyn_dslot >= 0) tab[(size_t)(j - lo) * R + dyn_dslot] = bracket_delta(j);
        }
        os << "__constant__ double dyn_tab[" << tab.size() << "] = {";
        for (size_t i = 0; i < tab.size(); ++i) os << (i ? "," : "") << (i % 8 ? " " : "\n  ") << lit(tab[i]);
        os << "};\n";
    }

    // Flip of the wave-uniform column `jvar` (one of the table's columns, or
    // dyn_hi + 1 for none) with direction `svar`: each row the table covers
    // takes one FMA with its entry (0 leaves x unchanged).  Returns the
    // highest level the table's columns touch.
    int dyn_flip(const char *jvar, const char *svar, std::map<int, std::string> &cur, const char *I) {
        int top_max = 0;
        for (int j = dyn_lo; j <= dyn_hi; ++j) top_max = std::max(top_max, p.col_top[j]);
        const size_t R = dyn_rows.size() + (dyn_dslot >= 0 ? 1 : 0);
        if (R == 0) return top_max;
        const std::string tp = fresh();
        os << I << "const double* " << tp << " = dyn_tab + (u32)(" << jvar << " - " << dyn_lo << ") * " << R << "u;\n";
        varies(tp);
        if (dyn_dslot >= 0)
            for (unsigned sgm : subsets(T0)) {
                const std::string d = sub("dp", sgm);
                os << I << d << " = fma(" << svar << ", " << tp << "[" << dyn_dslot << "], " << d << ");\n";
                note(d, "fma", {svar, tp + std::to_string(dyn_dslot), d}, 1);
                if (counting) ++sign_fmas;
            }
        for (size_t i = 0; i < dyn_rows.size(); ++i) {
            const int r = dyn_rows[i];
            touch_row(r);
            std::string target;
            if (r < p.k) {
                target = xname(r);
            } else {
                target = fresh();
                os << I << "double " << target << " = " << cold_addr(r) << ";\n";
                cur[r] = target;
            }
            os << I << target << " = fma(" << svar << ", " << tp << "[" << i << "], " << target << ");\n";
            note(target, "fma", {svar, tp, std::to_string(i), target}, 1);
            if (counting) ++sign_fmas;
            if (cm && r < p.k && Tr[r])
                for (unsigned sgm : subsets(Tr[r])) {
                    if (!sgm) continue;
                    const std::string x = xv(r, sgm);
                    os << I << x << " = fma(" << svar << ", " << tp << "[" << i << "], " << x << ");\n";
                    note(x, "fma", {svar, tp, std::to_string(i), x}, 1);
                    if (counting) ++sign_fmas;
                }
            if (r >= p.k) os << I << cold_addr(r) << " = " << target << ";\n";
        }
        return top_max;
    }

    // Static block of steps i = 1 .. 2^u - 1 inside a 2^(u+1)-aligned pair of
    // blocks; `second` selects the second block (where the step i = 2^(u-1)
    // excludes instead of includes).
    // (Column-0 pairing: i counts paired steps and step i flips column
    // ctz(i) + 1, with Theorem 1's direction taken from i.)
    void static_block(bool second, const char *ind) {
        const int U = 1 << p.u;
        const int c0 = p.pair0 ? 1 : 0;
        for (int i = 1; i < U; ++i) {
            const int j = __builtin_ctz(i);
            bool neg;
            if (j + 1 < p.u)
                neg = (i >> (j + 1)) & 1;  // Theorem 1 with the chunk-local index
            else
                neg = second;              // bit u of the local index
            step(j + c0, neg ? Sign::Minus : Sign::Plus, (i & 1) ? -1 : 1, (i >> 1) & 1, ind);
        }
        if (U > 1) reduce_racc(ind);
    }

    std::string run() {
        const Ccs &B = p.B;
        const int n = p.n, k = p.k, L = p.nlevels;
        const int kappa = p.kappa, u = p.u, U = 1 << u;
        const uint64_t DELTA = 1ull << kappa;
        // the walk: local steps of a chunk, its length and the column offset
        // (column-0 pairing: paired steps flipping columns 1 ..)
        const int c0 = p.pair0 ? 1 : 0;
        const int kw = kappa - c0;
        horner = p.nested && !p.cold && L >= 2;
        hx = horner && p.exact;
        rdef.assign(L, 0);
        if (hx && !p.pair0) os << "#error exact nested kernels are paired\n";  // the plan pairs them
        dtrack = horner && p.pair0 && p.B.colptr[1] - p.B.colptr[0] == 2;
        cm = horner ? p.copy_cols : 0;
        cbase = c0;
        lv0 = horner && !p.pair0 ? 0 : 1;
        dirty.assign(L, 0);
        ts = 0u;
        T0 = 0u;
        Tr.assign(n, 0u);
        Tl.assign(L, 0u);
        for (int c = cbase; c < cbase + cm; ++c)
            for (int q = B.colptr[c]; q < B.colptr[c + 1]; ++q) {
                const int r = B.rowidx[q];
                if (p.pair0 && p.row_level[r] == 0) {
                    if (dtrack) T0 |= 1u << (c - cbase);
                } else {
                    Tr[r] |= 1u << (c - cbase);
                    Tl[p.row_level[r]] |= 1u << (c - cbase);
                }
            }
        cz.assign(L, 0);
        const uint64_t DW = DELTA >> c0;
        const unsigned evm = 1u << c0;  // Gray terms per walked step
        os << "// generated by libperm_mi355x: n=" << n << " nnz=" << p.nnz << " k=" << k << " c=" << p.c
           << " levels=" << L << " kappa=" << kappa << " u=" << u << " block=" << p.block
           << (p.pair0 ? " pair0" : "") << (horner ? " nested" : "") << (cm ? " copies=" + std::to_string(cm) : "")
           << "\n";
        os << "typedef unsigned long long u64;\n"
              "typedef unsigned int u32;\n"
              "struct dd { double h, l; };\n"
              "__device__ __forceinline__ dd two_sum(double a, double b) {\n"
              "  const double s = a + b; const double bb = s - a;\n"
              "  dd r; r.h = s; r.l = (a - (s - bb)) + (b - bb); return r; }\n"
              "__device__ __forceinline__ dd dd_add(dd x, dd y) {\n"
              "  const dd s = two_sum(x.h, y.h); const double e = s.l + (x.l + y.l);\n"
              "  dd r; r.h = s.h + e; r.l = e - (r.h - s.h); return r; }\n";
        // perm_lane: the Gray-term sum of chunk m (one lane's work); cold rows
        // of this lane live at xg[(r - k) * xs + lid].
        // `ev` counts the terms whose product this lane actually evaluates
        // (skipped ones excluded), for the device-work statistics.
        if (kw >= 1 && u + 1 <= kw - 1) build_dyn_table(u + 1 + c0, kappa - 1);
        // LDS tier: the cold rows of a workgroup's lanes, [row][lane], so a
        // wave's accesses to one row are 64 consecutive doubles
        if (p.cold_lds) os << "__shared__ double xl[" << (n - k) * p.block << "];\n";
        // Block queue: used where block pairs are pruned (zero-aware, u >= 1)
        // and their rows all live in VGPRs, within 40 KiB of LDS per workgroup;
        // at most 64 slots per wave, so the workgroup drains in one pass.
        {
            int bt = 0;
            for (int j = 0; j <= u && j < n - 1; ++j) bt = std::max(bt, p.col_top[j]);
            qtop = bt;
            qrows.clear();
            for (int r = 0; r < n; ++r)
                if (p.row_level[r] <= bt) qrows.push_back(r);
            // slots per wave: as given, or the most of 64, 32, 16, 8; the queue
            // may take 40 KiB of LDS per workgroup (four 256-lane workgroups
            // per CU): more slots beat the fifth wave that a 32 KiB cap keeps
            // (n = 36 0/1: 3.25 ms with 64 slots in 35 KiB against 3.51 ms with
            // 32 in 17 KiB; n = 40: 7.9 against 9.2 ms)
            auto fits = [&](int slots) { return (long)(p.block / 64) * qfields() * slots * 8 <= 40960; };
            qslots = 0;
            if (p.queue_slots > 0) {
                if (fits(p.queue_slots)) qslots = p.queue_slots;
            } else if (p.queue_slots == 0) {
                for (int slots : {64, 32, 16, 8})
                    if (fits(slots)) {
                        qslots = slots;
                        break;
                    }
            }
            use_queue = qslots > 0 && kappa >= 1 && u >= 1 && u + 1 <= kappa && p.zero_skip && !p.cold &&
                        bt + 1 <= L - 1;
        }
        const int QS = qslots;
        if (use_queue) {
            os << "__shared__ double bq[" << (p.block / 64) * qfields() * QS << "];\n";
            os << "__shared__ u32 bqn[" << p.block / 64 << "];\n";
        }
        os << "constexpr u32 kBlockQueueWords = " << (use_queue ? qfields() * QS : 1) << "u;\n";
        // block_eval: the 2^(u+1) - 1 steps of a queued block pair from its
        // start state it[field * QS] (rows of levels <= qtop, S_{qtop+1}, the
        // direction of the middle step), the same arithmetic as in place.
        os << "__device__ __forceinline__ dd block_eval(const double* __restrict__ it, u32 &ev, double* __restrict__ xo,\n"
              "                                         const double pmod, const double pinv) {\n";
        if (use_queue) {
            for (size_t i = 0; i < qrows.size(); ++i)
                os << "  double " << xname(qrows[i]) << " = it[" << i * QS << "];\n";
            os << "  double S" << qtop + 1 << " = it[" << qrows.size() * QS << "];\n";
            os << "  const double lsgn = it[" << (qrows.size() + 1) * QS << "];\n";
            if (p.exact) os << "  double R" << qtop + 1 << " = it[" << (qrows.size() + 2) * QS << "];\n";
            for (int l = qtop; l >= 1; --l) os << "  double S" << l << (p.exact ? ", R" + std::to_string(l) : "") << ";\n";
            {
                std::map<int, std::string> cur;
                for (int l = qtop; l >= 1; --l) refresh_level(l, cur, "  ");
            }
            os << "  double acc0 = 0.0, acc1 = 0.0;\n";
            if (p.exact) os << "  double racc = 0.0, accA = 0.0;\n";
            os << "  ev += " << (2 * U - 1) << "u;\n";
            static_block(false, "  ");
            step(u, Sign::Lane, 1, 0, "  ");
            static_block(true, "  ");
            if (p.exact) os << "  xo[0] += racc; xo[1] += accA;\n";
            else os << "  (void)xo; (void)pmod; (void)pinv;\n";
            os << "  return two_sum(acc0, acc1);\n";
        } else {
            os << "  (void)it; (void)ev; (void)xo; (void)pmod; (void)pinv;\n  dd r; r.h = 0.0; r.l = 0.0; return r;\n";
        }
        os << "}\n";
        // perm_lane: `act` is false for a lane past the last chunk (it queues
        // nothing); qw is this wave's queue region and qc its fill (uniform).
        // exact mode: xo receives the lane's residue of its term sum modulo
        // pmod and its sum |term| (the error bound's sum)
        os << "__device__ __forceinline__ dd perm_lane(const u64 m, double* __restrict__ xg, const u64 xs,\n"
              "                                        const u64 lid, const bool act, double* __restrict__ qw,\n"
              "                                        u32 &qc, u32 &ev, double* __restrict__ xo,\n"
              "                                        const double pmod, const double pinv) {\n";
        if (!p.exact) os << "  (void)xo; (void)pmod; (void)pinv;\n";
        if (!use_queue) os << "  (void)act; (void)qw; (void)qc;\n";
        os << "  ev = " << evm << "u;\n";
        os << "  const u64 g0 = m << "
           << kappa
           << ";\n"
              "  const u64 G = g0 ^ (g0 >> 1);\n";
        // ---- chunk start: x(Gray_{m 2^kappa}) ----
        for (int r = 0; r < n; ++r)
            os << "  double " << (r < k ? xname(r) : "cx" + std::to_string(r)) << " = " << lit(p.base_x_hi[r]) << ";\n";
        const int jlo = kappa >= 1 ? kappa - 1 : 0;  // lower Gray bits of an aligned start are zero
        // Bit j of the Gray code is bit j - kappa of m xor bit j - kappa + 1.
        // A wave's 64 chunks are consecutive and 64-aligned (every launch
        // starts at a multiple of the workgroup size), so from j = kappa + 6
        // on the bit is the same in all its lanes: read it once from the
        // first lane and add the column only when it is set (a lane past the
        // last chunk may then start from another chunk's x; it adds nothing).
        const int juni = kappa + 6;
        if (juni < n - 1)
            // (the builtin returns int: each half goes through u32, not sign-extended)
            os << "  const u64 Gw = ((u64)(u32)__builtin_amdgcn_readfirstlane((int)(u32)(G >> 32)) << 32) |\n"
                  "                 (u64)(u32)__builtin_amdgcn_readfirstlane((int)(u32)G);\n";
        for (int j = jlo; j < n - 1; ++j) {
            if (B.colptr[j + 1] == B.colptr[j]) continue;
            if (j >= juni)
                os << "  if ((Gw >> " << j << ") & 1ull) {\n";
            else
                os << "  { const double b = (double)((G >> " << j << ") & 1ull);\n";
            for (int q = B.colptr[j]; q < B.colptr[j + 1]; ++q) {
                const int r = B.rowidx[q];
                const std::string v = r < k ? xname(r) : "cx" + std::to_string(r);
                if (j >= juni)
                    os << "    " << v << " += " << lit(B.val[q]) << ";\n";
                else
                    os << "    " << v << " = fma(b, " << lit(B.val[q]) << ", " << v << ");\n";
            }
            os << "  }\n";
        }
        std::map<int, std::string> cur;
        for (int r = k; r < n; ++r) {
            os << "  " << cold_addr(r) << " = cx" << r << ";\n";
            cur[r] = "cx" + std::to_string(r);
        }
        if (cm) {
            // the copied columns are out of x at every chunk start; the other copies
            for (int r = 0; r < n; ++r)
                for (unsigned sgm : subsets(Tr[r])) {
                    if (!sgm) continue;
                    double add = 0.0;
                    for (int c = cbase; c < cbase + cm; ++c)
                        if (sgm & (1u << (c - cbase)))
                            for (int q = B.colptr[c]; q < B.colptr[c + 1]; ++q)
                                if (B.rowidx[q] == r) add += B.val[q];
                    os << "  double " << xv(r, sgm) << " = " << xname(r) << " + " << lit(add) << ";\n";
                }
        }
        for (int l = L - 1; l >= lv0; --l) {
            if (p.exact && !horner) {
                const std::vector<std::string> qs = part_products(l, cur, "  ");
                const std::string pl = product(qs, "  ");
                os << "  double S" << l << " = " << pl << (l + 1 < L ? " * S" + std::to_string(l + 1) : "") << ";\n";
                const std::string r = residue_chain(qs, 0, l + 1 < L ? "R" + std::to_string(l + 1) : "", "  ");
                os << "  double R" << l << " = " << r << ";\n";
                continue;
            }
            std::vector<std::string> v = level_values(l, cur, "  ");
            if (horner) {
                const std::string pr = product(v, "  ");
                os << "  double P" << l << " = " << pr << ";\n";
                if (hx) level_residue(l, 0u, cur, "  ", true);
                for (unsigned sgm : subsets(Tl[l])) {
                    if (!sgm) continue;
                    const std::string pi = product(level_values_in(l, sgm, cur, "  "), "  ");
                    os << "  double " << sub("P" + std::to_string(l), sgm) << " = " << pi << ";\n";
                    if (hx) level_residue(l, sgm, cur, "  ", true);
                }
                continue;
            }
            if (l + 1 < L) v.push_back("S" + std::to_string(l + 1));
            std::string prod = product(v, "  ");
            os << "  double S" << l << " = " << prod << ";\n";
        }
        os << "  double acc0 = 0.0, acc1 = 0.0;\n";
        if (p.exact) os << "  double racc = 0.0, accA = 0.0;\n";
        if (dtrack) {
            double cr, cs;
            bracket_coeffs(cr, cs);
            os << "  double dp = fma(" << lit(cs) << ", " << value_of(p.pair_s, cur, "  ") << ", fma(" << lit(cr) << ", "
               << value_of(p.pair_r, cur, "  ") << ", " << lit(cr * cs) << "));\n";
            for (unsigned sgm : subsets(T0)) {
                if (!sgm) continue;
                double add = 0.0;
                for (int c = cbase; c < cbase + cm; ++c)
                    if (sgm & (1u << (c - cbase))) add += bracket_delta(c);
                os << "  double " << sub("dp", sgm) << " = dp + " << lit(add) << ";\n";
            }
        }
        if (horner) {
            // every accumulator live and zero at the top of the loop
            os << "  double c0 = 0.0";
            for (int l = 1; l < L; ++l) os << ", c" << l << " = 0.0";
            os << ";\n";
            if (hx) {
                os << "  double a0 = 0.0, r0 = 0.0";
                for (int l = 1; l < L; ++l) os << ", a" << l << " = 0.0, r" << l << " = 0.0";
                os << ";\n";
            }
            std::fill(cz.begin(), cz.end(), 0);
        }
        acc_written = 0;
        accumulate(+1, 0, cur, "  ", nullptr, true);  // term g = m 2^kappa (even index: sign +)
        // ---- Gray loop over local steps 1 .. 2^kappa - 1 ----
        if (kappa >= 1) {
            os << "  const double lsgn = (m & 1ull) ? -1.0 : 1.0;  // direction at local step 2^(kappa-1)\n";
            // Zero-aware skipping (exact): a product with a factor that is
            // exactly 0 adds exactly 0.  Rows on levels above every level the
            // chunk's columns touch stay constant for the whole chunk; when
            // their cached product is 0 in all 64 lanes the wave skips the chunk.
            int chunk_top = 0;
            for (int j = 0; j < kappa; ++j) chunk_top = std::max(chunk_top, p.col_top[j]);
            rtop = chunk_top;
            const bool skip_chunk = p.zero_skip && chunk_top + 1 <= L - 1;
            if (skip_chunk) os << "  if (!__all(S" << chunk_top + 1 << " == 0.0)) {\n";
            // local step base + 2^u flips column u; its direction is bit u+1
            // of the local index (uniform), or the chunk parity when u+1 = kappa
            const int term_u = (u == 0) ? -1 : 1;
            // The same for one pair of static blocks (2^(u+1) - 1 steps touching
            // columns 0..u only): when the rows above those columns' levels
            // have a zero product in every lane, all those terms are 0 and the
            // blocks reduce to their net effect on x, one flip of column u.
            int block_top = 0;
            for (int j = 0; j <= u; ++j) block_top = std::max(block_top, p.col_top[j]);
            const bool skip_block = p.zero_skip && u >= 1 && block_top + 1 <= L - 1;
            lazy_r = p.exact && skip_block;
            // Larger intervals (zero-aware, exact): after position pos (a
            // multiple of 2^v, v >= u + 2) the next 2^v - 1 steps flip only
            // columns < v, so the rows on levels above those columns' levels
            // stay constant; when their product is 0 in every lane all those
            // terms are 0 and the interval reduces to one flip of column v - 1
            // (the Gray codes at pos and pos + 2^v - 1 differ in that bit only),
            // direction + when bit v of pos is 0.  Testing, at every position
            // reached, the largest such interval that starts there (then
            // smaller ones) visits the dyadic intervals of the chunk depth
            // first and prunes every all-zero one.  ptop(v) = highest level
            // columns < v touch grows with v, and S_l == 0 implies S_l' == 0
            // for l' < l, so the intervals are tried per distinct level.
            struct Group {
                int level, lo, hi;
            };
            std::vector<Group> groups;  // level descending
            if (p.zero_skip && u + 2 <= kappa - 1) {
                int pt = 0;
                for (int j = 0; j < u + 1; ++j) pt = std::max(pt, p.col_top[j]);
                std::vector<int> lev(kappa, 0);
                for (int v = u + 2; v <= kappa - 1; ++v) {
                    pt = std::max(pt, p.col_top[v - 1]);
                    lev[v] = pt + 1;
                }
                for (int v = kappa - 1; v >= u + 2; --v) {
                    if (lev[v] > L - 1) continue;
                    if (!groups.empty() && groups.back().level == lev[v])
                        groups.back().lo = v;
                    else
                        groups.push_back(Group{lev[v], v, v});
                }
            }
            const bool tree = !groups.empty();
            auto block_pair = [&](const char *posv, const char *ind) {
                std::string in2 = std::string(ind) + "  ";
                if (skip_block) {
                    if (use_queue) {
                        // lanes that need this block queue its start state and
                        // skip it like the rest; a full queue evaluates in place
                        const std::string in3 = in2 + "  ";
                        os << ind << "const bool need = act && (S" << block_top + 1 << " != 0.0);\n";
                        os << ind << "const u64 bal = __ballot(need);\n";
                        os << ind << "const u32 nk = (u32)__popcll(bal);\n";
                        os << ind << "if (nk == 0u || qc + nk <= " << QS << "u) {\n";
                        if (lazy_r) {
                            // the queued start state carries the residue of the
                            // rows above the block's levels
                            std::map<int, std::string> rc;
                            os << in2 << "if (nk != 0u) {\n";
                            recompute_residues(block_top + 1, rc, (in2 + "  ").c_str());
                            os << in2 << "}\n";
                        }
                        os << in2 << "if (need) {\n";
                        os << in3 << "const u32 sl = qc + __builtin_amdgcn_mbcnt_hi((u32)(bal >> 32), "
                                     "__builtin_amdgcn_mbcnt_lo((u32)bal, 0u));\n";
                        for (size_t i = 0; i < qrows.size(); ++i)
                            os << in3 << "qw[" << i * QS << "u + sl] = " << xname(qrows[i]) << ";\n";
                        os << in3 << "qw[" << qrows.size() * QS << "u + sl] = S" << block_top + 1 << ";\n";
                        if (p.exact)
                            os << in3 << "qw[" << (qrows.size() + 2) * QS << "u + sl] = R" << block_top + 1 << ";\n";
                        os << in3 << "qw[" << (qrows.size() + 1) * QS << "u + sl] = ";
                        if (u + 1 == kappa)
                            os << "lsgn;\n";
                        else
                            os << "((" << posv << " >> " << (u + 1) << ") & 1u) ? -1.0 : 1.0;\n";
                        os << in2 << "}\n";
                        os << in2 << "qc += nk;\n";
                    } else {
                        os << ind << "if (__all(S" << block_top + 1 << " == 0.0)) {\n";
                    }
                    std::map<int, std::string> cur;
                    walk_s_only = lazy_r;
                    if (u + 1 == kappa) {
                        update(u, Sign::Lane, cur, in2.c_str());
                    } else {
                        os << in2 << "const bool neg = (" << posv << " >> " << (u + 1) << ") & 1u;\n";
                        update(u, Sign::Uniform, cur, in2.c_str());
                    }
                    for (int l = block_top; l >= 1; --l) refresh_level(l, cur, in2.c_str());
                    walk_s_only = false;
                    os << ind << "} else {\n";
                }
                const char *bi = skip_block ? in2.c_str() : ind;
                if (lazy_r) {
                    // evaluated in place: the residues of every level from x
                    std::map<int, std::string> rc;
                    recompute_residues(1, rc, bi);
                }
                os << bi << "ev += " << evm * (2 * U - 1) << "u;\n";
                static_block(false, bi);
                if (u + 1 == kw) {
                    step(u + c0, Sign::Lane, term_u, 0, bi);
                } else {
                    os << bi << "{\n" << bi << "  const bool neg = (" << posv << " >> " << (u + 1) << ") & 1u;\n";
                    varies("neg");
                    step(u + c0, Sign::Uniform, term_u, 0, (std::string(bi) + "  ").c_str());
                    os << bi << "}\n";
                }
                static_block(true, bi);
                if (U == 1) reduce_racc(bi);
                if (skip_block) os << ind << "}\n";
            };
            // local step ell (a multiple of 2^(u+1)): column jj = ctz(ell) >= u + 1,
            // the same in every lane, flipped branch-free with its entries read
            // from the constant table, then every level these columns can reach
            // is refreshed.  At ell = 2^kappa (not a step of this chunk) the
            // table row is zero and the weight w = 0 drops the term.  (A branch there instead makes the
            // compiler restructure the loop at a large cost in registers.)
            auto dynamic_step = [&](const char *ellv, const char *ind) {
                std::string in2 = std::string(ind) + "  ";
                const char *I2 = in2.c_str();
                os << ind << "{\n";
                os << I2 << "const double w = (" << ellv << " < " << DW << "u) ? 1.0 : 0.0;\n";
                os << I2 << "const int jr = __builtin_ctz(" << ellv << ");\n";
                os << I2 << "const int jj = jr + " << c0 << ";\n";
                os << I2 << "const double sgu = ((" << ellv << " >> (jr + 1)) & 1u) ? -1.0 : 1.0;\n";
                os << I2 << "const double sg = (jj == " << kappa - 1 << ") ? lsgn : sgu;\n";
                varies("w");
                varies("sg");
                std::map<int, std::string> cur;
                walk_s_only = lazy_r;
                if (horner) flush_to(loop_top, I2);
                const int top_max = dyn_flip("jj", "sg", cur, I2);
                for (int l = top_max; l >= lv0; --l) refresh_level(l, cur, I2);
                accumulate(1, 1, cur, I2, "w", horner && loop_top >= 1);
                walk_s_only = false;
                os << ind << "}\n";
            };
            if (!tree) {
                if (horner && u + 1 <= kw - 1) {
                    // the accumulators empty at the loop's top (and at its end)
                    loop_top = 0;
                    for (int j = dyn_lo; j <= dyn_hi; ++j) loop_top = std::max(loop_top, p.col_top[j]);
                    for (int j = c0; j <= u + c0; ++j) loop_top = std::max(loop_top, p.col_top[j]);
                    for (int l = 1; l < loop_top; ++l) cz[l] = 1;
                }
                if (hx) settle_residues("  ");  // the same state at every iteration's top
                os << "#pragma clang loop unroll(disable)\n";
                os << "  for (u32 base = 0; base < " << DW << "u; base += " << 2 * U << "u) {\n";
                auto body = [&]() {
                    block_pair("base", "    ");
                    if (u + 1 <= kw - 1) {
                        os << "    const u32 ell = base + " << 2 * U << "u;\n";
                        dynamic_step("ell", "    ");
                    }
                    if (hx) settle_residues("    ");
                };
                if (horner) {
                    // count the body's operations: a first pass finds the
                    // names it assigns (they vary at the loop's top), the
                    // second emits it and counts
                    const std::string before = os.str();
                    const int tmp0 = tmp;
                    const std::vector<char> cz0 = cz;
                    const unsigned ts0 = ts;
                    const std::vector<char> dirty0 = dirty;
                    const std::vector<int> rdef0 = rdef;
                    const long acc0_written = acc_written;
                    track = true;
                    vid.clear();
                    interned.clear();
                    unit.clear();
                    assigned.clear();
                    body();
                    os.str(before);
                    os.clear();
                    os.seekp(0, std::ios_base::end);
                    tmp = tmp0;
                    cz = cz0;
                    ts = ts0;
                    dirty = dirty0;
                    rdef = rdef0;
                    acc_written = acc0_written;
                    vid.clear();
                    unit.clear();
                    for (const std::string &a : assigned) vid[a] = {intern("phi:" + a), true};
                    seen.clear();
                    cnt_ops = cnt_flops = hoist_ops = hoist_flops = 0;
                    counting = true;
                    all_vary = DW == (uint64_t)(2 * U);  // one pass: nothing to hoist
                    body();
                    body_acc = acc_written - acc0_written;
                    counting = track = all_vary = false;
                    const double terms = (double)(2 * U) * evm;
                    loop_terms = terms;
                    loop_iters = DW / (uint64_t)(2 * U);
                    // per Gray term of a chunk: the body every iteration, the
                    // hoisted operations once
                    const double it = (double)loop_iters;
                    loop_ops = (cnt_ops * it + hoist_ops) / (terms * it);
                    loop_flops = (cnt_flops * it + hoist_flops) / (terms * it);
                } else {
                    body();
                }
                if (ts != 0u) os << "#error copies of x not restored by the loop\n";
                os << "  }\n";
                os << "  ev += " << evm * (DW / (2 * U) - 1) << "u;  // the dynamic steps\n";
            } else {
                // pos: the local index whose term was added last (a multiple of 2^(u+1))
                os << "  u32 pos = 0u;\n";
                os << "#pragma clang loop unroll(disable)\n";
                os << "  do {\n";
                os << "    u32 vs = 0u;\n";
                os << "    {\n";
                os << "      const u32 v = (pos == 0u) ? " << kappa - 1 << "u : (u32)__builtin_ctz(pos);\n";
                for (size_t gi = 0; gi < groups.size(); ++gi) {
                    const Group &g = groups[gi];
                    os << "      " << (gi ? "else " : "") << "if (v >= " << g.lo << "u && __all(S" << g.level
                       << " == 0.0)) vs = (v < " << g.hi << "u) ? v : " << g.hi << "u;\n";
                }
                os << "    }\n";
                // vs is the same in every lane; saying so keeps pos and what
                // depends on it in scalar registers
                os << "    vs = __builtin_amdgcn_readfirstlane(vs);\n";
                os << "    if (vs == 0u) {\n";
                block_pair("pos", "      ");
                os << "    }\n";
                // net flip of a skipped interval (column vs - 1), its entries
                // read from the constant table.  (With entries chosen by scalar
                // selects, a branch here made the compiler keep two copies of x;
                // with the table it does not, and skipping the FMAs when nothing
                // was pruned measured 2-6 % faster.)  The cached products are
                // refreshed by the dynamic step that follows.
                os << "    if (vs != 0u) {\n";
                os << "      const u32 jn = vs - 1u;\n";
                os << "      const double sn = ((pos >> vs) & 1u) ? -1.0 : 1.0;\n";
                {
                    std::map<int, std::string> cur;
                    dyn_flip("jn", "sn", cur, "      ");
                }
                os << "    }\n";
                os << "    pos += (vs == 0u) ? " << 2 * U << "u : (1u << vs);\n";
                dynamic_step("pos", "    ");
                os << "    ev += (pos < " << DELTA << "u) ? 1u : 0u;\n";
                os << "  } while (pos < " << DELTA << "u);\n";
            }
            if (skip_chunk) os << "  }\n";
        }
        if (horner) {
            // everything up to the top level: c_{L-1} is the chunk's sum
            flush_to(L - 1, "  ");
            if (hx) settle_residues("  ");
            os << "  acc0 = c" << L - 1 << ";\n";
            if (hx) os << "  racc = r" << L - 1 << "; accA = a" << L - 1 << ";\n";
            acc_chunk = (double)acc_written + (double)body_acc * ((double)std::max<uint64_t>(loop_iters, 1) - 1.0);
        }
        if (p.exact) {
            reduce_racc("  ");
            os << "  xo[0] = racc; xo[1] = accA;\n";
        }
        os << "  return two_sum(acc0, acc1);\n}\n";
        // ---- the kernel: one chunk per lane, then a deterministic reduction
        //      lane -> wave (butterfly) -> workgroup ----
        const int nw = p.block / 64;
        os << "extern \"C\" __global__ void __launch_bounds__(" << p.block << ") ";
        if (p.waves_per_simd > 0) os << "__attribute__((amdgpu_waves_per_eu(" << p.waves_per_simd << "))) ";
        os << kGrayKernelName
           << "(const u64 chunk_begin, const u64 chunk_end, double* __restrict__ partials,\n"
              "    u64* __restrict__ counts, double* __restrict__ xg, const u64 xs,\n"
              "    double* __restrict__ xparts, const double pmod, const double pinv) {\n";
        if (!p.exact) os << "  (void)xparts;\n";
        os << "  const u64 lid = (u64)blockIdx.x * " << p.block << "u + threadIdx.x;\n"
              "  const bool active = chunk_begin + lid < chunk_end;\n"
              "  // an inactive lane (past the last chunk) replays a valid chunk and contributes 0\n"
              "  const u64 m = active ? chunk_begin + lid : chunk_begin;\n"
              "  const u32 wid = threadIdx.x >> 6;\n"
              "  u32 ev = 0u, qc = 0u;\n";
        if (use_queue)
            os << "  double* qw = bq + wid * " << qfields() * QS << "u;\n";
        else
            os << "  double* qw = nullptr;\n";
        os << "  double xo[2] = {0.0, 0.0};\n"
              "  dd cs = perm_lane(m, xg, xs, lid, active, qw, qc, ev, xo, pmod, pinv);\n"
              "  if (!active) { cs.h = 0.0; cs.l = 0.0; xo[0] = 0.0; xo[1] = 0.0; }\n";
        if (use_queue) {
            // the workgroup's queued blocks, item g (waves in order, then
            // slots) evaluated by thread g: at most 64 per wave, so one pass
            os << "  if ((threadIdx.x & 63u) == 0u) bqn[wid] = qc;\n"
                  "  __syncthreads();\n"
                  "  {\n"
                  "    u32 total = 0u;\n"
                  "    for (int w = 0; w < " << nw << "; ++w) total += bqn[w];\n"
                  "    const u32 g = threadIdx.x;\n"
                  "    if (g < total) {\n"
                  "      u32 ww = 0u, b0 = 0u;\n"
                  "      while (g >= b0 + bqn[ww]) { b0 += bqn[ww]; ++ww; }\n"
                  "      cs = dd_add(cs, block_eval(bq + ww * " << qfields() * QS << "u + (g - b0), ev, xo, pmod, pinv));\n"
                  "    }\n"
                  "  }\n";
        }
        os << "  u64 e64 = ev;  // terms this lane evaluated\n"
              "  for (int off = 32; off > 0; off >>= 1) {\n"
              "    dd o; o.h = __shfl_xor(cs.h, off, 64); o.l = __shfl_xor(cs.l, off, 64);\n"
              "    cs = dd_add(cs, o);\n"
              "    e64 += __shfl_xor(e64, off, 64);\n"
              "  }\n";
        if (p.exact) {
            // residues: each lane's back in (-p/2 - 2, p/2 + 2), then exact sums
            // (64 lanes, then the waves: below 2^34); A: a plain sum
            os << "  double xr = fma(-rint(xo[0] * pinv), pmod, xo[0]), xa = xo[1];\n"
                  "  for (int off = 32; off > 0; off >>= 1) {\n"
                  "    xr += __shfl_xor(xr, off, 64); xa += __shfl_xor(xa, off, 64);\n"
                  "  }\n";
            os << "  __shared__ double wx[" << 2 * nw << "];\n"
                  "  if ((threadIdx.x & 63u) == 0) { wx[2 * wid] = xr; wx[2 * wid + 1] = xa; }\n";
        }
        os << "  __shared__ double wsum[" << 2 * nw << "];\n"
              "  __shared__ u64 wev[" << nw << "];\n"
              "  if ((threadIdx.x & 63u) == 0) { wsum[2 * wid] = cs.h; wsum[2 * wid + 1] = cs.l; wev[wid] = e64; }\n"
              "  __syncthreads();\n"
              "  if (threadIdx.x == 0) {\n"
              "    dd t; t.h = wsum[0]; t.l = wsum[1];\n";
        os << "    for (int w = 1; w < " << nw << "; ++w) { dd o; o.h = wsum[2 * w]; o.l = wsum[2 * w + 1]; t = dd_add(t, o); }\n";
        os << "    u64 te = 0;\n    for (int w = 0; w < " << nw << "; ++w) te += wev[w];  // lane-terms\n";
        os << "    counts[blockIdx.x] = te;\n";
        os << "    partials[2 * (u64)blockIdx.x] = t.h;\n"
              "    partials[2 * (u64)blockIdx.x + 1] = t.l;\n";
        if (p.exact)
            os << "    double r = 0.0, a = 0.0;\n"
                  "    for (int w = 0; w < " << nw << "; ++w) { r += wx[2 * w]; a += wx[2 * w + 1]; }\n"
                  "    xparts[2 * (u64)blockIdx.x] = fma(-rint(r * pinv), pmod, r);\n"
                  "    xparts[2 * (u64)blockIdx.x + 1] = a;\n";
        os << "  }\n"
              "}\n";
        return os.str();
    }
};

}  // namespace

std::string generate_source(const Plan &p, LoopCount *lc) {
    Gen g(p);
    std::string src = g.run();
    if (lc) {
        lc->counted = g.loop_ops >= 0;
        lc->ops_per_step = g.loop_ops;
        lc->flops_per_step = g.loop_flops;
        lc->loop = g.loop_iters > 1;
        lc->iters = g.loop_iters;
        lc->body_ops = g.cnt_ops;
        lc->terms_per_iter = g.loop_terms;
        lc->sign_fmas = g.sign_fmas;
        int cv = 0;
        for (int r = 0; r < p.n && g.cm; ++r) cv += (1 << __builtin_popcount(g.Tr[r])) - 1;
        for (int l = 1; l < p.nlevels && g.cm; ++l)
            if (g.level_rows[l].size() > 1) cv += (1 << __builtin_popcount(g.Tl[l])) - 1;
        if (g.cm) cv += (1 << __builtin_popcount(g.T0)) - 1;
        lc->copy_values = cv;
        int al = 0;
        while (std::ldexp(1.0, al) < g.acc_chunk + p.n + 2) ++al;
        lc->acc_log2 = al;
    }
    return src;
}

}  // namespace permx
