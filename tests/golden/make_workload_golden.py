"""Write oracle values for sampled matrices of the batch and serving workloads.

Calls only the CPU oracle (oracle/) on inputs from the seeded generators, and
records each result with its provenance.  The sample is chosen here, from the
generators and the oracle's structural rank alone:

* batch (2000 matrices, seed 1): the first 8 structurally nonsingular
  matrices of each size class n = 23..24, 25..28, 29..30 (4-row groups 6, 7
  and 8 of the batch kernels), U(-1, 1) values: long double Alg. 1;
* serving (seed 1): structurally nonsingular requests with n >= 23: the first
  two 0/1 requests of every n = 23..36 (exact integer oracle), the first real
  request of every n = 23..32 and of n = 33 and 36 (long double Alg. 1), and
  the 0/1 requests with n <= 28 among the first 400 whose FP64 rounding bound
  (2n + 2) 2^-53 A exceeds 1/2 (A from the long double oracle).

Usage:  python tests/golden/make_workload_golden.py [batch|serving|all]
Writes tests/golden/workload_samples.json (merged with what is there).
"""
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2501_15126_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workload_samples.json")
SEED = 1


def _src_hash():
    with open(os.path.join(ROOT, "oracle", "perm_oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _nonsingular(ccs):
    return O.structural_rank(ccs) == ccs[0]


def batch_sample():
    classes = {6: [], 7: [], 8: []}
    for i in range(2000):
        m = W.batch_matrix(SEED, i)
        n = m[0]
        if n < 23 or not _nonsingular(m):
            continue
        ng = (n + 3) // 4
        if len(classes[ng]) < 8:
            classes[ng].append(i)
        if all(len(v) == 8 for v in classes.values()):
            break
    return [("batch", i) for ng in (6, 7, 8) for i in classes[ng]]


def serving_sample():
    want01 = {n: 2 for n in range(23, 37)}
    wantr = {n: 1 for n in list(range(23, 33)) + [33, 36]}
    picked = []
    for i in range(4000):
        r = W.serving_request(SEED, i)
        n = r[0]
        if n < 23 or not _nonsingular(r):
            continue
        binary = bool((r[3] == 1.0).all())
        want = want01 if binary else wantr
        if want.get(n, 0) > 0:
            want[n] -= 1
            picked.append(("serving", i))
        if not any(want01.values()) and not any(wantr.values()):
            break
    # 0/1 requests whose FP64 rounding bound exceeds 1/2 (cancellation-heavy)
    for i in range(400):
        r = W.serving_request(SEED, i)
        n = r[0]
        if not (20 <= n <= 28) or not (r[3] == 1.0).all() or not _nonsingular(r):
            continue
        _, a = O.perm_nw(r)
        if (2 * n + 2) * 2.0 ** -53 * a > 0.5 and ("serving", i) not in picked:
            picked.append(("serving", i))
    return picked


def record(kind, i, threads):
    ccs = W.batch_matrix(SEED, i) if kind == "batch" else W.serving_request(SEED, i)
    n = ccs[0]
    rec = {"workload": kind, "seed": SEED, "index": i, "n": n, "nnz": int(len(ccs[2])),
           "oracle_src": _src_hash(), "threads": threads, "host": platform.node(),
           "cpu": platform.processor() or platform.machine()}
    binary = bool((ccs[3] == 1.0).all())
    t0 = time.time()
    if binary:
        rec["kind"] = "01"
        rec["perm_exact"] = str(O.perm_int(ccs, threads))
        rec["seconds_int"] = round(time.time() - t0, 1)
    else:
        rec["kind"] = "real"
    if not binary or n <= 30:
        t1 = time.time()
        (h, l), (ah, al) = O.nw_range(ccs, 0, 1 << (n - 1), threads)
        f = 4 * (n % 2) - 2
        rec["perm_ld_hi"] = h * f
        rec["perm_ld_lo"] = l * f
        rec["abs_sum"] = 2 * (ah + al)
        rec["seconds_ld"] = round(time.time() - t1, 1)
    return "%s:%d:%d" % (kind, SEED, i), rec


def main(argv):
    which = argv[0] if argv else "all"
    threads = int(os.environ.get("ORACLE_THREADS", O.default_threads()))
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    todo = []
    if which in ("batch", "all"):
        todo += batch_sample()
    if which in ("serving", "all"):
        todo += serving_sample()
    # cheapest first, so an interrupted run keeps the most
    def cost(t):
        ccs = W.batch_matrix(SEED, t[1]) if t[0] == "batch" else W.serving_request(SEED, t[1])
        return ccs[0]
    todo.sort(key=cost)
    print("sample:", todo, flush=True)
    for kind, i in todo:
        key = "%s:%d:%d" % (kind, SEED, i)
        if key in data and data[key].get("oracle_src") == _src_hash():
            continue
        key, rec = record(kind, i, threads)
        data[key] = rec
        print(json.dumps(rec), flush=True)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:])
