"""Write the stored expected values for the full-size workloads.

Calls only the CPU oracle (oracle/) on inputs from the seeded generators and
records each result with its provenance (oracle source hash, threads, seconds,
host).  Usage:

    python tests/golden/make_golden.py n24_p0.15_01:1 n36_p0.30_real:1 n40_p0.10_01:1

Each argument is ``<workload>:<seed>``.  0/1 workloads are evaluated with the
exact integer oracle (and the long double oracle too when cheap); real
workloads with the long double oracle.
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")


def _src_hash():
    with open(os.path.join(ROOT, "oracle", "perm_oracle.c"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def main(argv):
    threads = int(os.environ.get("ORACLE_THREADS", O.default_threads()))
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for arg in argv:
        name, seed = arg.split(":")
        seed = int(seed)
        ccs = W.WORKLOADS[name](seed)
        n = ccs[0]
        rec = {"workload": name, "seed": seed, "n": n, "nnz": int(len(ccs[2])),
               "oracle_src": _src_hash(), "threads": threads, "host": platform.node(),
               "cpu": platform.processor() or platform.machine()}
        binary = bool((ccs[3] == 1.0).all())
        t0 = time.time()
        if binary:
            rec["perm_exact"] = str(O.perm_int(ccs, threads))
            rec["kind"] = "01"
            rec["seconds_int"] = round(time.time() - t0, 1)
            if n <= 30:
                t1 = time.time()
                v, a = O.perm_nw(ccs, threads)
                rec["perm_ld"] = v
                rec["abs_sum"] = a
                rec["seconds_ld"] = round(time.time() - t1, 1)
        else:
            (h, l), (ah, al) = O.nw_range(ccs, 0, 1 << (n - 1), threads)
            f = 4 * (n % 2) - 2
            rec["perm_ld_hi"] = h * f
            rec["perm_ld_lo"] = l * f
            rec["abs_sum"] = 2 * (ah + al)
            rec["kind"] = "real"
            rec["seconds_ld"] = round(time.time() - t0, 1)
        data["%s:%d" % (name, seed)] = rec
        print(json.dumps(rec), flush=True)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:])
