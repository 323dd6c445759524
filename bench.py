"""Benchmark: Gray-code steps/s of the sparse permanent on one MI355X.

One benchmark step = one full permanent of the n=40, density-0.10 0/1 matrix
(random permutation pattern OR Bernoulli(0.10), seed 1) with every one of its
2^39 Gray-code terms evaluated (Alg. 1 as the paper's generated kernels run
it), through the C ABI (validation, structural check, ordering, partition,
code generation with a cached code object, launches, fixed-order reduction,
the exact integer count on the host).  Beside it: the same permanent with
exact zero-aware pruning (permanents/s), the 2000-matrix batch, the serving
run, and the CPU oracle.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--mode auto]
                    [--workload n40_p0.10_01] [--seed 1] [--no-cpu-baseline]

The dominant kernel's achieved FP64 rate is computed from the library's HIP
events (recorded on the launch stream around the Gray-kernel launches of each
call) and the generated code's FP64 operations per step.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gray-code steps/s & % FP64 peak (n=40); batched permanents/s; p50/p99 latency"
FP64_PEAK_TFLOPS = 78.6  # MI355X published FP64 vector peak (an FMA counts 2)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(ccs, seconds_target=20.0, one_core_seconds=6.0, int_seconds=8.0):
    """The oracle on bounded samples of the same matrix's Gray-index range:
    Alg. 1 in long double with every term evaluated (like the headline), on
    all host threads and on one; and the exact integer form with zero
    skipping (products with a zero factor skipped, as the pruned GPU path
    does), on all host threads.  Rates in Gray-code steps/s."""
    from oracle import oracle as O
    O.build(force=False)
    threads = O.default_threads()
    n = ccs[0]
    total = 1 << (n - 1)

    def timed(fn, target, nthreads):
        probe = min(total, 1 << 20)
        t0 = time.perf_counter()
        fn(0, probe, nthreads)
        dt = max(time.perf_counter() - t0, 1e-3)
        steps = int(min(total, max(probe, probe * target / dt)))
        t0 = time.perf_counter()
        fn(0, steps, nthreads)
        return steps, time.perf_counter() - t0

    s_all, t_all = timed(lambda b, e, t: O.nw_range(ccs, b, e, t), seconds_target, threads)
    s_one, t_one = timed(lambda b, e, t: O.nw_range(ccs, b, e, t), one_core_seconds, 1)
    out = {"value": s_all / t_all, "unit": "Gray-code steps/s", "cores": threads, "kind": "oracle",
           "sample": "Gray indices [0, %d) = 2^%.2f of the same matrix (of 2^%d), long double Alg. 1, every term "
                     "evaluated, %.1f s" % (s_all, math.log2(s_all), n - 1, t_all),
           "one_core": {"value": s_one / t_one, "sample": "Gray indices [0, %d), %.1f s" % (s_one, t_one)},
           "cpu_model": _cpu_model(), "host_threads": os.cpu_count()}
    if (ccs[3] == 1.0).all():
        s_int, t_int = timed(lambda b, e, t: O.nw_int_range(ccs, b, e, t), int_seconds, threads)
        out["zero_skipping_int"] = {
            "value": s_int / t_int, "unit": "Gray-code steps/s (terms with a zero factor skipped)",
            "cores": threads, "kind": "oracle",
            "sample": "Gray indices [0, %d) = 2^%.2f, exact integer Alg. 1, %.1f s" % (s_int, math.log2(s_int), t_int)}
    return out


def batch_bench(seed=1, count=2000, reps=3, sequential=True, opts=None):
    """The batch workload (2000 matrices, n ~ U{16..30}, density ~ U[0.15, 0.40],
    U(-1,1) values), host preparation included: perm_batch with one wave per
    work item, each kernel instance on its class stream, against one matrix
    per launch, synchronised after each, with the same kernels.  `opts`
    (perm_batch keywords, e.g. from perm_batch_autotune) apply to both."""
    import paper_2501_15126_amd.perm as P
    from paper_2501_15126_amd import workloads as W
    mats = W.batch(seed, count)
    opts = dict(opts or {})
    opts.pop("batch_mode", None)

    def best_of(mode):
        P.perm_batch(mats, batch_mode=mode, **opts)  # warm-up: device buffers
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            out, st = P.perm_batch_ex(mats, batch_mode=mode, **opts)
            dt = time.perf_counter() - t0
            best = (dt, st, out) if best is None or dt < best[0] else best
        return best

    dt, st, out = best_of("streams")

    def roof(st):
        ks = st["kernel_ms"] / 1e3
        return {"bound": "alu", "achieved": st["flops"] / ks / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": st["flops"] / ks / 1e12 / FP64_PEAK_TFLOPS, "fp64_ops": st["fp64_ops"],
                "fp64_issue_frac": st["fp64_ops"] / ks / 3.93216e13}

    res = {"workload": "%d sparse real matrices, n ~ U{16..30}, density ~ U[0.15,0.40], U(-1,1), seed %d"
                       % (count, seed),
           "permanents_per_s": count / dt, "wall_ms": dt * 1e3, "kernel_ms": st["kernel_ms"],
           "form": "one launch per kernel instance, instances on class streams",
           "options": opts,
           "prep_ms": st["prep_ms"], "gray_steps": st["steps"], "gray_steps_per_s": st["steps"] / dt,
           "structurally_singular": st["singular"],
           # the batch kernels' own FP64 work (counted exactly per chunk from
           # their code) over the device time of the launches
           "roofline": roof(st)}
    if sequential:
        t0 = time.perf_counter()
        out_seq, st_seq = P.perm_batch_ex(mats, batch_mode="sequential", **opts)
        dt_seq = time.perf_counter() - t0
        res.update({"sequential_permanents_per_s": count / dt_seq, "sequential_wall_ms": dt_seq * 1e3,
                    "speedup_vs_sequential": dt_seq / dt,
                    "bitwise_equal_to_sequential": bool(np.array_equal(out, out_seq))})
    return res


def serving_bench(duration_s=60.0, rate_hz=200.0, seed=1, compare_fifo=True, round_steps=0.0):
    """Poisson arrivals at rate_hz of requests with n ~ U{12..36}, density ~
    U[0.10,0.35], 70 % 0/1 else U(0,1).  Latency = time the result is seen by
    the client minus the scheduled arrival time (queueing included)."""
    import threading
    import paper_2501_15126_amd.perm as P
    from paper_2501_15126_amd import workloads as W
    arrivals = W.serving_trace(seed, rate_hz, duration_s)
    reqs = [W.serving_request(seed, i) for i in range(len(arrivals))]
    steps = sum(2.0 ** (r[0] - 1) for r in reqs)

    def run_server():
        srv = P.Server(round_steps=round_steps)
        srv.wait(srv.submit(reqs[0]))  # warm-up
        tickets = [None] * len(reqs)
        done = [None] * len(reqs)
        t0 = time.perf_counter() + 0.05

        def submitter():
            for i, a in enumerate(arrivals):
                d = t0 + a - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(reqs[i])

        th = threading.Thread(target=submitter)
        th.start()
        pending = set()
        nxt = 0
        while nxt < len(reqs) or pending:
            while nxt < len(reqs) and tickets[nxt] is not None:
                pending.add(nxt)
                nxt += 1
            now = time.perf_counter()
            for i in list(pending):
                if srv.poll(tickets[i]) is not None:
                    done[i] = now
                    pending.discard(i)
            time.sleep(0.0002)
        th.join()
        st = srv.stats()
        srv.close()
        lat = np.array([done[i] - (t0 + arrivals[i]) for i in range(len(reqs))]) * 1e3
        span = max(done) - t0
        return lat, span, st

    def run_fifo():
        # the sequential baseline: one request at a time, in arrival order
        t0 = time.perf_counter() + 0.05
        done = []
        for i, a in enumerate(arrivals):
            d = t0 + a - time.perf_counter()
            if d > 0:
                time.sleep(d)
            P.perm_batch([reqs[i]], batch_mode="sequential")
            done.append(time.perf_counter())
        lat = np.array([done[i] - (t0 + arrivals[i]) for i in range(len(reqs))]) * 1e3
        return lat, done[-1] - t0

    lat, span, st = run_server()
    print("bench: server run done (%d requests), sequential baseline next" % len(reqs), file=sys.stderr, flush=True)
    out = {"workload": "Poisson %.0f req/s for %.0f s, n ~ U{12..36}, density ~ U[0.10,0.35], 70%% 0/1 else U(0,1), "
                       "seed %d" % (rate_hz, duration_s, seed),
           "requests": len(reqs), "offered_gray_steps_per_s": steps / duration_s,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
           "permanents_per_s": len(reqs) / span, "rounds": st["rounds"], "arena_peak_bytes": st["arena_peak"],
           "server_busy_fraction": st["busy_ms"] / 1e3 / span,
           "exact_certified": st["exact_certified"], "exact_uncertified": st["exact_uncertified"],
           "exact_extra_passes": st["extra_passes"]}
    if compare_fifo:
        flat, fspan = run_fifo()
        out["fifo_sequential"] = {"p50_ms": float(np.percentile(flat, 50)), "p99_ms": float(np.percentile(flat, 99)),
                                  "permanents_per_s": len(reqs) / fspan}
    return out


# The paper's Table 3 (A100, seconds per permanent), for context only: another
# machine, another code base.  Keys (n, 10 p).
PAPER_TABLE3_CODEGEN_HYBRID = {
    (40, 1): 3.18, (40, 2): 3.94, (40, 3): 4.77, (40, 4): 5.96, (40, 5): 6.51,
    (45, 1): 92.06, (45, 2): 93.69, (45, 3): 155.28, (45, 4): 196.25, (45, 5): 251.07,
    (48, 1): 741.59, (48, 2): 1059.77, (48, 3): 1361.69, (48, 4): 1906.64, (48, 5): 2023.94}


def er_grid_bench(ns, variants, seed=1, ps=None):
    """The paper's synthetic grid: one permanent per cell and kernel variant.
    The code is matrix-specific, so each call includes its hipRTC compile;
    the kernel time (HIP events) and the compile time are reported apart.
    Variant "tuned" runs perm_autotune first (its search time is reported as
    tune_s) and then the permanent with the options it returns."""
    import paper_2501_15126_amd.perm as P
    from paper_2501_15126_amd import workloads as W
    rows = []
    for n, p in W.ER_GRID:
        if n not in ns or (ps and int(round(10 * p)) not in ps):
            continue
        ccs = W.er_grid_matrix(n, p, seed)
        for var in variants:
            tune = None
            if var == "tuned":
                opts, tune = P.perm_autotune(ccs)
                print("grid cell n=%d p=%.1f tuned in %.1f s: %s" % (n, p, tune["tune_ms"] / 1e3, {
                    k: opts[k] for k in ("mode", "cold_tier", "chunk_log2", "unroll_log2", "block",
                                         "waves_per_simd")}), file=sys.stderr, flush=True)
            else:
                mode, tier = {"auto": ("auto", "global"), "hybrid": ("hybrid", "global"),
                              "hybrid-lds": ("hybrid", "lds")}[var]
                opts = {"mode": mode, "cold_tier": tier}
            t0 = time.perf_counter()
            v, st = P.perm_sparse_ex(ccs, progress=n >= 45, **opts)
            wall = time.perf_counter() - t0
            steps = 2.0 ** (n - 1)
            ks = st["kernel_ms"] / 1e3
            row = {"n": n, "p": p, "variant": var, "nnz": len(ccs[2]), "permanent": v, "kernel_s": ks,
                   "wall_s": wall, "compile_s": st["compile_ms"] / 1e3, "steps_per_s": steps / ks,
                   "fp64_ops_per_step": st["ops_per_step"],
                   "fp64_issue_frac": st["ops_per_step"] * steps / ks / 3.93216e13,
                   "tflops": st["flops_per_step"] * steps / ks / 1e12, "vgprs": st["vgprs"],
                   "waves_per_simd": st["waves_per_simd"], "lds_bytes": st["lds_bytes"], "k": st["k"],
                   "levels": st["levels"], "chunk_log2": st["chunk_log2"], "unroll_log2": st["unroll_log2"],
                   "block": st["block"], "waves_hint": st["waves_hint"],
                   "tune_s": tune["tune_ms"] / 1e3 if tune else None,
                   "paper_codegen_hybrid_a100_s": PAPER_TABLE3_CODEGEN_HYBRID[(n, int(round(10 * p)))]}
            print("grid cell n=%d p=%.1f %s: %.3f s kernel" % (n, p, var, ks), file=sys.stderr, flush=True)
            rows.append(row)
    return rows


def oracle_value(workload, seed):
    """The oracle's exact count for this workload and seed, stored by
    tests/golden/make_golden.py (which calls only the oracle); None if absent."""
    path = os.path.join(ROOT, "tests", "golden", "full_size.json")
    try:
        with open(path) as f:
            rec = json.load(f).get("%s:%d" % (workload, seed))
    except OSError:
        return None
    return rec.get("perm_exact") if rec else None


def measured_traffic(src):
    """HBM bytes per dispatch of this exact generated kernel, from the committed
    rocprofv3 counter summary (None when the kernel source has changed)."""
    import hashlib
    import re
    h = hashlib.sha256(src.encode()).hexdigest()[:16]
    pdir = os.path.join(ROOT, "profiles")
    for f in sorted(os.listdir(pdir)) if os.path.isdir(pdir) else []:
        with open(os.path.join(pdir, f)) as fh:
            for m in re.finditer(r"traffic: (\{.*\})", fh.read()):
                rec = json.loads(m.group(1))
                if rec.get("source_sha256_16") == h:
                    return rec["bytes_per_dispatch"]
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="auto", choices=["auto", "pure", "hybrid"])
    ap.add_argument("--workload", default="n40_p0.10_01")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--zero-skip", default="auto", choices=["auto", "on", "off"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch-workload measurement")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the library's default options instead of the options perm_autotune picks")
    ap.add_argument("--opts", default="",
                    help="time these options (JSON of perm_sparse_ex keywords) instead of searching, e.g. for "
                         "profiling the kernel an earlier run chose")
    ap.add_argument("--no-pruned", action="store_true",
                    help="skip the run of the same permanent with exact zero-aware pruning")
    ap.add_argument("--no-exact-leg", action="store_true",
                    help="skip the all-terms run with the exact mode's certificate")
    ap.add_argument("--pruned-only", action="store_true",
                    help="run only the pruned permanent (for profiling its kernel)")
    ap.add_argument("--serving-seconds", type=float, default=60.0,
                    help="length of the Poisson serving run (0 skips it)")
    ap.add_argument("--serving-rate", type=float, default=200.0,
                    help="Poisson arrival rate of the serving run (requests/s)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving measurement (with --serving-seconds, --serving-rate)")
    ap.add_argument("--grid", default="",
                    help="run only the paper's synthetic grid for these n (comma list, e.g. 40,45,48)")
    ap.add_argument("--grid-variants", default="auto",
                    help="kernel variants for --grid: auto, hybrid, hybrid-lds, tuned (comma list)")
    ap.add_argument("--grid-p", default="",
                    help="restrict --grid to these densities, in tenths (comma list, e.g. 4,5)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batch-workload measurement (for profiling the batch kernels)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (torch), to scale HBM byte counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": src.numel() * 8, "dispatches": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the permanent's chunk ranges would shard across GPUs with a "
              "16-byte gather per GPU, but this benchmark runs and reports a single GPU only", file=sys.stderr)
        sys.exit(2)

    import paper_2501_15126_amd.perm as P
    from paper_2501_15126_amd import workloads as W

    if args.grid:
        ns = [int(x) for x in args.grid.split(",")]
        ps = [int(x) for x in args.grid_p.split(",")] if args.grid_p else None
        rows = er_grid_bench(ns, args.grid_variants.split(","), seed=args.seed, ps=ps)
        print(json.dumps({"er_grid": rows, "workload": "Erdos-Renyi n in %s, p in 0.1..0.5, U[0,1], seed %d"
                          % (ns, args.seed)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch": batch_bench(reps=2, sequential=False)}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(args.serving_seconds, rate_hz=args.serving_rate)}), flush=True)
        return
    ccs = W.WORKLOADS[args.workload](args.seed)
    n = ccs[0]
    steps_per_perm = 2.0 ** (n - 1)
    print("bench: workload %s seed %d n=%d nnz=%d mode %s" % (args.workload, args.seed, n, len(ccs[2]), args.mode),
          file=sys.stderr, flush=True)

    def tuned(**base):
        """Launch options: the autotuner's pick (searched before and outside
        the timed region), given ones, or the defaults."""
        opts = dict(base)
        tune = None
        if args.opts:
            opts.update(json.loads(args.opts))
        elif not args.no_tune:
            t = time.perf_counter()
            opts, tune = P.perm_autotune(ccs, **opts)
            tune["wall_s"] = time.perf_counter() - t
            print("bench: autotuned %s in %.1f s" % (base, tune["wall_s"]), file=sys.stderr, flush=True)
        return opts, tune

    def timed_calls(opts, steps, warmup):
        first = None
        for _ in range(warmup):
            v, st = P.perm_sparse_ex(ccs, **opts)
            first = st if first is None else first
        kernel_ms, evaluated, values, stats = [], [], [], None
        t0 = time.perf_counter()
        for _ in range(steps):
            v, st = P.perm_sparse_ex(ccs, **opts)  # synchronous: result on the host
            kernel_ms.append(st["kernel_ms"])
            evaluated.append(st["evaluated_steps"])
            values.append(v)
            stats = st
        elapsed = time.perf_counter() - t0
        return elapsed, kernel_ms, evaluated, values, stats, first

    def kernel_record(st, kernel_ms, evaluated, first):
        avg_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
        eval_steps = sum(evaluated) / len(evaluated)
        return {"name": "perm_gray", "avg_ms": avg_kernel_s * 1e3, "evaluated_steps_per_launch_set": eval_steps,
                "evaluated_steps_per_s": eval_steps / avg_kernel_s, "flops_per_step": st["flops_per_step"],
                "fp64_ops_per_step": st["ops_per_step"], "exact_ops_per_step": st["exact_ops_per_step"],
                "fp64_issue_frac": st["ops_per_step"] * eval_steps / avg_kernel_s / 3.93216e13,
                "vgprs": st["vgprs"], "sgprs": st["sgprs"], "scratch_bytes": st["scratch_bytes"],
                "waves_per_simd": st["waves_per_simd"], "waves_hint": st["waves_hint"],
                "vgpr_spills": st["vgpr_spills"], "chunk_log2": st["chunk_log2"], "unroll_log2": st["unroll_log2"],
                "levels": st["levels"], "k": st["k"], "c": st["c"], "nblocks": st["nblocks"],
                "reduce_ms": st["reduce_ms"], "host_ms": st["host_ms"],
                "compile_ms_cold": first["compile_ms"] if first else None,
                "exact": st["exact"], "exact_passes": st["exact_passes"], "err_bound": st["err_bound"],
                "estimate": st["estimate"], "skipped_fraction": 1.0 - eval_steps / steps_per_perm}

    def pruned_leg():
        """The same permanent with exact zero-aware pruning (beyond the paper):
        permanents/s, with the product's default exact certificate."""
        popts, ptune = tuned(mode=args.mode, zero_skip={"auto": "auto", "on": True}[args.zero_skip])
        pel, pk, pev, pvals, pst, pfirst = timed_calls(popts, max(args.steps, 20), args.warmup)
        pkern = kernel_record(pst, pk, pev, pfirst)
        pflops = pst["flops_per_step"] * pkern["evaluated_steps_per_launch_set"]
        return {
            "permanents_per_s": len(pk) / pel, "ms_per_permanent": pel / len(pk) * 1e3,
            "evaluated_steps_per_s": pkern["evaluated_steps_per_s"],
            "note": "most of the 2^(n-1) terms are exactly zero and skipped; evaluated_steps_per_s counts the "
                    "lane-steps the kernel evaluated",
            "kernel": pkern, "permanent": pvals[-1], "certified": pst["exact"] == 1,
            "roofline": {"bound": "alu", "achieved": pflops / (pkern["avg_ms"] / 1e3) / 1e12,
                         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": pflops / (pkern["avg_ms"] / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
                         "traffic": measured_traffic(P.perm_codegen(
                             ccs, **dict(popts, waves_per_simd=pst["waves_hint"] or -1)))},
            "options": {k: popts.get(k) for k in ("mode", "chunk_log2", "unroll_log2", "block", "waves_per_simd",
                                                   "block_queue")},
            "autotune": ptune}

    if args.pruned_only:
        print(json.dumps({"pruned": pruned_leg()}), flush=True)
        return

    # ---- headline: every Gray-code term evaluated (no pruning), accumulated
    # in FP64 as the paper does (the exact mode's residue certificate is a
    # separate leg below) ----
    opts, tune = tuned(mode=args.mode, zero_skip=False, exact=False)
    chosen = {k: opts.get(k) for k in ("mode", "chunk_log2", "unroll_log2", "block", "waves_per_simd",
                                          "block_queue", "cold_tier") if k in opts}
    print("bench: headline, %d timed permanents" % args.steps, file=sys.stderr, flush=True)
    elapsed, kernel_ms, evaluated, values, st, first = timed_calls(opts, args.steps, args.warmup)
    kern = kernel_record(st, kernel_ms, evaluated, first)
    avg_kernel_s = kern["avg_ms"] / 1e3
    # algorithmic work: the FP64 operations of the generated code per step
    # (Alg. 1's updates, products and accumulation, plus the exact mode's
    # residue and bound operations) over every evaluated step
    flops = st["flops_per_step"] * kern["evaluated_steps_per_launch_set"]
    achieved_tflops = flops / avg_kernel_s / 1e12
    src = P.perm_codegen(ccs, **dict(opts, waves_per_simd=st["waves_hint"] or -1,
                                     **({"copy_cols": st["copy_cols"]} if st["copy_cols"] else {})))
    out = {
        "metric": METRIC,
        "value": steps_per_perm * args.steps / elapsed,
        "unit": "Gray-code steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single sparse 0/1 matrix n=%d, permutation pattern OR Bernoulli(0.10), seed %d, "
                               "all 2^%d Gray-code terms evaluated, FP64 accumulation" % (n, args.seed, n - 1),
                   "n": n, "nnz": len(ccs[2]), "mode": args.mode,
                   "options": "given" if args.opts else ("library defaults" if args.no_tune else
                                                         "perm_autotune, searched before the timed region"),
                   "chosen": chosen, "gray_steps_per_permanent": steps_per_perm},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / FP64_PEAK_TFLOPS, "traffic": measured_traffic(src)},
        "kernel": kern,
        "permanent": values[-1],
        "deterministic": all(x == values[0] for x in values),
    }
    if tune is not None:
        out["autotune"] = tune
    ref = oracle_value(args.workload, args.seed)
    if ref is not None:
        out["oracle_integer"] = ref
        out["matches_oracle_integer"] = values[-1] == float(int(ref))
    # ---- the same, with the exact mode's certificate (residue modulo a
    # prime and a rigorous FP64 error bound), same launch options ----
    if not args.no_exact_leg:
        print("bench: exact all-terms leg", file=sys.stderr, flush=True)
        # the tuned launch shape, but the exact kernels' own static block and copies
        xopts = dict(opts, exact="auto", chunk_log2=0, unroll_log2=0, copy_cols=0)
        xel, xk, xev, xvals, xst, xfirst = timed_calls(xopts, max(2, args.steps // 4), 1)
        xkern = kernel_record(xst, xk, xev, xfirst)
        out["exact_all_terms"] = {
            "ms_per_permanent": xel / len(xk) * 1e3, "gray_steps_per_s": steps_per_perm * len(xk) / xel,
            "kernel": xkern, "permanent": xvals[-1], "certified": xst["exact"] == 1,
            "note": "every term evaluated, plus the residue and error-bound operations that certify the integer"}
    if args.zero_skip != "off" and not args.no_pruned:
        print("bench: pruned leg", file=sys.stderr, flush=True)
        out["pruned"] = pruned_leg()
    if not args.no_batch:
        bopts = None
        if not args.no_tune:
            from paper_2501_15126_amd import workloads as W2
            bopts, btune = P.perm_batch_autotune(W2.batch(1, 2000))
            print("bench: batch autotuned: %s" % bopts, file=sys.stderr, flush=True)
        out["batch"] = batch_bench(opts={k: bopts[k] for k in ("block", "batch_kappa_shift")} if bopts else None)
        print("bench: batch done, %.1f permanents/s" % out["batch"]["permanents_per_s"], file=sys.stderr, flush=True)
    if args.serving_seconds > 0:
        print("bench: serving run, %.0f s (then the sequential baseline on the same trace)" % args.serving_seconds,
              file=sys.stderr, flush=True)
        out["serving"] = serving_bench(args.serving_seconds, rate_hz=args.serving_rate)
        print("bench: serving done, p50 %.2f ms p99 %.2f ms" % (out["serving"]["p50_ms"], out["serving"]["p99_ms"]),
              file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        print("bench: CPU oracle samples", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(ccs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
