#!/usr/bin/env python
"""Benchmark: whole solves of the max-cut band SDP (n = m = 4000, bandwidth
20, each in-band edge with probability 1/2, weights U[0,1], seed 0) to a
relative gap of 1e-7 with the matrix-completion PDIPM on one MI355X.

One step = one sdpc_solve from the initial point (Section 2.2, Steps 0-4
repeated until the stopping test holds); the handle (symbolic phase and the
upload of the problem) is created before the timed region, so the inputs are
resident in HBM when it starts.  Prints one JSON line:

  value            solves per second (whole job, one GPU)
  scm_s_per_iter   device time of one Schur complement evaluation on its own
                   (sdpc_scm at the final iterate, median of 5): Y = N N^T,
                   the X factor (Algorithm 1), the substitutions forming X^ and
                   Y^{-1}, the SCM assembly and the SCM Cholesky
  scm_s_per_iter_in_solve
                   the same phases as they run inside a solve, per iteration:
                   there the factor of Y comes from the dual step and the X
                   factor is formed in the previous iteration's shadow, so only
                   the substitutions, the assembly with the right-hand side and
                   the Cholesky with the SCE solve are on the iteration's path
  phase_roofline   per phase of the standalone evaluation: its algorithmic bytes
                   and flops, achieved GB/s and GFLOP/s, and the fraction of the
                   roofline max(bytes / 8 TB/s, flops / 78.6 TFLOP/s) / time
  measured_peaks   a 1 GiB device copy and an FP64 GEMM (n = 8192, the vendor
                   library) timed on this GPU, beside the datasheet peaks
  roofline         the SCM Cholesky (the largest dense kernel of an iteration):
                   m^3/3 FP64 flops per factorisation over its average device
                   time, measured with events on the library's stream during
                   the timed solves, against the FP64 matrix peak
  cpu_baseline     the CPU oracle (dense FP64 PDIPM, NumPy/SciPy on all host
                   cores) on a bounded sample: its first iterations on the same
                   instance, scaled by the iteration count the oracle needs to
                   reach gap 1e-7 on it (stored by tests/golden/make_golden.py)
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SCM assembly+Cholesky s/iter and solves/sec on 1 MI355X vs plain, gap 1e-7"
FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


KERNEL_SOURCE = os.path.join(ROOT, "paper_1310_6919_amd", "csrc", "k_dense.hip")


def source_sha1(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


BAND = "maxcut-band n=m=4000 bandwidth 20 p=0.5 w~U[0,1] seed 0"
NORMMIN = ("norm-min [[t I, F(y)], [F(y)^T, t I]], F_i 2000 x 10 ~ N(0,1)/sqrt(2000), 63 y's plus t "
           "(n=2010, m=64), seed 0")
CYCLE = "maxcut cycle + chords at cyclic distance <=4 (p=0.5), n=m=64, w~U[0,1], seed 0"
GOLDEN = {"band4000": "oracle_cfg2.json", "normmin": "oracle_cfg3.json", "cfg1": "oracle_cfg1_s0.json"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def workload(name="band4000"):
    """(problem, create parameters, description) of a named workload.  band4000 is
    the metric's workload; latticeP is the max-cut SDP over the paper's P x 10
    lattice graph (MaxCut400 .. MaxCut1200 sizes at P = 400 .. 1200; weights
    U[0,1], seed 0) in the short-side-first elimination order."""
    import sdpgen
    if name == "band4000":
        return sdpgen.maxcut_band(4000, 20, 0.5, 0), {}, BAND
    if name == "normmin":
        return sdpgen.normmin(2000, 10, 63, 0), {}, NORMMIN
    if name == "cfg1":
        return sdpgen.maxcut_cycle_chords(64, 0), {}, CYCLE
    if name.startswith("lattice"):
        p = int(name[len("lattice"):])
        prob = sdpgen.maxcut_lattice(p, 10, 0)
        desc = (f"maxcut-lattice p={p} q=10 (n=m={10 * p}) w~U[0,1] seed 0, "
                "short-side-first elimination order")
        return prob, {"user_perm": sdpgen.lattice_short_first_order(p, 10)}, desc
    raise SystemExit(f"unknown workload {name}")


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        return os.cpu_count()


def cpu_full_solves(prob, runs=6):
    """Whole oracle solves to gap 1e-7 (small instances): median of runs - 1 after a
    discarded first run, on all BLAS threads and on one."""
    import oracle
    from threadpoolctl import threadpool_limits
    out = {}
    for label, limit in (("all_threads", None), ("one_thread", 1)):
        times = []
        with threadpool_limits(limits=limit):
            threads = blas_threads()
            for _ in range(runs):
                t0 = time.perf_counter()
                res = oracle.dense_pdipm(prob, oracle.Params())
                times.append(time.perf_counter() - t0)
        med = statistics.median(times[1:])
        out[label] = {"value": 1.0 / med, "s_per_solve": med, "cores": int(threads), "iters": int(res["iters"])}
    best = out["all_threads"]
    return {
        "value": best["value"],
        "unit": "solves/s",
        "cores": best["cores"],
        "kind": "oracle",
        "sample": (f"whole dense-oracle solves to gap 1e-7 ({best['iters']} iterations), median of {runs - 1} "
                   f"after a discarded first run; single-threaded: {out['one_thread']['value']:.2f} solves/s"),
        "one_thread": out["one_thread"],
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
    }


def cpu_baseline(prob, iters, golden="oracle_cfg2.json"):
    """Time the oracle's first `iters` iterations on the same instance."""
    import numpy as np  # noqa: F401
    import oracle
    threads = blas_threads()
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", golden)))
    n_it = gold.get("iters_to_1e-7") or gold["iters"]
    t0 = time.perf_counter()
    res = oracle.dense_pdipm(prob, oracle.Params(), max_iter=iters)
    wall = time.perf_counter() - t0
    t_iter = [h["t_iter"] for h in res["history"] if "t_iter" in h]
    t_scm = [h["t_scm"] for h in res["history"] if "t_scm" in h]
    per_iter = statistics.mean(t_iter)
    return {
        "value": 1.0 / (per_iter * n_it),
        "unit": "solves/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"first {len(t_iter)} iterations of the dense oracle PDIPM on the same instance "
                   f"({wall:.1f} s wall), mean {per_iter:.2f} s/iter scaled by the {n_it} iterations "
                   f"the oracle takes to reach gap 1e-7"),
        "s_per_iter": per_iter,
        "scm_s_per_iter": statistics.mean(t_scm),
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
    }


def measured_peaks():
    """A 1 GiB device-to-device copy (read + write) and an FP64 GEMM of order 8192
    through the vendor library, timed with events on torch's stream."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    a = torch.randn(8192, 8192, dtype=torch.float64, device="cuda")
    b = torch.randn(8192, 8192, dtype=torch.float64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(2):
        dst.copy_(src)
        c = a @ b
    ev[0].record()
    for _ in range(5):
        dst.copy_(src)
    ev[1].record()
    ev[2].record()
    for _ in range(3):
        c = a @ b
    ev[3].record()
    torch.cuda.synchronize()
    copy_s = ev[0].elapsed_time(ev[1]) / 5 / 1e3
    gemm_s = ev[2].elapsed_time(ev[3]) / 3 / 1e3
    del src, dst, a, b, c
    torch.cuda.empty_cache()
    return {"copy_GBs": 2 * (1 << 30) / copy_s / 1e9, "dgemm_TFLOPs": 2 * 8192.0 ** 3 / gemm_s / 1e12,
            "datasheet_hbm_GBs": HBM_PEAK_GBS, "datasheet_fp64_mfma_TFLOPs": FP64_MFMA_PEAK_TFLOPS}


def solve_flops(h):
    """Flops of the substitutions forming one dense inverse L^{-T} L^{-1} column by
    column with the sparse factor (pattern of E): for column k the forward solve runs
    over the elimination-tree ancestors of k, the backward solve (rows >= k only) over
    every column >= k; 2 flops per stored entry of each column visited."""
    import numpy as np
    iE, jE, perm = h.sdpc_get_pattern()
    pos = np.empty(len(perm), dtype=np.int64)
    pos[perm] = np.arange(len(perm))
    ok = iE >= 0
    pi, pj = pos[iE[ok]], pos[jE[ok]]
    n = len(perm)
    cc = np.bincount(pj, minlength=n).astype(np.float64)
    off = pi > pj
    parent = np.full(n, -1, dtype=np.int64)
    first_below = np.full(n, n, dtype=np.int64)
    np.minimum.at(first_below, pj[off], pi[off])
    parent[first_below < n] = first_below[first_below < n]
    anc = cc.copy()
    for k in range(n - 1, -1, -1):   # parents have larger positions
        if parent[k] >= 0:
            anc[k] += anc[parent[k]]
    suffix = np.cumsum(cc[::-1])[::-1]
    return float(2.0 * (anc.sum() + suffix.sum()))


def assembly_work(prob):
    """(Hadamard form?, flops of the general assembly): per constraint q the product
    X^ A_q over the nonzero columns of A_q (2 n nnz(A_q)) and the support-restricted
    product with Y^{-1} (2 |support| |K_q|)."""
    import numpy as np
    had = True
    sup = set()
    per_q = []
    for k in range(1, prob.m + 1):
        r, c, v = prob.triplets(k)
        nz = v != 0
        r, c = r[nz], c[nz]
        if not (len(r) and np.all(r == c) and np.all(r == r[0])):
            had = False
        cols = set(c.tolist()) | set(r.tolist())
        nnz_full = len(r) + int(np.sum(r != c))
        per_q.append((nnz_full, len(cols)))
        sup.update(zip(r.tolist(), c.tolist()))
        sup.update(zip(c.tolist(), r.tolist()))
    S = len(sup)
    return had, float(sum(2.0 * prob.n * nz + 2.0 * S * kq for nz, kq in per_q))


def standalone_scm(h, prob, reps=5):
    """One Schur complement evaluation on its own at the handle's current iterate,
    phase by phase (median of reps), with the algorithmic work of each phase."""
    import torch
    X, Y, _ = h.sdpc_get_solution()
    B = torch.empty(prob.m, prob.m, dtype=torch.float64, device="cuda").T
    rows = []
    for _ in range(reps):
        h.sdpc_scm(X, Y, B, factor=True)
        rows.append(h.sdpc_get_scm_timing())
    med = [statistics.median(r[i] for r in rows) for i in range(5)]
    n, m = prob.n, prob.m
    had, fl_asm = assembly_work(prob)
    # algorithmic work: the substitutions write X^ and Y^{-1} (n^2 doubles each); the
    # max-cut assembly reads both lower triangles and writes B's, the general one does
    # the dense x sparse and support-restricted products; the Cholesky does m^3 / 3
    # flops on B's lower triangle, read and written once
    phases = {
        "y_factor": {"ms": med[0], "bound": "latency"},
        "x_factor": {"ms": med[1], "bound": "latency"},
        "solves": {"ms": med[2], "bytes": 2 * 8.0 * n * n, "flops": 2 * solve_flops(h)},
        "assembly": {"ms": med[3], "bytes": (3 * 8.0 * m * (m + 1) / 2) if had else None,
                     "flops": None if had else fl_asm},
        "cholesky": {"ms": med[4], "bytes": 2 * 8.0 * m * (m + 1) / 2, "flops": m ** 3 / 3.0},
    }
    for ph in phases.values():
        t = ph["ms"] * 1e-3
        if t <= 0:
            continue
        bt = ph.get("bytes")
        ft = ph.get("flops")
        if bt:
            ph["achieved_GBs"] = bt / t / 1e9
        if ft:
            ph["achieved_GFLOPs"] = ft / t / 1e9
        if bt or ft:
            ideal = max((bt or 0) / (HBM_PEAK_GBS * 1e9), (ft or 0) / (FP64_MFMA_PEAK_TFLOPS * 1e12))
            ph["frac"] = ideal / t
    return sum(med) * 1e-3, phases


def batch_solve(args):
    """The same 256 instances through the batched solver (sdpc_batch_solve): host
    workers with one HIP stream each keep many instances in flight; the block width
    is tuned per size class.  One step is the whole batch (analysis, tuning, creates,
    solves and releases)."""
    import numpy as np
    import torch
    import sdpgen
    from paper_1310_6919_amd.sdpc import sdpc_batch_solve
    probs = sdpgen.maxcut_ktree_batch(256, 0)
    prm = [{"user_perm": np.arange(p.n)[::-1].astype(np.int32)} for p in probs]
    times, opts, iters = [], [], []
    for step in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res, _, opt = sdpc_batch_solve(probs, prm, workers=args.batch_workers, autotune=True, want_z=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if step >= args.warmup:
            times.append(dt)
            opts.append(opt)
            iters.extend(r["iters"] for r in res)
        log(f"batch pass {step}: {dt:.2f} s (tune {opt['tune_ms']:.0f} ms, create {opt['create_ms']:.0f} ms, "
            f"solve {opt['solve_ms']:.0f} ms), widths {opt['tuned_width']}")
    elapsed = sum(times)
    out = {
        "metric": "batched solves of the 256-instance k-tree max-cut batch, gap 1e-7",
        "value": len(probs) * args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "256 max-cut SDPs, n~U[50,800], random k-trees k~U[3,12], 30% edges dropped, "
                               "w~U[0,1], seed 0, reverse insertion order; batched", "gap_tol": 1e-7,
                   "workers": args.batch_workers,
                   "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES", "runtime default")},
        "phases_ms": {k: statistics.median(o[k] for o in opts) for k in ("tune_ms", "create_ms", "solve_ms",
                                                                          "total_ms")},
        "tuned_width": opts[-1]["tuned_width"],
        "iters_mean": float(np.mean(iters)),
        "iters_max": int(max(iters)),
    }
    print(json.dumps(out), flush=True)


def batch_loop(args):
    """256 independent max-cut SDPs (n uniform in [50, 800], random k-trees with k in
    [3, 12] and 30% of the edges dropped, weights U[0,1], seed 0), each created and
    solved by the plain solver in the reverse insertion order of its k-tree (a
    perfect elimination order): the reference for a batched solver.  One step is the
    whole batch, creates included."""
    import numpy as np
    import torch
    import sdpgen
    from paper_1310_6919_amd import sdpc_create
    probs = sdpgen.maxcut_ktree_batch(256, 0)
    times = []
    t_create = 0.0
    iters = []
    for step in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for p in probs:
            t1 = time.perf_counter()
            h = sdpc_create(p, user_perm=np.arange(p.n)[::-1].astype(np.int32))
            t_create += time.perf_counter() - t1 if step >= args.warmup else 0.0
            r = h.sdpc_solve()
            if r["status"] != 0:
                raise SystemExit(f"solve failed on {p.name}: {r}")
            if step >= args.warmup:
                iters.append(r["iters"])
            h.close()
        torch.cuda.synchronize()
        if step >= args.warmup:
            times.append(time.perf_counter() - t0)
        log(f"batch pass {step}: {time.perf_counter() - t0:.2f} s")
    elapsed = sum(times)
    out = {
        "metric": "plain per-instance solves of the 256-instance k-tree max-cut batch, gap 1e-7",
        "value": len(probs) * args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "256 max-cut SDPs, n~U[50,800], random k-trees k~U[3,12], 30% edges dropped, "
                               "w~U[0,1], seed 0, reverse insertion order", "gap_tol": 1e-7},
        "create_s_per_step": t_create / args.steps,
        "iters_mean": float(np.mean(iters)),
        "iters_max": int(max(iters)),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-iters", type=int, default=2, help="oracle iterations in the CPU sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the copy / FP64 GEMM peak measurement")
    ap.add_argument("--workload", default="band4000",
                    help="band4000 (the metric's workload), normmin (norm minimisation, n = 2010, m = 64), "
                         "cfg1 (max-cut, n = m = 64), latticeP (P x 10 lattice max-cut, e.g. lattice400), "
                         "ktree256 (256 uneven k-tree max-cut SDPs through the batched solver) or "
                         "ktree256plain (the same, one plain solve after another)")
    ap.add_argument("--batch-workers", type=int, default=16, help="host workers of the batched solver")
    ap.add_argument("--hw-queues", type=int, default=0,
                    help="hardware queues of the HIP runtime (GPU_MAX_HW_QUEUES, set before the runtime "
                         "starts; 0 keeps the runtime's default)")
    ap.add_argument("--factorization", type=int, default=0, choices=(0, 1),
                    help="0: X^ through Algorithm 1's Lhat (the method); 1: the earlier X^ = L^T D L "
                         "(the factorisation ablation)")
    ap.add_argument("--chol-kernel", type=int, default=0, choices=(0, 1),
                    help="SCM Cholesky: 0 one dataflow launch per factorisation, 1 one launch per "
                         "64-column block")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "potrf_traffic.json"),
                    help="HBM traffic per factorisation from rocprofv3 counters (json), if present")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (a plain copy kernel of known size, "
                         "to scale FETCH_SIZE / WRITE_SIZE counters taken on the same command)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    if args.workload == "ktree256" and args.hw_queues == 0:
        args.hw_queues = 16   # one hardware queue per batch worker
    if args.hw_queues > 0:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(args.hw_queues, 32))   # read when the runtime starts (at most 32)
    import torch
    from paper_1310_6919_amd import sdpc_create
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nbytes} bytes read, {nbytes} bytes written")
        del src, dst
    if args.workload == "ktree256":
        batch_solve(args)
        return
    if args.workload == "ktree256plain":
        batch_loop(args)
        return
    prob, cparams, desc = workload(args.workload)
    if args.factorization:
        cparams = dict(cparams, factorization=args.factorization)
    if args.chol_kernel:
        cparams = dict(cparams, chol_kernel=args.chol_kernel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = sdpc_create(prob, **cparams)
    torch.cuda.synchronize()
    create_ms = (time.perf_counter() - t0) * 1e3
    log(f"create: {create_ms:.1f} ms")
    for i in range(args.warmup):
        r = h.sdpc_solve()
        log(f"warmup {i}: status {r['status']} iters {r['iters']} {r['t_total_ms']:.1f} ms")
    results = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = h.sdpc_solve()
        results.append(r)
        log(f"step {i}: status {r['status']} iters {r['iters']} {r['t_total_ms']:.1f} ms "
            f"obj {(r['pobj'] + r['dobj']) / 2:.9f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for r in results:
        if r["status"] != 0:
            raise SystemExit(f"solve failed: {r}")
    iters = [r["iters"] for r in results]
    scm_in_solve = statistics.median([(r["t_scm_ms"] + r["t_chol_ms"]) / r["iters"] / 1e3 for r in results])
    scm_alone, phases = standalone_scm(h, prob)
    potrf_ms = sum(r["t_potrf_ms"] for r in results) / max(1, sum(r["n_potrf"] for r in results))
    m = prob.m
    flow = int(h.params.chol_kernel) == 0
    launches = 1 if flow else (m + 63) // 64
    flops = m ** 3 / 3.0
    achieved = flops / (potrf_ms * 1e-3) / 1e12
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        # counters count only for the kernel source they were taken on
        try:
            rec = json.load(open(args.traffic))
            if (rec.get("source_sha1") == source_sha1(KERNEL_SOURCE) and rec.get("m", 4000) == m
                    and rec.get("kernel") == ("k_chol_flow" if flow else "k_chol_step")):
                traffic = rec.get("bytes_per_factorisation")
        except Exception:
            traffic = None
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": prob.n, "m": m, "gap_tol": 1e-7,
                   "block_width": int(h.params.block_width), "factorization": int(h.params.factorization),
                   "chol_kernel": int(h.params.chol_kernel)},
        "scm_s_per_iter": scm_alone,
        "scm_s_per_iter_in_solve": scm_in_solve,
        "phase_roofline": phases,
        "iters": iters[0],
        "objective": (results[-1]["pobj"] + results[-1]["dobj"]) / 2,
        "create_ms": create_ms,
        "phase_ms_per_iter": {
            "scm": statistics.median([r["t_scm_ms"] / r["iters"] for r in results]),
            "chol_and_sce": statistics.median([r["t_chol_ms"] / r["iters"] for r in results]),
            "pmatrix_and_steps": statistics.median([r["t_pmatrix_ms"] / r["iters"] for r in results]),
        },
        "roofline": {
            "kernel": ("SCM Cholesky: k_chol_flow, one dataflow launch per factorisation" if flow else
                       "SCM Cholesky: k_chol_step, one launch per 64-column block (%d per factorisation); "
                       "per-launch figures are averages over the launches of a factorisation" % launches),
            "bound": "mfma",
            "achieved": achieved,
            "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_MFMA_PEAK_TFLOPS,
            "traffic": None if traffic is None else traffic / launches,
            "avg_ms": potrf_ms / launches,
            "flops_per_launch": flops / launches,
            "launches_per_factorisation": launches,
            "ms_per_factorisation": potrf_ms,
            "flops_per_factorisation": flops,
            "traffic_per_factorisation": traffic,
        },
    }
    h.close()
    asm = phases["assembly"]
    if asm.get("flops") and asm["ms"] > 0 and asm["flops"] > flops:
        # general constraint matrices: the assembly's dense products are the dominant
        # contraction of the iteration, not the small SCM Cholesky
        a = asm["flops"] / (asm["ms"] * 1e-3) / 1e12
        out["roofline"] = {
            "kernel": "SCM assembly, column-compressed general form (k_gemm_nn products X^ U_cat and "
                      "Y^{-1} U_cat, sparse rows, Hadamard block and pair contractions), one evaluation",
            "bound": "mfma", "achieved": a, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": a / FP64_MFMA_PEAK_TFLOPS, "traffic": None, "avg_ms": asm["ms"],
            "flops_per_evaluation": asm["flops"],
        }
    if args.workload.startswith("lattice"):
        # a bipartite graph: the relaxation's optimum is minus the total weight
        total = float(prob.meta["weights"].sum())
        out["optimum_closed_form"] = -total
        out["objective_rel_err"] = abs(out["objective"] + total) / total
    if not args.no_peaks:
        out["measured_peaks"] = measured_peaks()
    if not args.no_cpu_baseline and args.workload == "cfg1":
        log("cpu baseline: whole oracle solves ...")
        out["cpu_baseline"] = cpu_full_solves(prob)
    elif not args.no_cpu_baseline and args.workload in GOLDEN:
        log(f"cpu baseline: {args.cpu_iters} oracle iterations on the same instance ...")
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_iters, GOLDEN[args.workload])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
