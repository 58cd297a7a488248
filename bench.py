#!/usr/bin/env python
"""Benchmark: whole solves of the max-cut band SDP (n = m = 4000, bandwidth
20, each in-band edge with probability 1/2, weights U[0,1], seed 0) to a
relative gap of 1e-7 with the matrix-completion PDIPM on one MI355X.

One step = one sdpc_solve from the initial point (Section 2.2, Steps 0-4
repeated until the stopping test holds); the handle (symbolic phase and the
upload of the problem) is created before the timed region, so the inputs are
resident in HBM when it starts.  Prints one JSON line:

  value            solves per second (whole job, one GPU)
  scm_s_per_iter   device time per iteration of the Schur complement phase:
                   Y factor, Algorithm 1, substitutions, SCM assembly and the
                   right-hand side, plus the SCM Cholesky and SCE solve
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


def workload(name="band4000"):
    """(problem, create parameters, description) of a named workload.  band4000 is
    the metric's workload; latticeP is the max-cut SDP over the paper's P x 10
    lattice graph (MaxCut400 .. MaxCut1200 sizes at P = 400 .. 1200; weights
    U[0,1], seed 0) in the short-side-first elimination order."""
    import sdpgen
    if name == "band4000":
        return sdpgen.maxcut_band(4000, 20, 0.5, 0), {}, BAND
    if name.startswith("lattice"):
        p = int(name[len("lattice"):])
        prob = sdpgen.maxcut_lattice(p, 10, 0)
        desc = (f"maxcut-lattice p={p} q=10 (n=m={10 * p}) w~U[0,1] seed 0, "
                "short-side-first elimination order")
        return prob, {"user_perm": sdpgen.lattice_short_first_order(p, 10)}, desc
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(prob, iters):
    """Time the oracle's first `iters` iterations on the same instance."""
    import numpy as np  # noqa: F401
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_cfg2.json")))
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
        "host_cpus": os.cpu_count(),
    }


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
    ap.add_argument("--workload", default="band4000",
                    help="band4000 (the metric's workload), latticeP (P x 10 lattice max-cut, e.g. lattice400) "
                         "or ktree256 (256 uneven k-tree max-cut SDPs, one plain solve each)")
    ap.add_argument("--factorization", type=int, default=0, choices=(0, 1),
                    help="0: X^ through Algorithm 1's Lhat (the method); 1: the earlier X^ = L^T D L "
                         "(the factorisation ablation)")
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
        batch_loop(args)
        return
    prob, cparams, desc = workload(args.workload)
    if args.factorization:
        cparams = dict(cparams, factorization=args.factorization)
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
    scm_per_iter = statistics.median([(r["t_scm_ms"] + r["t_chol_ms"]) / r["iters"] / 1e3 for r in results])
    potrf_ms = sum(r["t_potrf_ms"] for r in results) / max(1, sum(r["n_potrf"] for r in results))
    m = prob.m
    launches = (m + 63) // 64
    flops = m ** 3 / 3.0
    achieved = flops / (potrf_ms * 1e-3) / 1e12
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        # counters count only for the kernel source they were taken on
        try:
            rec = json.load(open(args.traffic))
            if rec.get("source_sha1") == source_sha1(KERNEL_SOURCE) and rec.get("m", 4000) == m:
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
                   "block_width": int(h.params.block_width), "factorization": int(h.params.factorization)},
        "scm_s_per_iter": scm_per_iter,
        "iters": iters[0],
        "objective": (results[-1]["pobj"] + results[-1]["dobj"]) / 2,
        "create_ms": create_ms,
        "phase_ms_per_iter": {
            "scm": statistics.median([r["t_scm_ms"] / r["iters"] for r in results]),
            "chol_and_sce": statistics.median([r["t_chol_ms"] / r["iters"] for r in results]),
            "pmatrix_and_steps": statistics.median([r["t_pmatrix_ms"] / r["iters"] for r in results]),
        },
        "roofline": {
            "kernel": "SCM Cholesky: k_chol_step, one launch per 64-column block (%d per factorisation); "
                      "per-launch figures are averages over the launches of a factorisation" % launches,
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
    if args.workload.startswith("lattice"):
        # a bipartite graph: the relaxation's optimum is minus the total weight
        total = float(prob.meta["weights"].sum())
        out["optimum_closed_form"] = -total
        out["objective_rel_err"] = abs(out["objective"] + total) / total
    if not args.no_cpu_baseline and args.workload == "band4000":
        log(f"cpu baseline: {args.cpu_iters} oracle iterations on the same instance ...")
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
