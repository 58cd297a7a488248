"""Write the oracle's reference solutions used by the GPU parity tests.

Calls only the oracle (and the seeded generators).  Each file records the
dense PDIPM's solution at a tight gap so that a solver stopped at gap 1e-7
can be compared with it, plus per-iteration timings of the oracle.

    python tests/golden/make_golden.py cfg1        # five seeds, n = 64
    python tests/golden/make_golden.py cfg3        # norm-min, n = 2010, m = 64
    python tests/golden/make_golden.py cfg2        # max-cut band, n = m = 4000 (slow)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import sdpgen  # noqa: E402


def run(name, prob, gap):
    P = oracle.Params(gap_tol=gap, feas_tol=gap)
    t0 = time.time()
    res = oracle.dense_pdipm(prob, P, verbose=True)
    out = dict(name=name, problem=prob.name, n=prob.n, m=prob.m, gap_tol=gap,
               status=res["status"], iters=res["iters"], pobj=res["pobj"], dobj=res["dobj"],
               relgap=res["relgap"], pinf=res["pinf"], dinf=res["dinf"],
               z=res["z"].tolist(), seconds=time.time() - t0,
               t_scm=[h.get("t_scm") for h in res["history"] if "t_scm" in h],
               t_iter=[h.get("t_iter") for h in res["history"] if "t_iter" in h],
               history=[{k: h[k] for k in ("it", "pobj", "dobj", "relgap", "pinf", "dinf")}
                        for h in res["history"]])
    # iterations the same run needed to pass the default stopping test (gap and
    # infeasibilities <= 1e-7): the iteration count of a solve at gap 1e-7
    out["iters_to_1e-7"] = next((h["it"] for h in res["history"]
                                 if h["relgap"] <= 1e-7 and h["pinf"] <= 1e-7 and h["dinf"] <= 1e-7),
                                None)
    # also the trajectory at the default tolerance, for iteration counts
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(out, f)
    print(name, res["status"], res["iters"], res["pobj"], res["dobj"], flush=True)


def main(which):
    if which == "cfg1":
        for s in range(5):
            run(f"cfg1_s{s}", sdpgen.maxcut_cycle_chords(64, s), 1e-10)
    elif which == "cfg3":
        run("cfg3", sdpgen.normmin(2000, 10, 63, 0), 1e-10)
    elif which == "cfg2":
        run("cfg2", sdpgen.maxcut_band(4000, 20, 0.5, 0), 1e-9)
    elif which == "small":
        run("band300", sdpgen.maxcut_band(300, 20, 0.5, 1), 1e-10)
        run("normmin_small", sdpgen.normmin(200, 10, 15, 1), 1e-10)
    else:
        raise SystemExit(f"unknown set {which}")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "cfg1")
