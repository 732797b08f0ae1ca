"""Writes layered128_oracle_exits.json: the oracle's PCG exits on the 128^3
layered stack (2,146,689 DOF, 20 repeats of three layers, 10:1 flat
elements, theta 0.08, CG to a relative residual of 1e-8 as in the solver
settings of the numerical section).

Cases: the right-hand side as generated, from x0 = 0; the same with every
nonzero entry of b moved by one ulp (five seeded coin flips); and five seeded
starts x0 ~ U(0, 1).  With --add, the seeded start 0 again under one-ulp
changes of b (three seeds, "x0ulp") and with A's values scaled by
1 + j 2^-52 (j = 1, 2, 3, the setup rerun, "x0scale") are appended to the
record.  Each records the iteration count, the true relative residual and the
relative error against the exact discrete solution (the z-only
series-resistor profile).  Only the oracle and the input generators run here.
Run from the repository root:

    python tests/golden/make_layered128_oracle_exits.py [--workers 6] [--add]

Each case builds its own oracle hierarchy (about 5 GB, 20 s) and solves
(two to four minutes on one core); the cases run in parallel processes.
"""

import argparse
import json
import multiprocessing as mp
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "layered128_oracle_exits.json")


def problem():
    from workloads.q1 import layered_stack_3d
    return layered_stack_3d(n=128, repeats=20, stretch=10.0)


def exact(prob):
    import numpy as np
    kz = prob.meta["layer_k"]
    res = 1.0 / kz
    cf = np.concatenate([[0.0], np.cumsum(res)]) / res.sum()
    return cf[np.rint(prob.coords[:, 2] * 128).astype(int)]


def run_case(case):
    import dataclasses

    import numpy as np
    import oracle
    from workloads.q1 import seeded_start, ulp_perturbed
    kind, k = case
    prob = problem()
    b, x0 = prob.b, None
    if kind == "ulp":
        b = ulp_perturbed(prob.b, k)
    elif kind == "x0":
        x0 = seeded_start(prob.n, k)
    elif kind == "x0ulp":
        b = ulp_perturbed(prob.b, k)
        x0 = seeded_start(prob.n, 0)
    elif kind == "x0scale":
        # in exact arithmetic the hierarchy scales by c and the iterates by
        # 1/c; in floating point every rounding of setup and solve changes
        prob = dataclasses.replace(prob, val=prob.val * (1.0 + k * 2.0**-52))
        b = prob.b
        x0 = seeded_start(prob.n, 0)
    h = oracle.Hierarchy(prob)
    t = time.time()
    x, info = h.pcg(b, x0=x0)
    ex = exact(prob)
    return dict(case=kind, seed=k, iterations=info["iterations"], status=info["status"],
                rel_res=info["rel_res"], err_vs_exact=float(np.linalg.norm(x - ex) / np.linalg.norm(ex)),
                solve_s=round(time.time() - t, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--add", action="store_true", help="append the seeded-start spread cases to the record")
    args = ap.parse_args()
    prob = problem()
    from workloads.q1 import problem_digest
    digest = problem_digest(prob)
    del prob
    if args.add:
        with open(OUT) as f:
            out = json.load(f)
        assert out["input_sha256"] == digest
        cases = [("x0ulp", k) for k in range(3)] + [("x0scale", j) for j in (1, 2, 3)]
        with mp.get_context("spawn").Pool(args.workers) as pool:
            rows = pool.map(run_case, cases, chunksize=1)
        out["cases"] = [c for c in out["cases"] if c["case"] not in ("x0ulp", "x0scale")] + rows
        with open(OUT, "w") as f:
            json.dump(out, f, indent=1)
        for r in rows:
            print(r)
        return
    cases = [("b", 0)] + [("ulp", k) for k in range(5)] + [("x0", k) for k in range(5)]
    with mp.get_context("spawn").Pool(args.workers) as pool:
        rows = pool.map(run_case, cases, chunksize=1)
    out = dict(workload="layered stack 128^3, 20 repeats x 3 layers, 10:1 flat, theta 0.08, tol 1e-8",
               input_sha256=digest, host=platform.processor() or platform.machine(), cases=rows)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    for r in rows:
        print(r)


if __name__ == "__main__":
    main()
