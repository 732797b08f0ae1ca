"""Writes serving_oracle_outcomes.json: the oracle's PCG outcome (FP64, tol
1e-8, at most 1000 iterations, the server's cap) on every layered request of
the seeded serving stream (256 requests, seed 0) with at most 64 elements
per side -- the thin stacks (60 layers on 32 to 64 elements) on which the
server reports NOT_CONVERGED -- so that the server's failures can be matched
against the oracle's.  --add appends the layered requests with more
elements per side (65 to 128; hours of CPU time) to the existing file.  Only
the oracle and the input generators run here.  From the repository root:

    python tests/golden/make_serving_oracle_outcomes.py [--workers 6] [--add]

With --ulp it reads that file back, selects the requests a GPU test serves
(converged within 600 iterations on at most 100000 unknowns, or stopped at
the cap 10x above the tolerance on at most 110592 unknowns) and writes
serving_oracle_ulp_exits.json: the oracle's outcome on each, with b as
generated (seed null, scale 0), with b moved by one unit in the last place
(three seeds), and with A's values scaled by 1 + j 2^-52 (scale j = 1, 2,
3; setup and solve rerun), and the true relative residual of each run: the
spread of its exit under rounding-level changes of the data and of every
rounding in the setup.
"""

import argparse
import dataclasses
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "serving_oracle_outcomes.json")
ULP_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "serving_oracle_ulp_exits.json")
ULP_SEEDS = (0, 1, 2)
OP_SCALES = (1, 2, 3)


def selected(cases):
    conv = [c["request"] for c in cases if c["status"] == 0 and c["iterations"] <= 600 and c["dof"] <= 100000]
    stuck = [c["request"] for c in cases if c["status"] != 0 and c["rel_res"] >= 1e-7 and c["dof"] <= 110592]
    return conv, stuck


def run(req):
    import oracle
    from workloads import problem_from_request

    prob = problem_from_request(req)
    t = time.time()
    h = oracle.Hierarchy(prob)
    _, info = h.pcg(prob.b, maxit=1000)
    return dict(request=req["id"], n=req["n"], dof=prob.n, iterations=info["iterations"], status=info["status"],
                rel_res=info["rel_res"], seconds=round(time.time() - t, 1))


def run_ulp(req):
    import numpy as np

    import oracle
    from workloads import problem_from_request, ulp_perturbed

    prob = problem_from_request(req)
    h = oracle.Hierarchy(prob)
    rows = []
    for seed in (None,) + ULP_SEEDS:
        b = prob.b if seed is None else ulp_perturbed(prob.b, seed)
        x, info = h.pcg(b, maxit=1000)
        # the residual recomputed from x (the solver reports its recurrence's
        # residual when it stops at the cap)
        true = np.linalg.norm(b - oracle.spmv(prob.rowptr, prob.col, prob.val, x)) / np.linalg.norm(b)
        rows.append(dict(seed=seed, scale=0, iterations=info["iterations"], status=info["status"],
                         rel_res=info["rel_res"], rel_res_true=float(true)))
    # A's values scaled by c = 1 + j 2^-52: in exact arithmetic the hierarchy
    # scales by c and the iterates by 1/c, so relative residuals do not move;
    # in floating point every rounding of the setup and the solve changes
    for j in OP_SCALES:
        c = 1.0 + j * 2.0**-52
        ps = dataclasses.replace(prob, val=prob.val * c)
        hs = oracle.Hierarchy(ps)
        x, info = hs.pcg(ps.b, maxit=1000)
        true = np.linalg.norm(ps.b - oracle.spmv(ps.rowptr, ps.col, ps.val, x)) / np.linalg.norm(ps.b)
        rows.append(dict(seed=None, scale=j, iterations=info["iterations"], status=info["status"],
                         rel_res=info["rel_res"], rel_res_true=float(true)))
    return dict(request=req["id"], runs=rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--ulp", action="store_true")
    ap.add_argument("--add", action="store_true")
    args = ap.parse_args()
    from workloads import serving_stream

    if args.add:
        with open(OUT) as f:
            rec = json.load(f)
        have = {c["request"] for c in rec["cases"]}
        more = [r for r in serving_stream(num=256, rate=20.0)
                if r["kind"] == "layered" and r["n"] > 64 and r["id"] not in have]
        more.sort(key=lambda r: -r["n"])
        with mp.get_context("spawn").Pool(args.workers) as pool:
            rows = pool.map(run, more, chunksize=1)
        rec["cases"] = sorted(rec["cases"] + rows, key=lambda r: r["request"])
        rec["stream"] = "serving_stream(num=256, rate=20.0, seed=0), every layered request"
        with open(OUT, "w") as f:
            json.dump(rec, f, indent=1)
        print(f"{sum(r['status'] != 0 for r in rows)} of {len(rows)} added requests not converged")
        return

    reqs = [r for r in serving_stream(num=256, rate=20.0) if r["kind"] == "layered" and r["n"] <= 64]
    if args.ulp:
        with open(OUT) as f:
            conv, stuck = selected(json.load(f)["cases"])
        want = set(conv) | set(stuck)
        sub = sorted((r for r in reqs if r["id"] in want), key=lambda r: -r["n"])
        with mp.get_context("spawn").Pool(args.workers) as pool:
            rows = pool.map(run_ulp, sub, chunksize=1)
        rows.sort(key=lambda r: r["request"])
        with open(ULP_OUT, "w") as f:
            json.dump(dict(converged=conv, stopped=stuck, ulp_seeds=list(ULP_SEEDS), op_scales=list(OP_SCALES),
                           max_iter=1000, tol=1e-8,
                           cases=rows), f, indent=1)
        print(f"{len(rows)} requests, seven solves each")
        return
    reqs.sort(key=lambda r: -r["n"])
    with mp.get_context("spawn").Pool(args.workers) as pool:
        rows = pool.map(run, reqs, chunksize=1)
    rows.sort(key=lambda r: r["request"])
    with open(OUT, "w") as f:
        json.dump(dict(stream="serving_stream(num=256, rate=20.0, seed=0), layered requests with n <= 64",
                       max_iter=1000, tol=1e-8, cases=rows), f, indent=1)
    print(f"{sum(r['status'] != 0 for r in rows)} of {len(rows)} not converged")


if __name__ == "__main__":
    main()
