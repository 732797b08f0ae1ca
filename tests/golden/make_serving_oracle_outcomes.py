"""Writes serving_oracle_outcomes.json: the oracle's PCG outcome (FP64, tol
1e-8, at most 1000 iterations, the server's cap) on every layered request of
the seeded serving stream (256 requests, seed 0) with at most 64 elements
per side -- the thin stacks (60 layers on 32 to 64 elements) on which the
server reports NOT_CONVERGED -- so that the server's failures can be matched
against the oracle's.  Only the oracle and the input generators run here.
From the repository root:

    python tests/golden/make_serving_oracle_outcomes.py [--workers 6]
"""

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "serving_oracle_outcomes.json")


def run(req):
    import oracle
    from workloads import problem_from_request

    prob = problem_from_request(req)
    t = time.time()
    h = oracle.Hierarchy(prob)
    _, info = h.pcg(prob.b, maxit=1000)
    return dict(request=req["id"], n=req["n"], dof=prob.n, iterations=info["iterations"], status=info["status"],
                rel_res=info["rel_res"], seconds=round(time.time() - t, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    args = ap.parse_args()
    from workloads import serving_stream

    reqs = [r for r in serving_stream(num=256, rate=20.0) if r["kind"] == "layered" and r["n"] <= 64]
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
