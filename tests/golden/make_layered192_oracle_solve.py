"""Writes layered192_oracle_solve.json: the oracle's PCG solve on the 192^3
layered stack (7,189,057 DOF, 50 repeats of three layers, 20:1 flat
elements, theta 0.08, 16 levels, CG from x0 = 0 to a relative residual of
1e-8 with at most 4000 iterations).

Recorded: the exit iteration and status, the solver's and the recomputed
true relative residual, the relative error against the series-resistor
profile (which is not the discrete solution here: 150 layers do not align
with 192 elements) and the solution at 4096 seeded positions
(default_rng(192) without replacement), so that a GPU solve can be held to
the oracle's accuracy and compared with its solution.  Only the oracle and
the input generators run here (one core, about three hours).  From the
repository root:

    python tests/golden/make_layered192_oracle_solve.py
"""

import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "layered192_oracle_solve.json")
SAMPLES = 4096


def exact(prob):
    kz = prob.meta["layer_k"]
    res = 1.0 / kz
    cf = np.concatenate([[0.0], np.cumsum(res)]) / res.sum()
    return cf[np.rint(prob.coords[:, 2] * prob.shape[2]).astype(int)]


def main():
    import oracle
    from workloads.q1 import layered_stack_3d, problem_digest

    prob = layered_stack_3d(n=192, repeats=50, stretch=20.0, config_id=4)
    t = time.time()
    h = oracle.Hierarchy(prob, max_levels=16)
    t_setup = time.time() - t
    print(f"setup {t_setup:.0f} s, levels {h.stats()['n']}", flush=True)
    t = time.time()
    x, info = h.pcg(prob.b, maxit=4000)
    t_solve = time.time() - t
    r = prob.b - oracle.spmv(prob.rowptr, prob.col, prob.val, x)
    ex = exact(prob)
    idx = np.sort(np.random.default_rng(192).choice(prob.n, size=SAMPLES, replace=False))
    out = dict(workload="layered stack 192^3, 50 repeats x 3 layers, 20:1 flat, theta 0.08, 16 levels, tol 1e-8, "
                        "at most 4000 iterations",
               input_sha256=problem_digest(prob), host=platform.processor() or platform.machine(),
               levels=h.stats()["n"], iterations=info["iterations"], status=info["status"], rel_res=info["rel_res"],
               rel_res_true=float(np.linalg.norm(r) / np.linalg.norm(prob.b)),
               err_vs_exact=float(np.linalg.norm(x - ex) / np.linalg.norm(ex)),
               setup_s=round(t_setup, 1), solve_s=round(t_solve, 1),
               sample_rng="default_rng(192).choice(n, 4096, replace=False), sorted", sample_index=idx.tolist(),
               sample_x=x[idx].tolist())
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if not k.startswith("sample_")}), flush=True)


if __name__ == "__main__":
    main()
