"""Writes <workload>_oracle_spread.json: how far the oracle's own hierarchy
moves under rounding-level changes of its input.

The input values of A are scaled by c = 1 + j 2^-52 (j = 1, 2, 3).  In exact
arithmetic this changes nothing but a factor: the strength measure, masks
and aggregates do not read A's values; the damping factors, spectral
estimates and prolongators are invariant; every coarse operator scales by c.
In floating point every rounding changes, so the differences below are the
oracle's sensitivity to rounding, level by level:

  omega, lam_pf, lam_cheb   max over j of |x_j - x| / |x|
  A, P, R                   max over j of the row-scaled difference of the
                            values (A_j / c against A), each row's largest
                            entry as its scale
  vcycle                    max over j of |c z_j - z| / |z| for one V-cycle
                            z = M^{-1} r of r ~ N(0, 1) from default_rng(5)
                            (the preconditioner scales by 1/c)

The GPU parity tests hold the library's hierarchy to these spreads (times a
safety factor) on the levels where they exceed round-off.  Only the oracle
and the input generators run here.  From the repository root:

    python tests/golden/make_oracle_spread.py layered128 [layered192]
"""

import dataclasses
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

HERE = os.path.dirname(os.path.abspath(__file__))

WORKLOADS = {
    "layered128": (lambda q1: q1.layered_stack_3d(n=128, repeats=20, stretch=10.0), {}),
    "layered192": (lambda q1: q1.layered_stack_3d(n=192, repeats=50, stretch=20.0, config_id=4),
                   {"max_levels": 16}),
    "aniso96": (lambda q1: q1.rotated_anisotropic_3d(n=96, block=8), {}),
}


def level_values(h, l):
    out = {"A": h.level_csr(l, "A")}
    if l + 1 < h.nlev:
        out["P"] = h.level_csr(l, "P")
        out["R"] = h.level_csr(l, "R")
    return out


def main(name):
    import oracle
    from parity_util import row_scaled_diff
    from workloads import q1

    make, kw = WORKLOADS[name]
    prob = make(q1)
    base = oracle.Hierarchy(prob, **kw)
    nlev = base.nlev
    r = np.random.default_rng(5).standard_normal(prob.n)
    z = base.vcycle(r)
    vspread = 0.0
    spread = [dict(omega=0.0, lam_pf=0.0, lam_cheb=0.0, A=0.0, P=0.0, R=0.0) for _ in range(nlev)]
    for j in (1, 2, 3):
        c = 1.0 + j * 2.0**-52
        h = oracle.Hierarchy(dataclasses.replace(prob, val=prob.val * c), **kw)
        assert h.nlev == nlev
        for l in range(nlev):
            s = spread[l]
            if l + 1 < nlev:
                a, b = base.info(l), h.info(l)
                for key in ("omega", "lam_pf", "lam_cheb"):
                    s[key] = max(s[key], abs(b[key] - a[key]) / abs(a[key]) if a[key] else abs(b[key]))
            va, vb = level_values(base, l), level_values(h, l)
            for key in va:
                rp, ci, x = va[key]
                rq, cj, y = vb[key]
                assert np.array_equal(rp, rq) and np.array_equal(ci, cj)
                if key == "A":
                    y = y / c
                s[key] = max(s[key], row_scaled_diff(rp, y, x))
        vspread = max(vspread, float(np.linalg.norm(c * h.vcycle(r) - z) / np.linalg.norm(z)))
        del h
        print(f"{name}: scale {j} done", flush=True)
    out = dict(workload=name, levels=[base.info(l)["n"] for l in range(nlev)], spread=spread, vcycle=vspread)
    with open(os.path.join(HERE, f"{name}_oracle_spread.json"), "w") as f:
        json.dump(out, f, indent=1)
    for l, s in enumerate(spread):
        print(l, {k: f"{v:.1e}" for k, v in s.items()})
    print(f"V-cycle {vspread:.1e}")


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        main(arg)
