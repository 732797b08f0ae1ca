"""GPU: new values of A on a kept coarsening (amg_update_values) against the
oracle's reuse setup and against fresh setups."""

import dataclasses
import sys

import numpy as np
import pytest

import oracle
from workloads.q1 import config1_checkerboard_2d, layered_stack_3d, rotated_anisotropic_3d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amg():
    import torch

    import paper_2602_05686_amd as amg

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    amg.load()
    return amg


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def scaled(prob, c):
    return dataclasses.replace(prob, val=prob.val * c, b=prob.b * c, elem_sigma=prob.elem_sigma * c)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_scaled_update_is_bitwise_a_fresh_setup(amg, precision):
    """sigma and A times 4 (exact in floating point) keep every mask and
    aggregate, so the update must give bit for bit the hierarchy and the
    solve of a fresh setup on the scaled problem."""
    banner(f"update: layered 16^3 scaled by 4, {precision}")
    prob = layered_stack_3d(n=16, repeats=4)
    p4 = scaled(prob, 4.0)
    h = amg.Hierarchy.from_problem(prob, max_coarse=100, precision=precision)
    h.solve(prob.b)  # captures the CG graphs before the update
    h.update_values(p4.val)
    f = amg.Hierarchy.from_problem(p4, max_coarse=100, precision=precision)
    sh, sf = h.stats(), f.stats()
    assert sh["levels"] == sf["levels"] >= 3
    assert sh["omega"] == sf["omega"] and sh["lam_cheb"] == sf["lam_cheb"]
    assert sh["t_update_s"] > 0.0
    for l in range(sh["levels"]):
        for which in (("A",) if l + 1 == sh["levels"] else ("A", "P", "R")):
            a, b = h.level_csr(l, which), f.level_csr(l, which)
            for u, v in zip(a, b):
                assert np.array_equal(u, v), (l, which)
    xh, ih = h.solve(p4.b)
    xf, if_ = f.solve(p4.b)
    assert ih["iterations"] == if_["iterations"] and np.array_equal(xh, xf)
    h.close()
    f.close()


def test_update_matches_the_oracle_reuse_setup(amg):
    """New random rotations on the same mesh: the update keeps the setup's
    coarsening and equals the oracle's reuse setup (patterns bitwise, values
    to round-off, iterations +-1, solution 1e-6).  A hierarchy that solved
    before its update must solve afterwards exactly as one updated before
    any solve (the captured CG steps are rebuilt)."""
    banner("update: rotated anisotropy 16^3, seed 0 -> seed 1")
    p0 = rotated_anisotropic_3d(n=16, block=4, seed=0)
    p1 = rotated_anisotropic_3d(n=16, block=4, seed=1)
    assert np.array_equal(p0.col, p1.col) and not np.array_equal(p0.val, p1.val)
    kw = dict(max_coarse=100)
    o0 = oracle.Hierarchy(p0, **kw)
    orr = oracle.Hierarchy(p1, reuse=o0)
    h = amg.Hierarchy.from_problem(p0, **kw)
    h.solve(p0.b)
    h.update_values(p1.val)
    g = amg.Hierarchy.from_problem(p0, **kw)
    g.update_values(p1.val)
    st = h.stats()
    assert st["levels"] == orr.nlev
    for l in range(orr.nlev):
        rp, ci, va = h.level_csr(l, "A")
        orp, oci, ova = orr.level_csr(l, "A")
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
        assert np.max(np.abs(va - ova)) <= 1e-10 * np.max(np.abs(ova)), f"A values on level {l}"
        if l + 1 < orr.nlev:
            assert np.array_equal(h.aggregates(l), orr.get(l, "agg"))
            assert np.array_equal(h.soc_mask(l), orr.get(l, "mask"))
            prp, pci, pva = h.level_csr(l, "P")
            orp, oci, ova = orr.level_csr(l, "P")
            assert np.array_equal(prp, orp) and np.array_equal(pci, oci)
            assert np.max(np.abs(pva - ova)) <= 1e-10, f"P values on level {l}"
            assert st["omega"][l] == pytest.approx(orr.info(l)["omega"], rel=1e-10)
            assert st["lam_cheb"][l] == pytest.approx(orr.info(l)["lam_cheb"], rel=1e-10)
    xo, io = orr.pcg(p1.b)
    x, info = h.solve(p1.b)
    xg, ig = g.solve(p1.b)
    print(f"update: iterations gpu={info['iterations']} oracle={io['iterations']}")
    assert info["status"] == "OK" and abs(info["iterations"] - io["iterations"]) <= 1
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-6
    assert ig["iterations"] == info["iterations"] and np.array_equal(x, xg)
    h.close()
    g.close()


def test_update_rejects_a_changed_dirichlet_set_and_keeps_the_hierarchy(amg):
    banner("update: changed Dirichlet set is refused")
    prob = config1_checkerboard_2d(n=32, cells=4)
    h = amg.Hierarchy.from_problem(prob, max_coarse=40)
    x0, i0 = h.solve(prob.b)
    val = prob.val.copy()
    i = int(np.flatnonzero(~prob.dirichlet)[7])
    lo, hi = prob.rowptr[i], prob.rowptr[i + 1]
    row = val[lo:hi]
    row[prob.col[lo:hi] != i] = 0.0
    with pytest.raises(amg.AmgError):
        h.update_values(val)
    x1, i1 = h.solve(prob.b)
    assert i1["iterations"] == i0["iterations"] and np.array_equal(x0, x1)
    h.close()
