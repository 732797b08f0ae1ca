"""Pins of the oracle's setup for new values of A on a kept coarsening (a
material update that reuses the aggregates; the paper weighs the material
measure's setup cost against solves with a fixed hierarchy in its battery
results).

Everything that does not depend on A's values (coordinates, tensors, masks,
aggregates, depth) is kept; the value-dependent steps run on the new values.
"""

import dataclasses

import numpy as np
import pytest

import oracle
from workloads.q1 import config1_checkerboard_2d, layered_stack_3d

ARRAYS = ["A_rowptr", "A_col", "A_val", "P_rowptr", "P_col", "P_val", "R_rowptr", "R_col", "R_val", "agg", "mask",
          "x", "sig", "S", "dirichlet", "dinv"]


def dense(rowptr, col, val, ncols):
    n = rowptr.shape[0] - 1
    a = np.zeros((n, ncols))
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    np.add.at(a, (rows, col), val)
    return a


def level_arrays(h, l):
    names = ARRAYS if l + 1 < h.nlev else ["A_rowptr", "A_col", "A_val", "x", "sig", "dinv"]
    return {w: h.get(l, w) for w in names}


def test_reuse_with_the_same_values_is_the_setup():
    prob = config1_checkerboard_2d(n=32, cells=4)
    h = oracle.Hierarchy(prob, max_coarse=40)
    r = oracle.Hierarchy(prob, reuse=h)
    assert r.nlev == h.nlev
    for l in range(h.nlev):
        a, b = level_arrays(h, l), level_arrays(r, l)
        for w in a:
            assert np.array_equal(a[w], b[w]), (l, w)
        assert r.info(l) == h.info(l)
    assert np.array_equal(r.get(h.nlev - 1, "chol"), h.get(h.nlev - 1, "chol"))


def scaled(prob, c):
    return dataclasses.replace(prob, val=prob.val * c, b=prob.b * c, elem_sigma=prob.elem_sigma * c)


@pytest.mark.parametrize("soc", ["material", "sa"])
def test_scaled_material_reuse_equals_a_fresh_setup(soc):
    """Scaling sigma and A by 4 (a power of two, so every step scales
    exactly) leaves the strength measures, masks and aggregates unchanged; the
    kept-coarsening setup on 4A then equals a fresh setup on 4A bit for bit,
    and its coarse operators are exactly 4 times the original ones."""
    prob = layered_stack_3d(n=12, repeats=3)
    h = oracle.Hierarchy(prob, soc=soc, max_coarse=60)
    p4 = scaled(prob, 4.0)
    fresh = oracle.Hierarchy(p4, soc=soc, max_coarse=60)
    r = oracle.Hierarchy(p4, reuse=h)
    assert fresh.nlev == r.nlev == h.nlev >= 3
    for l in range(h.nlev):
        a, b = level_arrays(fresh, l), level_arrays(r, l)
        for w in a:
            if w == "sig":
                continue  # the kept tensors are the original material's
            assert np.array_equal(a[w], b[w]), (l, w)
        assert np.array_equal(r.get(l, "A_val"), 4.0 * h.get(l, "A_val"))
        if l + 1 < h.nlev:
            assert np.array_equal(r.get(l, "P_val"), h.get(l, "P_val"))
            assert r.info(l) == fresh.info(l)
    assert np.array_equal(r.get(h.nlev - 1, "sig"), h.get(h.nlev - 1, "sig"))


def test_new_material_on_the_kept_coarsening():
    """New layer conductivities: masks and aggregates stay those of the
    original setup while a fresh setup would choose others; P follows the
    dense formula (filtered matrix of the new A under the kept mask), the
    coarse operator is P^T A P, and the preconditioner still converges."""
    prob0 = layered_stack_3d(n=10, repeats=3, seed=0)
    prob1 = layered_stack_3d(n=10, repeats=3, seed=1)
    assert np.array_equal(prob0.col, prob1.col) and not np.array_equal(prob0.val, prob1.val)
    h = oracle.Hierarchy(prob0, max_coarse=40)
    r = oracle.Hierarchy(prob1, reuse=h)
    fresh = oracle.Hierarchy(prob1, max_coarse=40)
    assert any(not np.array_equal(fresh.get(l, "mask"), h.get(l, "mask"))
               for l in range(min(fresh.nlev, h.nlev) - 1))
    n = prob1.n
    A = prob1.dense()
    mask, agg = r.get(0, "mask"), r.get(0, "agg")
    assert np.array_equal(mask, h.get(0, "mask")) and np.array_equal(agg, h.get(0, "agg"))
    nc = r.info(0)["nc"]
    rows = np.repeat(np.arange(n), np.diff(prob1.rowptr))
    keep = np.zeros((n, n), bool)
    keep[rows, prob1.col] = mask
    AF = np.where(keep, A, 0.0)
    np.fill_diagonal(AF, 0.0)
    AF[np.arange(n), np.arange(n)] = A.sum(1) - AF.sum(1)
    Dt = np.abs(AF).sum(1)
    rowabs = np.abs(A).sum(1)
    kept_off = np.abs(np.where(keep & ~np.eye(n, dtype=bool), A, 0.0)).sum(1)
    Dt[(Dt <= 2.0**-46 * rowabs) | ((kept_off <= 2.0**-46 * rowabs) & ~prob1.dirichlet)] = 0.0
    Dtinv = np.where(Dt > 0, 1.0 / np.where(Dt > 0, Dt, 1.0), 0.0)
    Phat = np.zeros((n, nc))
    Phat[agg >= 0, agg[agg >= 0]] = 1.0
    omega = r.info(0)["omega"]
    assert omega == pytest.approx((4.0 / 3.0) / r.info(0)["lam_pf"], rel=1e-15)
    assert omega != h.info(0)["omega"]
    P = dense(*r.level_csr(0, "P"), nc)
    assert np.allclose(P, Phat - omega * (AF * Dtinv[:, None]) @ Phat, rtol=0, atol=1e-13)
    Ac = dense(*r.level_csr(1, "A"), nc)
    ref = P.T @ A @ P
    assert np.allclose(Ac, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    x, info = r.pcg(prob1.b, tol=1e-8, maxit=1000)
    assert info["status"] == oracle.OK
    assert np.linalg.norm(prob1.b - A @ x) <= 1e-8 * np.linalg.norm(prob1.b)


def test_reuse_rejects_a_different_pattern_or_dirichlet_set():
    prob = config1_checkerboard_2d(n=16, cells=4)
    h = oracle.Hierarchy(prob, max_coarse=40)
    other = config1_checkerboard_2d(n=17, cells=1)
    with pytest.raises(oracle.OracleError):
        oracle.Hierarchy(other, reuse=h)
    # a free row whose off-diagonals become exact zeros turns into a Dirichlet row
    val = prob.val.copy()
    i = int(np.flatnonzero(~prob.dirichlet)[5])
    lo, hi = prob.rowptr[i], prob.rowptr[i + 1]
    off = prob.col[lo:hi] != i
    val[lo:hi][off] = 0.0
    with pytest.raises(oracle.OracleError):
        oracle.Hierarchy(dataclasses.replace(prob, val=val), reuse=h)
