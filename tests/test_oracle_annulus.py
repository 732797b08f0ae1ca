"""Pins of the oracle on the anisotropic annulus (section "Anisotropic
thermal diffusion", Figs. 8-9 and Table 1).

The paper shows that with a high circumferential conductivity the
material-weighted distance Laplacian keeps the circumferential connections
and drops the radial ones on the first level, so the first-level aggregates
are one-dimensional arcs (semi-coarsening along the strong direction), while
the homogeneous material (kappa = 1) aggregates in all directions.  The
meshes here are small enough for the oracle to finish in seconds.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from workloads import annulus_3d


def ring_index(prob):
    """(radial index, thickness index) of every node"""
    N0, N1 = prob.shape[0] + 1, prob.shape[1]
    ids = np.arange(prob.n)
    return ids % N0, ids // (N0 * N1)


@pytest.mark.parametrize("kappa,theta", [(1e2, 0.05), (1e4, 0.05), (1e4, 0.1)])
def test_strong_circumferential_anisotropy_semicoarsens(kappa, theta):
    prob = annulus_3d(0, kappa=kappa)
    h = oracle.Hierarchy(prob, theta=theta)
    mask = h.get(0, "mask")
    rows = np.repeat(np.arange(prob.n), np.diff(prob.rowptr))
    off = mask & (rows != prob.col)
    i, k = ring_index(prob)
    same_ring = (i[rows] == i[prob.col]) & (k[rows] == k[prob.col])
    # every kept off-diagonal edge runs around a ring, and every free node keeps its two ring neighbours
    assert np.all(same_ring[off])
    free = ~prob.dirichlet
    kept_per_row = np.bincount(rows[off], minlength=prob.n)
    assert np.all(kept_per_row[free] == 2)
    # so each aggregate is an arc of one ring
    agg = h.get(0, "agg")
    assert np.all(agg[prob.dirichlet] == -1) and np.all(agg[free] >= 0)
    key = i * 1000 + k
    for a in np.unique(agg[free]):
        assert np.unique(key[agg == a]).size == 1


def test_homogeneous_annulus_coarsens_in_every_direction():
    prob = annulus_3d(0, kappa=1.0)
    h = oracle.Hierarchy(prob, theta=0.05)
    agg = h.get(0, "agg")
    i, k = ring_index(prob)
    free = ~prob.dirichlet
    spans_rings = [np.unique((i * 1000 + k)[agg == a]).size > 1 for a in np.unique(agg[free])]
    assert np.mean(spans_rings) > 0.9
    # and coarsens much harder than the semi-coarsened kappa = 1e4 case
    n1 = h.info(1)["n"]
    h4 = oracle.Hierarchy(annulus_3d(0, kappa=1e4), theta=0.05)
    assert n1 < 0.5 * h4.info(1)["n"]


def test_annulus_pcg_reaches_the_direct_solution():
    prob = annulus_3d(0, kappa=1e4)
    h = oracle.Hierarchy(prob, theta=0.1)
    x, info = h.pcg(prob.b, tol=1e-10)
    assert info["status"] == oracle.OK
    A = sp.csr_matrix((prob.val, prob.col, prob.rowptr), shape=(prob.n, prob.n))
    xd = spla.spsolve(A.tocsc(), prob.b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-8
    # Dirichlet rows reproduce the data exactly
    assert np.allclose(x[prob.dirichlet], prob.g[prob.dirichlet], rtol=1e-12, atol=1e-14)
    # levels and coarsening target: the base mesh (6300 nodes) needs one coarsening to reach <= 5000
    st = h.stats()
    assert st["levels"] == 2 and st["n"][1] <= 5000 < st["n"][0]
