"""Pins of the oracle's Clement interpolant and material strength of connection.

The closed forms below are derived by hand from the definitions of the distance
Laplacian and the material distance (sections "Strength-of-connection measures
and dropping criteria" and "A material based strength-of-connection measure")
on the 5x5-node two-material grid of the paper's test-problem figure
(nodes numbered 1..25 row-major from the bottom left, low material for x < 1.5,
high material for x > 1.5, 9-point pattern, pointwise nodal sigma).
"""

import math

import numpy as np
import pytest

import oracle
from workloads import box_mesh, poisson_box
from workloads.q1 import config1_checkerboard_2d, rotated_anisotropic_3d


def fig4_grid(kappa, anisotropic=False):
    prob = poisson_box((4, 4), lengths=(4.0, 4.0), dirichlet="none")
    x = prob.coords
    sig = np.zeros((prob.n, 3))
    low = x[:, 0] < 1.5
    sig[low] = [1.0, 0.0, 1.0]
    sig[~low] = [kappa, 0.0, kappa] if not anisotropic else [kappa, 0.0, 1.0]
    return prob, x, sig


def entry(prob, S, i, j):
    """S at (node i, node j) with 1-based node numbers of the figure."""
    i0, j0 = i - 1, j - 1
    lo, hi = prob.rowptr[i0], prob.rowptr[i0 + 1]
    k = lo + np.searchsorted(prob.col[lo:hi], j0)
    assert prob.col[k] == j0
    return S[k]


@pytest.mark.parametrize("kappa", [1.0, 1e2, 1e4, 1e8])
def test_fig4_scalar_closed_forms(kappa):
    prob, x, sig = fig4_grid(kappa)
    lv, ld, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, x, sig, soc="material", theta=0.08)
    assert ld[11] == pytest.approx(6.0, rel=1e-15)                     # L_12,12
    assert ld[12] == pytest.approx(4 * kappa + 2, rel=1e-15)           # L_13,13
    assert entry(prob, S, 12, 11) == pytest.approx(1 / math.sqrt(24), rel=1e-14)
    assert entry(prob, S, 12, 13) == pytest.approx(1 / math.sqrt(6 * (4 * kappa + 2)), rel=1e-14)
    # S_13,14 = kappa / sqrt((4 kappa + 2) 6 kappa)
    assert entry(prob, S, 13, 14) == pytest.approx(kappa / math.sqrt((4 * kappa + 2) * 6 * kappa), rel=1e-14)
    # the low/high edge decays like kappa^{-1/2} (eq. low_high_soc_parameter_relation)
    if kappa >= 1e4:
        assert entry(prob, S, 12, 13) * math.sqrt(kappa) == pytest.approx(1 / math.sqrt(24), rel=1e-3)


@pytest.mark.parametrize("kappa", [1e2, 1e4])
def test_fig4_anisotropic_closed_forms(kappa):
    prob, x, sig = fig4_grid(kappa, anisotropic=True)
    lv, ld, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, x, sig, soc="material", theta=0.08)
    l13 = kappa + 4 + 2 * kappa / (kappa + 1)
    l14 = 2 * kappa + 2 + 4 * kappa / (kappa + 1)
    assert ld[12] == pytest.approx(l13, rel=1e-14)
    assert ld[13] == pytest.approx(l14, rel=1e-14)
    assert entry(prob, S, 12, 13) == pytest.approx(1 / math.sqrt(6 * l13), rel=1e-14)
    assert entry(prob, S, 13, 14) == pytest.approx(kappa / math.sqrt(l13 * l14), rel=1e-14)
    # vertical edge inside the high region is weak: ~1/kappa -> semi-coarsening in x
    assert entry(prob, S, 13, 8) == pytest.approx(1 / l13, rel=1e-14)


def test_fig4_drop_at_kappa_100():
    prob, x, sig = fig4_grid(100.0)
    _, _, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, x, sig, soc="material", theta=0.08)
    assert not entry(prob, mask.astype(float), 12, 13)   # interface edge dropped
    assert entry(prob, mask.astype(float), 12, 11)       # low-low edge kept


def test_full_tensor_quadratic_form_matches_inverse():
    """l_ij = 1/max(q_i, q_j), q = d^T sigma^{-1} d with a full SPD tensor."""
    rng = np.random.default_rng(7)
    prob = poisson_box((3, 3, 3), dirichlet="none")
    n = prob.n
    sig = np.zeros((n, 6))
    full = []
    for i in range(n):
        B = rng.normal(size=(3, 3))
        T = B @ B.T + 0.5 * np.eye(3)
        full.append(T)
        sig[i] = [T[0, 0], T[0, 1], T[0, 2], T[1, 1], T[1, 2], T[2, 2]]
    x = prob.coords + rng.normal(scale=0.05, size=prob.coords.shape)
    lv, ld, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 3, x, sig, soc="material")
    for i in range(n):
        for k in range(prob.rowptr[i], prob.rowptr[i + 1]):
            j = prob.col[k]
            if j == i:
                continue
            d = x[j] - x[i]
            q = max(d @ np.linalg.solve(full[i], d), d @ np.linalg.solve(full[j], d))
            assert lv[k] == pytest.approx(1.0 / q, rel=1e-12)
        assert ld[i] == pytest.approx(sum(lv[prob.rowptr[i]:prob.rowptr[i + 1]]), rel=1e-14)


def test_strength_invariants_on_checkerboard():
    prob = config1_checkerboard_2d(n=16, cells=4)
    sig = oracle.clement(prob.n, 2, prob.elem_nodes, prob.elem_sigma)
    d = oracle.detect_dirichlet(prob.rowptr, prob.col, prob.val)
    assert np.array_equal(d, prob.dirichlet)
    lv, ld, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, prob.coords, sig, dirichlet=d)
    rows = np.repeat(np.arange(prob.n), np.diff(prob.rowptr))
    diag = rows == prob.col
    assert np.all(S[diag] == 1.0)
    off = ~diag & ~d[rows] & ~d[prob.col]
    assert np.all(S[off] > 0) and np.all(S[off] <= 1.0 + 1e-15)
    # bitwise symmetry of |L| and of the mask
    key = {(int(r), int(c)): k for k, (r, c) in enumerate(zip(rows, prob.col))}
    for k, (r, c) in enumerate(zip(rows, prob.col)):
        kt = key[(int(c), int(r))]
        assert lv[k] == lv[kt]
        assert mask[k] == mask[kt]
    # the square-free test agrees with S >= theta away from ties
    far = off & (np.abs(S - 0.08) > 1e-12)
    assert np.array_equal(mask[far], S[far] >= 0.08)
    # Dirichlet rows/cols keep no edge
    assert not np.any(mask[~diag & (d[rows] | d[prob.col])])


def test_constant_sigma_material_equals_distance_laplacian():
    """With sigma = c I (c a power of two) the material measure is the Euclidean
    distance Laplacian measure exactly (S is scale invariant)."""
    prob = rotated_anisotropic_3d(n=4, block=2)
    sig = np.tile([4.0, 0, 0, 4.0, 0, 4.0], (prob.n, 1))
    _, _, S1, m1 = oracle.strength(prob.rowptr, prob.col, prob.val, 3, prob.coords, sig, soc="material")
    _, _, S2, m2 = oracle.strength(prob.rowptr, prob.col, prob.val, 3, prob.coords, sig, soc="distance")
    assert np.array_equal(S1, S2) and np.array_equal(m1, m2)


def test_classical_sa_measure():
    prob = poisson_box((4, 4), dirichlet="none")
    lv, ld, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, prob.coords,
                                      np.ones((prob.n, 3)), soc="sa", theta=0.1)
    A = prob.dense()
    rows = np.repeat(np.arange(prob.n), np.diff(prob.rowptr))
    ref = np.abs(A[rows, prob.col]) / np.sqrt(np.abs(A[rows, rows] * A[prob.col, prob.col]))
    assert np.allclose(S, ref, rtol=1e-14, atol=0)


def test_clement_constant_and_interface():
    from workloads.q1 import layered_stack_3d
    prob = layered_stack_3d(n=4, repeats=1)
    sig = oracle.clement(prob.n, 3, prob.elem_nodes, prob.elem_sigma)
    # node on the first layer boundary: mean of 4 elements below and 4 above
    kz = prob.meta["layer_k"]
    zi = np.rint(prob.coords[:, 2] * 4).astype(int)
    ix = np.rint(prob.coords[:, 0] / prob.lengths[0] * 4).astype(int)
    iy = np.rint(prob.coords[:, 1] / prob.lengths[1] * 4).astype(int)
    interior = (ix > 0) & (ix < 4) & (iy > 0) & (iy < 4)
    for i in np.nonzero(interior & (zi == 1))[0]:
        assert sig[i, 0] == pytest.approx((4 * kz[0] + 4 * kz[1]) / 8, rel=1e-15)
        assert sig[i, 1] == 0.0 and sig[i, 2] == 0.0
        assert sig[i, 3] == sig[i, 0] and sig[i, 5] == sig[i, 0]
    # constant tensors are reproduced exactly, and component order is the upper triangle
    T = np.array([[3.0, 0.5, -0.25], [0.5, 2.0, 0.125], [-0.25, 0.125, 1.0]])
    es = np.repeat(T[None], prob.nelem, axis=0)
    sig = oracle.clement(prob.n, 3, prob.elem_nodes, es)
    assert np.all(sig == np.array([3.0, 0.5, -0.25, 2.0, 0.125, 1.0]))


def test_clement_2d_corner_edge_counts():
    coords, en = box_mesh((2, 2), (1.0, 1.0))
    es = np.zeros((4, 2, 2))
    for e in range(4):
        es[e] = (e + 1.0) * np.eye(2)
    sig = oracle.clement(9, 2, en, es)
    # centre node touches all four elements; corner node 0 only element 0
    assert sig[4, 0] == (1 + 2 + 3 + 4) / 4
    assert sig[0, 0] == 1.0 and sig[8, 0] == 4.0
    assert sig[1, 0] == (1 + 2) / 2


# ----------------------------------------------------------------- cut-drop
def literal_cut_drop(prob, S, dirichlet, theta):
    """The cut-drop criterion as the paper states it, on the strength values
    S (with the square root): per row, order the off-diagonal |S_ij|
    decreasingly, k = first position with theta*s_k >= s_{k+1}, keep
    |S_ij| >= s_k (everything if no such k) and the diagonal; then keep (i, j)
    only if both rows keep it.  Edges touching a Dirichlet node are dropped."""
    n = prob.n
    keep = np.zeros(len(prob.col), dtype=bool)
    for i in range(n):
        lo, hi = prob.rowptr[i], prob.rowptr[i + 1]
        if dirichlet[i]:
            keep[lo:hi] = prob.col[lo:hi] == i
            continue
        ks = [k for k in range(lo, hi) if prob.col[k] != i and not dirichlet[prob.col[k]]]
        keep[lo:hi] = prob.col[lo:hi] == i
        vals = sorted((abs(S[k]) for k in ks), reverse=True)
        cut = -1.0
        for p in range(len(vals) - 1):
            if theta * vals[p] >= vals[p + 1]:
                cut = vals[p]
                break
        for k in ks:
            keep[k] = prob.col[k] == i or abs(S[k]) >= cut
    mask = np.zeros_like(keep)
    for i in range(n):
        for k in range(prob.rowptr[i], prob.rowptr[i + 1]):
            j = prob.col[k]
            lo, hi = prob.rowptr[j], prob.rowptr[j + 1]
            kt = lo + np.searchsorted(prob.col[lo:hi], i)
            mask[k] = keep[k] and keep[kt]
    return mask


def test_cut_drop_uniform_material_keeps_every_edge():
    prob, x, sig = fig4_grid(1.0)
    _, _, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, x, sig, soc="material", theta=0.08,
                                    drop="cut")
    assert mask.all()


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e8])
def test_cut_drop_fig4_drops_the_interface_only(kappa):
    prob, x, sig = fig4_grid(kappa)
    _, _, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, x, sig, soc="material", theta=0.08,
                                    drop="cut")
    m = mask.astype(float)
    # node 12 (low side): its low-low edges stay; the low-high edge has the
    # closed form 1/sqrt(6 (4 kappa + 2)), i.e. 1/sqrt(24) * kappa^{-1/2} against
    # 1/sqrt(24) for the low-low edge: a gap below theta = 0.08 opens only
    # once kappa^{-1/2} < 0.08 (kappa = 1e2 gives 0.1: nothing is cut)
    assert entry(prob, m, 12, 11) and entry(prob, m, 12, 7) and entry(prob, m, 12, 17)
    cut = kappa ** -0.5 < 0.08
    assert bool(entry(prob, m, 12, 13)) != cut
    assert bool(entry(prob, m, 12, 8)) != cut and bool(entry(prob, m, 12, 18)) != cut
    # inside the high region every edge is kept (no gap there)
    assert entry(prob, m, 14, 15) and entry(prob, m, 14, 9) and entry(prob, m, 14, 19)
    assert np.array_equal(mask, literal_cut_drop(prob, S, np.zeros(prob.n, bool), 0.08))


@pytest.mark.parametrize("soc", ["material", "distance", "sa"])
@pytest.mark.parametrize("theta", [0.08, 0.3, 0.6])
def test_cut_drop_equals_the_literal_definition(soc, theta):
    """Random full SPD tensors, jittered coordinates and Dirichlet faces: the
    square-free evaluation equals the literal sorted definition."""
    rng = np.random.default_rng(11)
    prob = rotated_anisotropic_3d(n=6, block=2, seed=3)
    n = prob.n
    sig = oracle.clement(n, 3, prob.elem_nodes, prob.elem_sigma)
    sig = sig * rng.uniform(0.5, 2.0, size=(n, 1)) ** 2
    x = prob.coords + rng.normal(scale=0.01, size=prob.coords.shape)
    d = oracle.detect_dirichlet(prob.rowptr, prob.col, prob.val)
    _, _, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 3, x, sig, dirichlet=d, soc=soc,
                                    theta=theta, drop="cut")
    ref = literal_cut_drop(prob, S, d, theta)
    assert np.array_equal(mask, ref)
    # symmetric, diagonal kept, nothing strong at a Dirichlet node
    rows = np.repeat(np.arange(n), np.diff(prob.rowptr))
    M = np.zeros((n, n), dtype=bool)
    M[rows, prob.col] = mask
    assert np.array_equal(M, M.T)
    assert M[np.arange(n), np.arange(n)].all()
    off = M & ~np.eye(n, dtype=bool)
    assert not off[d].any()


def test_cut_drop_with_theta_one_keeps_the_largest_only():
    """theta = 1: the first gap follows the largest value, so each row keeps
    only its strongest off-diagonal entries (all of them on a tie); an edge
    survives when it is the strongest for both of its nodes."""
    prob = config1_checkerboard_2d(n=8, cells=2)
    sig = oracle.clement(prob.n, 2, prob.elem_nodes, prob.elem_sigma)
    d = oracle.detect_dirichlet(prob.rowptr, prob.col, prob.val)
    _, _, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, prob.coords, sig, dirichlet=d,
                                    theta=1.0, drop="cut")
    n = prob.n
    rows = np.repeat(np.arange(n), np.diff(prob.rowptr))
    ordered = (rows != prob.col) & ~d[rows] & ~d[prob.col]
    best = np.zeros(n)
    np.maximum.at(best, rows[ordered], np.abs(S[ordered]))
    strongest = np.zeros((n, n), dtype=bool)
    strongest[rows[ordered], prob.col[ordered]] = np.abs(S[ordered]) == best[rows[ordered]]
    expect = (strongest & strongest.T)[rows, prob.col] | (rows == prob.col)
    assert np.array_equal(mask, expect)
    assert (mask & (rows != prob.col)).any()


def test_cut_drop_uniform_grid_closed_form():
    """Uniform 2D Q1 grid, isotropic material: an interior row has four axis
    edges with S = 1/6 and four diagonal edges with S = 1/12 (distance
    Laplacian weights 1/h^2 and 1/(2h^2), L_ii = 6/h^2).  The single gap, of
    ratio 1/2, opens once theta > 1/2: below that every edge stays, above it
    only the axis edges do.  Pointwise dropping at such tolerances keeps no
    edge at all (1/6 < theta)."""
    prob = poisson_box((10, 10), lengths=(1.0, 1.0), dirichlet="none")
    x = prob.coords
    n = prob.n
    sig = np.tile([1.0, 0.0, 1.0], (n, 1))
    rows = np.repeat(np.arange(n), np.diff(prob.rowptr))
    side = 11
    ix, iy = np.arange(n) % side, np.arange(n) // side
    interior = (ix > 1) & (ix < side - 2) & (iy > 1) & (iy < side - 2)
    sel = interior[rows] & (rows != prob.col)
    axis = (ix[rows] == ix[prob.col]) | (iy[rows] == iy[prob.col])
    for theta, keep_diag in ((0.4, True), (0.49, True), (0.51, False), (0.64, False)):
        _, _, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 2, x, sig, soc="material",
                                        theta=theta, drop="cut")
        assert np.allclose(np.abs(S[sel & axis]), 1 / 6, rtol=1e-14)
        assert np.allclose(np.abs(S[sel & ~axis]), 1 / 12, rtol=1e-14)
        assert mask[sel & axis].all()
        assert bool(mask[sel & ~axis].all()) == keep_diag and bool(mask[sel & ~axis].any()) == keep_diag
        _, _, _, pw = oracle.strength(prob.rowptr, prob.col, prob.val, 2, x, sig, soc="material",
                                      theta=theta, drop="pointwise")
        assert not pw[sel].any()
