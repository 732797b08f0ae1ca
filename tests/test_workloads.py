"""Input generators: the row-streamed C assembler reproduces the numpy
assembly bit for bit, and the request stream has the stated statistics."""

import math

import numpy as np
import pytest

import workloads.q1 as q1
from workloads import layered_stack_3d, poisson_box, rotated_anisotropic_3d, serving_stream

FIELDS = ["rowptr", "col", "val", "b", "coords", "elem_nodes", "elem_sigma", "dirichlet", "g"]


def numpy_only(fn, **kw):
    orig = q1._fast_lib
    q1._fast_lib = lambda: None
    try:
        return fn(**kw)
    finally:
        q1._fast_lib = orig


@pytest.mark.parametrize("fn,kw", [
    (layered_stack_3d, dict(n=12, repeats=3)),
    (layered_stack_3d, dict(shape=(9, 7, 11), repeats=2)),
    (rotated_anisotropic_3d, dict(n=10, block=4)),
    (poisson_box, dict(shape=(5, 6, 7), dirichlet="none")),
    (poisson_box, dict(shape=(5, 6, 7), dirichlet="x0")),
])
def test_fast_assembler_is_bitwise_the_numpy_assembly(fn, kw):
    assert q1._fast_lib() is not None
    a = fn(**kw)
    b = numpy_only(fn, **kw)
    for f in FIELDS:
        x, y = getattr(a, f), getattr(b, f)
        assert x.dtype == y.dtype and np.array_equal(x, y), f


def test_serving_stream_statistics():
    reqs = serving_stream(num=256)
    t = np.array([r["t_arrival"] for r in reqs])
    n = np.array([r["n"] for r in reqs])
    assert np.all(np.diff(t) > 0)
    # Poisson 20/s: mean gap 50 ms (loose 4-sigma band for 256 draws)
    assert abs(np.mean(np.diff(t, prepend=0.0)) - 0.05) < 4 * 0.05 / math.sqrt(256)
    assert n.min() >= 32 and n.max() <= 128
    # log-uniform: the median of ln n sits near the middle of [ln 32, ln 128]
    assert abs(np.median(np.log(n)) - 0.5 * (math.log(32) + math.log(128))) < 0.15
    kinds = {r["kind"] for r in reqs}
    assert kinds == {"layered", "aniso"}
    assert serving_stream(num=256) == reqs


# --------------------------------------------------------------------------
# general (trilinear) hexahedra and the annulus
# --------------------------------------------------------------------------
def _random_spd(rng, m):
    a = rng.normal(size=(m, 3, 3))
    return a @ np.swapaxes(a, 1, 2) + 0.5 * np.eye(3)


def test_hex_assembler_matches_box_assembly():
    """On an axis-aligned box the general-hex assembly equals the box
    assembly (exact 2-point Gauss either way) up to rounding order."""
    shape, lengths = (5, 4, 3), (1.0, 0.7, 0.4)
    rng = np.random.default_rng(7)
    ne = int(np.prod(shape))
    sig = _random_spd(rng, ne)
    sig = 0.5 * (sig + np.swapaxes(sig, 1, 2))
    f = rng.uniform(-1, 1, size=ne)
    coords, _ = q1.box_mesh(shape, lengths)
    gfun = 1.0 + coords[:, 1] - 2.0 * coords[:, 2]

    def dir_fn(x):
        return np.isclose(x[:, 0], 0.0), 1.0 + x[:, 1] - 2.0 * x[:, 2]

    ref = q1.assemble_q1("box", shape, lengths, sig, f, dir_fn)
    hexp = q1.assemble_hex("box", shape, coords, sig, f, np.isclose(coords[:, 0], 0.0), gfun)
    assert np.array_equal(ref.rowptr, hexp.rowptr) and np.array_equal(ref.col, hexp.col)
    assert np.array_equal(ref.elem_nodes, hexp.elem_nodes)
    scale = np.abs(ref.val).max()
    assert np.abs(ref.val - hexp.val).max() <= 1e-13 * scale
    assert np.abs(ref.b - hexp.b).max() <= 1e-13 * max(1.0, np.abs(ref.b).max())


def _csr_dense(p):
    a = np.zeros((p.n, p.n))
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    a[rows, p.col] = p.val
    return a


def _annulus_free(base, kappa, f_elem=None, sigma=None):
    """annulus mesh of the given base with no Dirichlet nodes (full matrix)"""
    p = q1.annulus_3d(0, kappa=kappa, base=base)
    sig = p.elem_sigma if sigma is None else np.broadcast_to(sigma, p.elem_sigma.shape)
    return q1.assemble_hex("annulus", p.shape, p.coords, sig, f_elem, np.zeros(p.n, bool), np.zeros(p.n),
                           periodic1=True)


def test_hex_patch_test_and_partition_of_unity():
    """Constant tensor: K annihilates constants at every node and linear
    functions at interior nodes (2-point Gauss passes the patch test on
    trilinear hexes); K is bitwise symmetric."""
    base = (4, 12, 2)
    rng = np.random.default_rng(3)
    S = _random_spd(rng, 1)[0]
    S = 0.5 * (S + S.T)
    p = _annulus_free(base, 1.0, sigma=S)
    A = _csr_dense(p)
    assert np.array_equal(A, A.T)
    scale = np.abs(A).max()
    assert np.abs(A.sum(axis=1)).max() <= 1e-13 * scale * 27
    u = p.coords @ np.array([0.3, -1.1, 2.0]) + 0.7
    Ku = A @ u
    n0, n1, n2 = base
    i = np.arange(p.n) % (n0 + 1)
    k = np.arange(p.n) // ((n0 + 1) * n1)
    interior = (i > 0) & (i < n0) & (k > 0) & (k < n2)
    assert interior.sum() == (n0 - 1) * n1 * (n2 - 1)
    assert np.abs(Ku[interior]).max() <= 1e-12 * scale * np.abs(u).max() * 27
    # a boundary row carries the flux of the linear field and is not zero
    assert np.abs(Ku[~interior]).max() > 1e-6 * scale
    # positive semidefinite with the constants as the only null vectors
    ev = np.linalg.eigvalsh(A)
    assert abs(ev[0]) <= 1e-10 * ev[-1] and ev[1] > 1e-6 * ev[-1]


def test_hex_load_integrates_the_polygonal_volume():
    """With f = 1 and no Dirichlet nodes the loads add up to the volume of
    the straight-sided annulus: n_phi/2 sin(2 pi/n_phi) (r_o^2 - r_i^2) t."""
    base = (3, 10, 2)
    nel = base[0] * base[1] * base[2]
    p = _annulus_free(base, 5.0, f_elem=np.ones(nel))
    vol = base[1] * 0.5 * math.sin(2 * math.pi / base[1]) * (1.0 - 0.25) * 0.1
    assert abs(p.b.sum() - vol) <= 1e-14 * 8 * nel


def test_annulus_tensor_and_symmetry():
    p = q1.annulus_3d(0, kappa=1e3, base=(2, 8, 1))
    sig = p.elem_sigma
    assert np.array_equal(sig, np.swapaxes(sig, 1, 2))
    # centre angle of element column e1 is 2 pi (e1 + 1/2) / n_phi: t = (-sin, cos, 0) carries kappa
    pc = 2 * math.pi * (np.repeat(np.arange(8), 2) + 0.5) / 8
    t = np.stack([-np.sin(pc), np.cos(pc), np.zeros_like(pc)], 1)
    r = np.stack([np.cos(pc), np.sin(pc), np.zeros_like(pc)], 1)
    assert np.allclose(np.einsum("eij,ej,ei->e", sig, t, t), 1e3, rtol=1e-12)
    assert np.allclose(np.einsum("eij,ej,ei->e", sig, r, r), 1.0, rtol=1e-9)
    assert np.allclose(np.einsum("eij,ej,ei->e", sig, t, r), 0.0, atol=1e-9)
    A = _csr_dense(p)
    assert np.array_equal(A, A.T)
    # Dirichlet rings: inner u = 0, outer u = 1 + cos(phi)/2, both diagonal-only rows
    i = np.arange(p.n) % 3
    j = (np.arange(p.n) // 3) % 8
    assert np.array_equal(p.dirichlet, (i == 0) | (i == 2))
    assert np.allclose(p.g, np.where(i == 2, 1.0 + 0.5 * np.cos(2 * math.pi * j / 8), 0.0), rtol=0, atol=1e-15)
    assert np.all(np.diff(p.rowptr)[p.dirichlet] == 1)


def test_annulus_rows_are_rotation_invariant():
    """Rows of one ring (same radial and thickness index) carry the same
    values: the mesh and the tensor turn together."""
    p = q1.annulus_3d(0, kappa=1e4, base=(4, 12, 2))
    N0, N1 = 5, 12
    for ring in (1, 2, 3):
        for k in (0, 1, 2):
            rows = [ring + N0 * (j + N1 * k) for j in range(N1)]
            vals = [np.sort(p.val[p.rowptr[r]:p.rowptr[r + 1]]) for r in rows]
            scale = np.abs(vals[0]).max()
            for v in vals[1:]:
                assert v.shape == vals[0].shape and np.abs(v - vals[0]).max() <= 1e-11 * scale


def test_annulus_solution_converges_to_the_exact_solution():
    """With sigma = kappa t t^T + r r^T + z z^T, u = 0 inside and
    u = 1 + cos(phi)/2 outside, the exact solution is
    ln(r/r_i)/ln(r_o/r_i) + f(r) cos(phi) with r^2 f'' + r f' = kappa f, i.e.
    f = (r^s - r_i^(2s) r^(-s)) / (2 (r_o^s - r_i^(2s) r_o^(-s))), s = sqrt(kappa):
    a boundary layer at the outer wall that sharpens with kappa.  The nodal
    error of the Q1 solution falls about fourfold per refinement."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    kappa = 100.0
    s = math.sqrt(kappa)
    errs = []
    for refine in (0, 1):
        p = q1.annulus_3d(refine, kappa=kappa, base=(5, 24, 1))
        A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n, p.n))
        u = spla.spsolve(A.tocsc(), p.b)
        r = np.hypot(p.coords[:, 0], p.coords[:, 1])
        phi = np.arctan2(p.coords[:, 1], p.coords[:, 0])
        f = (r**s - 0.5**(2 * s) * r**(-s)) / (2.0 * (1.0 - 0.5**(2 * s)))
        exact = np.log(r / 0.5) / math.log(2.0) + f * np.cos(phi)
        errs.append(np.abs(u - exact).max())
    assert errs[0] < 2e-2
    assert 3.5 < errs[0] / errs[1] < 4.8
