"""Pins of the oracle's prolongator, Galerkin product, smoother, V-cycle and PCG."""

import math

import numpy as np
import pytest

import oracle
from workloads.q1 import (config1_checkerboard_2d, layered_stack_3d, poisson_box, rotated_anisotropic_3d,
                          two_domain_2d)


def dense(rowptr, col, val, ncols):
    n = rowptr.shape[0] - 1
    a = np.zeros((n, ncols))
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    np.add.at(a, (rows, col), val)
    return a


@pytest.fixture(scope="module")
def aniso():
    prob = rotated_anisotropic_3d(n=8, block=4)
    return prob, oracle.Hierarchy(prob, max_coarse=40)


@pytest.fixture(scope="module")
def checker():
    prob = config1_checkerboard_2d(n=32, cells=4)
    return prob, oracle.Hierarchy(prob, max_coarse=40)


def test_prolongator_formula(checker):
    """P = (I - omega Dt^{-1} A_F) P^, with A_F the lumped filtered matrix and
    Dt its 1-norm diagonal (eqs. operator_smoothing, filtered_matrix,
    1_norm_diagonal), evaluated densely from the oracle's mask and aggregates."""
    prob, h = checker
    A = prob.dense()
    n = prob.n
    mask = h.get(0, "mask")
    agg = h.get(0, "agg")
    nc = h.info(0)["nc"]
    rows = np.repeat(np.arange(n), np.diff(prob.rowptr))
    keep = np.zeros((n, n), bool)
    keep[rows, prob.col] = mask
    AF = np.where(keep, A, 0.0)
    np.fill_diagonal(AF, 0.0)
    AF[np.arange(n), np.arange(n)] = A.diagonal() + (A - np.diag(A.diagonal())).sum(1) - AF.sum(1)
    assert np.allclose(AF.sum(1), A.sum(1), rtol=0, atol=1e-12 * np.abs(A).max())
    Dt = np.abs(AF).sum(1)
    rowabs = np.abs(A).sum(1)
    kept_off = np.abs(np.where(keep & ~np.eye(n, dtype=bool), A, 0.0)).sum(1)
    # empty filtered rows, and rows whose kept off-diagonals weigh nothing
    # (isolated, Dirichlet rows aside), are not smoothed
    Dt[(Dt <= 2.0**-46 * rowabs) | ((kept_off <= 2.0**-46 * rowabs) & ~prob.dirichlet)] = 0.0
    Dtinv = np.where(Dt > 0, 1.0 / np.where(Dt > 0, Dt, 1.0), 0.0)
    Phat = np.zeros((n, nc))
    Phat[agg >= 0, agg[agg >= 0]] = 1.0
    omega = h.info(0)["omega"]
    Pref = Phat - omega * (AF * Dtinv[:, None]) @ Phat
    P = dense(*h.level_csr(0, "P"), nc)
    assert np.allclose(P, Pref, rtol=0, atol=1e-13)
    # rows of P-hat sum to one on non-Dirichlet rows; Dirichlet rows are empty
    assert np.all(Phat[~prob.dirichlet].sum(1) == 1.0)
    prp = h.get(0, "P_rowptr")
    assert np.all(np.diff(prp)[prob.dirichlet] == 0)
    # constants are interpolated on rows where A's row sum vanishes
    zero_rows = (np.abs(A.sum(1)) < 1e-12 * np.abs(A).max(1)) & ~prob.dirichlet
    assert np.allclose(P[zero_rows].sum(1), 1.0, atol=1e-12)
    # 1-norm diagonal: rho(Dt^{-1} A_F) <= 1 (Gershgorin), so the estimate is <= 1
    assert h.info(0)["lam_pf"] <= 1.0 + 1e-12
    assert omega == pytest.approx((4.0 / 3.0) / h.info(0)["lam_pf"], rel=1e-15)


def test_empty_filtered_rows_keep_the_tentative_prolongator():
    """A node whose off-diagonals are all dropped has a filtered row equal to
    its lumped diagonal, the row sum of A.  On zero-sum rows that is zero in
    exact arithmetic (round-off in floating point): the row is not smoothed and
    P's row equals the tentative prolongator's row exactly."""
    prob = rotated_anisotropic_3d(n=16, block=8)
    h = oracle.Hierarchy(prob, max_coarse=100)
    seen = 0
    for l in range(h.nlev - 1):
        rp, ci, va = h.level_csr(l, "A")
        mask = h.get(l, "mask")
        agg = h.get(l, "agg")
        prp, pci, pva = h.level_csr(l, "P")
        for i in range(len(rp) - 1):
            lo, hi = rp[i], rp[i + 1]
            off = ci[lo:hi] != i
            if mask[lo:hi][off].any() or agg[i] < 0:
                continue
            seen += 1
            assert list(pci[prp[i]:prp[i + 1]]) == [agg[i]]
            assert list(pva[prp[i]:prp[i + 1]]) == [1.0]
    assert seen > 0


def test_galerkin_product_and_spd(aniso):
    prob, h = aniso
    for l in range(h.nlev - 1):
        inf = h.info(l)
        A = dense(*h.level_csr(l, "A"), inf["n"])
        P = dense(*h.level_csr(l, "P"), inf["nc"])
        R = dense(*h.level_csr(l, "R"), inf["n"])
        assert np.array_equal(R, P.T)
        Ac = dense(*h.level_csr(l + 1, "A"), inf["nc"])
        ref = P.T @ A @ P
        assert np.allclose(Ac, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert np.allclose(Ac, Ac.T, rtol=0, atol=1e-12 * np.abs(ref).max())
        assert np.linalg.eigvalsh(0.5 * (Ac + Ac.T)).min() > 0
        # the stored pattern is the symbolic product: every structurally reachable entry
        prp, pci, _ = h.level_csr(l, "P")
        Ppat = dense(prp, pci, np.ones(len(pci)), inf["nc"]) > 0
        arp, aci, _ = h.level_csr(l, "A")
        Apat = dense(arp, aci, np.ones(len(aci)), inf["n"]) > 0
        sym = (Ppat.T.astype(int) @ Apat.astype(int) @ Ppat.astype(int)) > 0
        stored = dense(h.get(l + 1, "A_rowptr"), h.get(l + 1, "A_col"),
                       np.ones(h.info(l + 1)["nnz"]), inf["nc"]) > 0
        assert np.array_equal(stored, sym)


def test_operator_complexity_at_least_one(aniso, checker):
    for _, h in (aniso, checker):
        assert h.stats()["op_complexity"] >= 1.0


def test_coarse_coordinates_and_tensors(checker):
    """Coarse x and sigma are aggregate means (eq. auxiliary_transfer)."""
    prob, h = checker
    agg = h.get(0, "agg")
    x0, s0 = h.get(0, "x"), h.get(0, "sig")
    x1, s1 = h.get(1, "x"), h.get(1, "sig")
    for a in range(h.info(0)["nc"]):
        m = agg == a
        assert np.allclose(x1[a], x0[m].mean(0), rtol=1e-15, atol=1e-15)
        assert np.allclose(s1[a], s0[m].mean(0), rtol=1e-14)
    # constant tensors stay constant bitwise through the hierarchy
    p2 = poisson_box((12, 12), k=0.75, dirichlet="x0")
    h2 = oracle.Hierarchy(p2, max_coarse=10)
    for l in range(h2.nlev):
        s = h2.get(l, "sig")
        assert np.all(s == np.array([0.75, 0.0, 0.75]))


@pytest.mark.parametrize("n", [8, 16])
def test_chebyshev_bound_vs_closed_form_spectrum_2d(n):
    """lambda_max(D^{-1} A) = 1 + cos^2(pi/n)/2 for Q1 on an n x n box with
    homogeneous Dirichlet data; 10 power steps stay below it and the boosted
    bound 1.1*lambda lies above it."""
    prob = poisson_box((n, n), dirichlet="all")
    dinv = 1.0 / prob.dense().diagonal()
    lam = oracle.power_method(prob.rowptr, prob.col, prob.val, dinv, iters=10)
    exact = 1.0 + math.cos(math.pi / n) ** 2 / 2.0
    assert lam <= exact * (1 + 1e-12)
    assert 1.1 * lam >= exact
    assert lam >= 0.9 * exact


def test_chebyshev_bound_vs_closed_form_spectrum_3d():
    n = 8
    prob = poisson_box((n, n, n), dirichlet="all")
    dinv = 1.0 / prob.dense().diagonal()
    lam = oracle.power_method(prob.rowptr, prob.col, prob.val, dinv, iters=10)
    a = np.cos(np.arange(1, n) * np.pi / n)
    X, Y, Z = np.meshgrid(a, a, a, indexing="ij")
    ev = ((2 - 2 * X) * (4 + 2 * Y) * (4 + 2 * Z) + (4 + 2 * X) * (2 - 2 * Y) * (4 + 2 * Z)
          + (4 + 2 * X) * (4 + 2 * Y) * (2 - 2 * Z)) / 96.0
    exact = ev.max()
    # ten power steps from a random start converge slowly on the dense top of
    # the 3D spectrum: the estimate is a lower bound within 15%
    assert 0.85 * exact <= lam <= exact * (1 + 1e-12)


def test_chebyshev_error_propagation_is_the_scaled_chebyshev_polynomial():
    """From x=0 the degree-2 smoother's error propagator I - S A equals
    T2((b+a-2 lambda)/(b-a)) / T2((b+a)/(b-a)) on the spectrum of D^{-1}A."""
    prob = poisson_box((6, 6), dirichlet="all")
    h = oracle.Hierarchy(prob, max_coarse=5)
    A = prob.dense()
    n = prob.n
    S = np.stack([h.smooth(0, e) for e in np.eye(n)], axis=1)
    E = np.eye(n) - S @ A
    beta = 1.1 * h.info(0)["lam_cheb"]
    alpha = beta / 30.0
    D = A.diagonal()
    lam, V = np.linalg.eigh(A / np.sqrt(np.outer(D, D)))
    t = lambda z: 2 * z * z - 1
    expect = t((beta + alpha - 2 * lam) / (beta - alpha)) / t((beta + alpha) / (beta - alpha))
    # E is similar to diag(expect) via D^{-1/2} V
    W = np.diag(1 / np.sqrt(D)) @ V
    assert np.allclose(np.linalg.solve(W, E @ W), np.diag(expect), atol=1e-12)


def test_vcycle_is_symmetric_positive_definite(aniso):
    prob, h = aniso
    n = prob.n
    idx = np.random.default_rng(0).choice(n, 40, replace=False)
    M = np.stack([h.vcycle(np.eye(n)[:, i]) for i in idx], axis=1)
    sub = M[idx, :]
    assert np.allclose(sub, sub.T, rtol=0, atol=1e-10 * np.abs(sub).max())
    assert np.linalg.eigvalsh(0.5 * (sub + sub.T)).min() > 0


def test_pcg_matches_dense_solve(checker):
    prob, h = checker
    x, info = h.pcg(prob.b, tol=1e-10)
    assert info["status"] == 0
    ref = np.linalg.solve(prob.dense(), prob.b)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-7
    r = prob.b - prob.dense() @ x
    assert np.linalg.norm(r) / np.linalg.norm(prob.b) <= 1e-10


def test_single_level_is_a_direct_solve():
    prob = poisson_box((6, 6), dirichlet="x0")
    h = oracle.Hierarchy(prob, max_coarse=1000)
    assert h.nlev == 1
    x, info = h.pcg(prob.b, tol=1e-10)
    assert info["status"] == 0 and info["iterations"] == 1


def test_layered_closed_form_solution():
    """f = 0, sides Neumann, u = 0 / 1 on the bottom / top: the exact solution
    lies in the Q1 space and depends on z only,
    u(z_k) = sum_{e<k} h/K_e / sum_e h/K_e."""
    prob = layered_stack_3d(n=12, repeats=2)
    h = oracle.Hierarchy(prob, max_coarse=60)
    x, info = h.pcg(prob.b, tol=1e-12)
    assert info["status"] == 0
    kz = prob.meta["layer_k"]
    res = 1.0 / kz
    cf = np.concatenate([[0.0], np.cumsum(res)]) / res.sum()
    zi = np.rint(prob.coords[:, 2] * 12).astype(int)
    assert np.max(np.abs(x - cf[zi])) < 1e-4


def test_dense_cholesky_matches_numpy():
    rng = np.random.default_rng(1)
    B = rng.normal(size=(30, 30))
    A = B @ B.T + 30 * np.eye(30)
    L = oracle.dense_cholesky(A)
    assert np.allclose(L, np.linalg.cholesky(A), rtol=1e-13, atol=1e-13)
    with pytest.raises(oracle.OracleError) as e:
        oracle.dense_cholesky(-A)
    assert e.value.code == oracle.NOT_SPD


def test_stagnation_reported():
    prob = poisson_box((8, 8), dirichlet="x0")
    with pytest.raises(oracle.OracleError) as e:
        oracle.Hierarchy(prob, max_coarse=2, max_levels=2)
    assert e.value.code == oracle.STAGNATED


def test_homogeneous_iterations_flat_under_refinement():
    """kappa = 1 two-domain problem: iteration counts stay nearly constant under
    refinement (the baseline behaviour of the two-domain study)."""
    its = []
    for n in (16, 32, 64):
        prob = two_domain_2d(n=n, kappa=1.0)
        h = oracle.Hierarchy(prob, max_coarse=30)
        _, info = h.pcg(prob.b)
        assert info["status"] == 0
        its.append(info["iterations"])
    assert max(its) - min(its) <= 4


def test_material_measure_beats_classical_on_contrast():
    """kappa = 1e4 two-domain problem: the material measure converges in fewer
    iterations than classical SA dropping at the same theta."""
    prob = two_domain_2d(n=64, kappa=1e4)
    its = {}
    for soc in ("material", "sa"):
        h = oracle.Hierarchy(prob, max_coarse=30, soc=soc, theta=0.08)
        _, info = h.pcg(prob.b, maxit=500)
        its[soc] = info["iterations"]
    assert its["material"] < its["sa"]


def test_jacobi_smoother_option_converges(checker):
    prob, _ = checker
    h = oracle.Hierarchy(prob, max_coarse=40, smoother="jacobi")
    _, info = h.pcg(prob.b)
    assert info["status"] == 0


@pytest.mark.parametrize("smoother,sweeps,omega", [("jacobi", 1, 2.0 / 3.0), ("jacobi", 2, 2.0 / 3.0),
                                                    ("jacobi", 3, 0.5), ("jacobi_scaled", 2, 2.0 / 3.0),
                                                    ("jacobi_scaled", 3, 0.9)])
def test_jacobi_error_propagator_is_a_power_of_the_damped_jacobi_matrix(smoother, sweeps, omega):
    """The Jacobi options (solver settings of the numerical section: damped
    Jacobi as the alternative to Chebyshev): `sweeps` sweeps of
    x <- x + w D^{-1}(b - A x) with D the plain diagonal of A and w = omega,
    or w = omega * 2 / (1.1 lambda) for the scaled option (lambda the level's
    spectral estimate).  From a zero start the smoother S satisfies
    I - S A = J^sweeps, J = I - w D^{-1} A; from any x0 the error is
    multiplied by the same J^sweeps.  A dropped weight on the zero-start
    sweep, a wrong sweep count or a wrong diagonal changes the power or the
    matrix."""
    prob = poisson_box((6, 6), dirichlet="all")
    h = oracle.Hierarchy(prob, max_coarse=5, smoother=smoother, jacobi_sweeps=sweeps, jacobi_omega=omega)
    A = prob.dense()
    n = prob.n
    w = omega if smoother == "jacobi" else omega * 2.0 / (1.1 * h.info(0)["lam_cheb"])
    if smoother == "jacobi_scaled":
        # the weight times the true spectral radius stays below 2
        rho = np.abs(np.linalg.eigvals(A / A.diagonal()[:, None])).max()
        assert w * rho < 2.0 and w != omega
    J = np.eye(n) - w * A / A.diagonal()[:, None]
    Js = np.linalg.matrix_power(J, sweeps)
    S = np.stack([h.smooth(0, e) for e in np.eye(n)], axis=1)
    assert np.allclose(np.eye(n) - S @ A, Js, rtol=0, atol=1e-13)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    xs = np.linalg.solve(A, b)
    x1 = h.smooth(0, b, x0)
    assert np.allclose(x1 - xs, Js @ (x0 - xs), rtol=0, atol=1e-12 * np.abs(xs).max())


@pytest.mark.parametrize("smoother", ["jacobi", "jacobi_scaled", "chebyshev"])
def test_two_level_vcycle_equals_the_dense_two_grid_operator(smoother):
    """Algorithm Vcycle on two levels with a zero start: pre-smoothing,
    residual, restriction P^T r, exact coarse solve of P^T A P, prolongation
    and post-smoothing give z = (I - E) A^{-1} r with
    E = X (I - P (P^T A P)^{-1} P^T A) X, X = I - S A the smoother's error
    propagator (pre- and post-smoothing apply the same polynomial)."""
    prob = poisson_box((4, 4, 4), dirichlet="x0")
    h = oracle.Hierarchy(prob, max_coarse=30, smoother=smoother)
    assert h.nlev == 2
    A = prob.dense()
    n = prob.n
    nc = h.info(0)["nc"]
    P = dense(*h.level_csr(0, "P"), nc)
    S = np.stack([h.smooth(0, e) for e in np.eye(n)], axis=1)
    X = np.eye(n) - S @ A
    Ac = P.T @ A @ P
    E = X @ (np.eye(n) - P @ np.linalg.solve(Ac, P.T @ A)) @ X
    M = (np.eye(n) - E) @ np.linalg.inv(A)
    rng = np.random.default_rng(4)
    for _ in range(3):
        r = rng.standard_normal(n)
        z = h.vcycle(r)
        assert np.allclose(z, M @ r, rtol=0, atol=1e-11 * np.abs(M @ r).max())
