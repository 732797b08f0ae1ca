"""GPU parity at the workloads' full sizes, in the configuration bench.py times.

* Layered stack 128^3 (2,146,689 DOF, the bench workload): every level's drop
  mask, aggregates and matrix patterns bitwise against the oracle's hierarchy;
  V-cycle output against the oracle's; PCG reaches a true relative residual of
  1e-8 in both precision forms.
* Rotated-anisotropy cube 96^3 (912,673 DOF): bitwise hierarchy, FP64 solution
  within 1e-6 of the oracle's with iterations within +-1, FP32-hierarchy form
  to 1e-8 with its error against the FP64 oracle reported.
* Layered stack 192^3 (7,189,057 DOF, 50 repeats, 20:1): with the paper's 10
  levels the coarsening stagnates above 5000 unknowns (reported as such); with
  a 16-level cap the oracle's own strength/drop and aggregation routines on the
  full finest level agree bitwise; PCG in the FP32-hierarchy and FP64 forms is
  recorded with its error against the exact discrete solution.
"""

import sys
import time

import numpy as np
import pytest

import oracle
from workloads.q1 import layered_stack_3d, rotated_anisotropic_3d

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def amg():
    import torch

    import paper_2602_05686_amd as amg

    assert torch.cuda.is_available()
    amg.load()
    return amg


def compare_hierarchies(h, orc, name):
    st = h.stats()
    assert st["levels"] == orc.nlev, name
    for l in range(orc.nlev):
        rp, ci, _ = h.level_csr(l, "A")
        assert np.array_equal(rp, orc.get(l, "A_rowptr")) and np.array_equal(ci, orc.get(l, "A_col")), \
            f"{name}: A pattern level {l}"
        assert np.array_equal(h.level_aux(l, "x"), orc.get(l, "x")), f"{name}: coordinates level {l}"
        assert np.array_equal(h.level_aux(l, "sig"), orc.get(l, "sig")), f"{name}: tensors level {l}"
        if l + 1 < orc.nlev:
            assert np.array_equal(h.soc_mask(l), orc.get(l, "mask")), f"{name}: mask level {l}"
            assert np.array_equal(h.aggregates(l), orc.get(l, "agg")), f"{name}: aggregates level {l}"
            prp, pci, _ = h.level_csr(l, "P")
            assert np.array_equal(prp, orc.get(l, "P_rowptr")) and np.array_equal(pci, orc.get(l, "P_col")), \
                f"{name}: P pattern level {l}"
    return st


@pytest.fixture(scope="module")
def layered128():
    banner("generating layered stack 128^3")
    return layered_stack_3d(n=128, repeats=20, stretch=10.0)


def test_layered128_hierarchy_and_vcycle(amg, layered128):
    import torch

    prob = layered128
    banner("layered128: oracle setup")
    t = time.time()
    orc = oracle.Hierarchy(prob)
    print(f"oracle setup {time.time() - t:.1f}s levels {orc.stats()['n']}")
    banner("layered128: GPU setup")
    h = amg.Hierarchy.from_problem(prob)
    compare_hierarchies(h, orc, "layered128")
    banner("layered128: V-cycle")
    r = np.random.default_rng(5).standard_normal(prob.n)
    zo = orc.vcycle(r)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    h.vcycle(rt, zt)
    torch.cuda.synchronize()
    z = zt.cpu().numpy()
    rel = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    # rounding differences in the restricted residual reach the output through
    # the coarsest solve amplified by up to cond(A_L)
    rp, ci, va = orc.level_csr(orc.nlev - 1, "A")
    nL = len(rp) - 1
    AL = np.zeros((nL, nL))
    AL[np.repeat(np.arange(nL), np.diff(rp)), ci] = va
    bound = max(1e-9, 10 * np.finfo(float).eps * np.linalg.cond(AL))
    print(f"layered128 V-cycle rel diff {rel:.2e} (bound {bound:.2e})")
    assert rel <= bound


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_layered128_solve(amg, layered128, precision):
    prob = layered128
    banner(f"layered128: {precision} PCG")
    h = amg.Hierarchy.from_problem(prob, precision=precision)
    x, info = h.solve(prob.b)
    r = prob.b - oracle.spmv(prob.rowptr, prob.col, prob.val, x)
    rel = np.linalg.norm(r) / np.linalg.norm(prob.b)
    print(f"layered128 {precision}: iterations {info['iterations']} true rel-res {rel:.2e} "
          f"solve {info['t_solve_s'] * 1e3:.1f} ms")
    assert info["status"] == "OK" and rel <= 1e-8


def test_aniso96_parity(amg):
    prob = rotated_anisotropic_3d(n=96, block=8)
    banner("aniso96: oracle setup + PCG")
    orc = oracle.Hierarchy(prob)
    xo, io = orc.pcg(prob.b)
    banner("aniso96: GPU")
    h = amg.Hierarchy.from_problem(prob)
    compare_hierarchies(h, orc, "aniso96")
    x, info = h.solve(prob.b)
    err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"aniso96 fp64: iters gpu={info['iterations']} oracle={io['iterations']} rel_err={err:.2e}")
    assert info["status"] == "OK" and info["rel_res"] <= 1e-8
    assert abs(info["iterations"] - io["iterations"]) <= 1
    assert err <= 1e-6
    h32 = amg.Hierarchy.from_problem(prob, precision="fp32")
    x32, i32 = h32.solve(prob.b)
    r = prob.b - oracle.spmv(prob.rowptr, prob.col, prob.val, x32)
    rel = np.linalg.norm(r) / np.linalg.norm(prob.b)
    err32 = np.linalg.norm(x32 - xo) / np.linalg.norm(xo)
    print(f"aniso96 fp32-hierarchy: iters {i32['iterations']} true rel-res {rel:.2e} rel_err vs fp64 oracle "
          f"{err32:.2e} solve {i32['t_solve_s'] * 1e3:.1f} ms vs fp64 {info['t_solve_s'] * 1e3:.1f} ms")
    assert i32["status"] == "OK" and rel <= 1e-8


def test_layered192_finest_level_and_fp32_solve(amg):
    banner("generating layered stack 192^3")
    prob = layered_stack_3d(n=192, repeats=50, stretch=20.0, config_id=4)
    banner("layered192: GPU material-measure setup")
    # z-only semi-coarsening of 150 thin layers needs more than the paper's
    # 10 levels to reach 5000 unknowns (with 10 the setup reports stagnation)
    with pytest.raises(amg.AmgError) as e:
        amg.Hierarchy.from_problem(prob, precision="fp32")
    assert e.value.status == "COARSENING_STAGNATED"
    h = amg.Hierarchy.from_problem(prob, precision="fp32", max_levels=16)
    banner("layered192: oracle strength and aggregation on the finest level")
    sig = oracle.clement(prob.n, 3, prob.elem_nodes, prob.elem_sigma)
    assert np.array_equal(h.level_aux(0, "sig"), sig)
    d = oracle.detect_dirichlet(prob.rowptr, prob.col, prob.val)
    _, _, S, mask = oracle.strength(prob.rowptr, prob.col, prob.val, 3, prob.coords, sig, dirichlet=d, theta=0.08)
    assert np.array_equal(h.soc_mask(0), mask)
    agg, nagg, rounds, _ = oracle.aggregate(prob.rowptr, prob.col, mask, d, seed=0, level=0)
    assert np.array_equal(h.aggregates(0), agg)
    assert h.stats()["n"][1] == nagg
    # With 1.28 elements per layer most separators are one element thick: the
    # Clement means of both interface nodes are ~K/2 of the conductive side, the
    # separator is invisible to the material distance and aggregates straddle
    # it, so PCG converges slowly.  Both forms run to 3000 iterations and are
    # recorded with their error against the exact discrete solution.
    kz = prob.meta["layer_k"]
    res = 1.0 / kz
    cf = np.concatenate([[0.0], np.cumsum(res)]) / res.sum()
    exact = cf[np.rint(prob.coords[:, 2] * 192).astype(int)]
    banner("layered192: FP32-hierarchy PCG, material measure")
    x, info = h.solve(prob.b, max_iter=3000, raise_on_error=False)
    st = h.stats()
    h.close()
    err32 = np.linalg.norm(x - exact) / np.linalg.norm(exact)
    print(f"layered192 material fp32: levels {st['n']} status {info['status']} iterations "
          f"{info['iterations']} rel-res {info['rel_res']:.2e} error vs exact {err32:.2e} "
          f"setup {st['t_setup_s'] * 1e3:.0f} ms solve {info['t_solve_s'] * 1e3:.0f} ms")
    assert info["status"] in ("OK", "NOT_CONVERGED") and info["rel_res"] <= 1e-6
    banner("layered192: FP64 PCG, material measure")
    h64 = amg.Hierarchy.from_problem(prob, precision="fp64", max_levels=16)
    x64, i64 = h64.solve(prob.b, max_iter=3000, raise_on_error=False)
    h64.close()
    err64 = np.linalg.norm(x64 - exact) / np.linalg.norm(exact)
    d = np.linalg.norm(x - x64) / np.linalg.norm(x64)
    print(f"layered192 material fp64: status {i64['status']} iterations {i64['iterations']} rel-res "
          f"{i64['rel_res']:.2e} error vs exact {err64:.2e} solve {i64['t_solve_s'] * 1e3:.0f} ms; "
          f"fp32-hierarchy vs fp64 form {d:.2e}")
    assert i64["status"] in ("OK", "NOT_CONVERGED") and i64["rel_res"] <= 1e-6


def test_layered128_wide_blocks_update_and_partition(amg, layered128, monkeypatch):
    """At the bench size the two finest operators stream 4096-entry blocks
    while the setup kernels keep 2048-entry ones: the device partitions
    agree with the host walk, and a value update (setup kernels on the kept
    blocks) still gives bit for bit a fresh setup of the scaled problem."""
    import dataclasses

    monkeypatch.setenv("MATAMG_CHECK_PARTITION", "1")
    prob = layered128
    p4 = dataclasses.replace(prob, val=prob.val * 4.0, b=prob.b * 4.0, elem_sigma=prob.elem_sigma * 4.0)
    banner("layered128: wide blocks, update vs fresh")
    h = amg.Hierarchy.from_problem(prob)
    h.update_values(p4.val)
    f = amg.Hierarchy.from_problem(p4)
    sh, sf = h.stats(), f.stats()
    assert sh["levels"] == sf["levels"]
    assert sh["omega"] == sf["omega"] and sh["lam_cheb"] == sf["lam_cheb"]
    for l in range(sh["levels"]):
        a, b = h.level_csr(l, "A"), f.level_csr(l, "A")
        assert all(np.array_equal(u, v) for u, v in zip(a, b)), l
    xh, ih = h.solve(p4.b)
    xf, if_ = f.solve(p4.b)
    assert ih["iterations"] == if_["iterations"] and np.array_equal(xh, xf)
    assert ih["rel_res"] <= 1e-8
    h.close()
    f.close()
