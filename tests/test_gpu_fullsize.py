"""GPU parity at the workloads' full sizes, in the configuration bench.py times.

* Layered stack 128^3 (2,146,689 DOF, the bench workload): every level's
  drop mask, aggregates and patterns bitwise against the oracle's hierarchy,
  values within 1e-10 or the oracle's own rounding spread, every level's SpMV
  row by row, the V-cycle, and PCG from x0 = 0 against the oracle's exits
  (live, and under 1-ulp changes of b from the stored record) and against
  the exact discrete solution.
* Rotated-anisotropy cube 96^3 (912,673 DOF): the same hierarchy checks, FP64
  solution within 1e-6 of the oracle's with iterations within +-1,
  FP32-hierarchy form to 1e-8 with its error against the FP64 oracle.
* Layered stack 192^3 (7,189,057 DOF, 50 repeats, 20:1): with the paper's 10
  levels the coarsening stagnates above 5000 unknowns (reported as such);
  with 16 levels the whole hierarchy against the oracle's, and PCG to a true
  relative residual of 1e-8 in both precision forms with their errors
  against the exact discrete solution.
"""

import json
import math
import os
import sys
import time

import numpy as np
import pytest

import oracle
from parity_util import level_spmv_rowwise, row_scaled_diff
from workloads.q1 import layered_stack_3d, problem_digest, rotated_anisotropic_3d

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


SAFETY = 10.0  # the library's rounding is another draw of the kind the spread samples


def load_spread(name):
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{name}_oracle_spread.json")) as f:
        return json.load(f)


def compare_hierarchies(h, orc, name, values=False, spread=None):
    """Patterns, masks, aggregates, coordinates and tensors bitwise on every
    level; with values=True also A, P and R values (each row's largest entry
    as its scale), damping factors and smoother bounds, within 1e-10, or on
    levels where the oracle itself moves further under rounding-level changes
    of the input, within SAFETY times that spread (spread: the record of
    tests/golden/make_oracle_spread.py)."""
    st = h.stats()
    assert st["levels"] == orc.nlev, name
    if spread is not None:
        assert spread["levels"] == [orc.info(l)["n"] for l in range(orc.nlev)], f"{name}: spread record"

    def tol(l, key):
        return max(1e-10, SAFETY * spread["spread"][l][key]) if spread is not None else 1e-10

    report = []
    for l in range(orc.nlev):
        rp, ci, va = h.level_csr(l, "A")
        assert np.array_equal(rp, orc.get(l, "A_rowptr")) and np.array_equal(ci, orc.get(l, "A_col")), \
            f"{name}: A pattern level {l}"
        row = {}
        if values:
            row["A"] = row_scaled_diff(rp, va, orc.get(l, "A_val"))
        assert np.array_equal(h.level_aux(l, "x"), orc.get(l, "x")), f"{name}: coordinates level {l}"
        assert np.array_equal(h.level_aux(l, "sig"), orc.get(l, "sig")), f"{name}: tensors level {l}"
        if l + 1 < orc.nlev:
            assert np.array_equal(h.soc_mask(l), orc.get(l, "mask")), f"{name}: mask level {l}"
            assert np.array_equal(h.aggregates(l), orc.get(l, "agg")), f"{name}: aggregates level {l}"
            assert st["mis_rounds"][l] == orc.info(l)["mis_rounds"], f"{name}: MIS rounds level {l}"
            for which in ("P", "R"):
                mrp, mci, mva = h.level_csr(l, which)
                assert np.array_equal(mrp, orc.get(l, f"{which}_rowptr")) and \
                    np.array_equal(mci, orc.get(l, f"{which}_col")), f"{name}: {which} pattern level {l}"
                if values:
                    row[which] = row_scaled_diff(mrp, mva, orc.get(l, f"{which}_val"))
            if values:
                for key in ("omega", "lam_cheb"):
                    ref = orc.info(l)[key]
                    row[key] = abs(st[key][l] - ref) / abs(ref)
        if values:
            report.append(row)
            print(f"{name} level {l}: " + ", ".join(f"{k} {v:.1e} (tol {tol(l, k):.0e})" for k, v in row.items()))
            for k, v in row.items():
                assert v <= tol(l, k), f"{name}: {k} differs by {v:.2e} on level {l} (tolerance {tol(l, k):.2e})"
    return st


def layered_exact(prob):
    kz = prob.meta["layer_k"]
    res = 1.0 / kz
    cf = np.concatenate([[0.0], np.cumsum(res)]) / res.sum()
    return cf[np.rint(prob.coords[:, 2] * prob.shape[2]).astype(int)]


@pytest.fixture(scope="module")
def layered128():
    banner("generating layered stack 128^3")
    return layered_stack_3d(n=128, repeats=20, stretch=10.0)


@pytest.fixture(scope="module")
def layered128_oracle(layered128):
    """The oracle's hierarchy and its PCG solve from x0 = 0 (solver settings of
    the numerical section: CG to a relative residual of 1e-8)."""
    prob = layered128
    banner("layered128: oracle setup")
    t = time.time()
    orc = oracle.Hierarchy(prob)
    print(f"oracle setup {time.time() - t:.1f}s levels {orc.stats()['n']}", flush=True)
    banner("layered128: oracle PCG from x0 = 0 (about a minute)")
    t = time.time()
    xo, io = orc.pcg(prob.b)
    eo = np.linalg.norm(xo - layered_exact(prob)) / np.linalg.norm(layered_exact(prob))
    print(f"oracle PCG {time.time() - t:.1f}s iterations {io['iterations']} rel-res {io['rel_res']:.2e} "
          f"error vs exact {eo:.3e}", flush=True)
    assert io["status"] == oracle.OK
    return orc, xo, io


def test_layered128_hierarchy_spmv_and_vcycle(amg, layered128, layered128_oracle):
    import torch

    prob = layered128
    orc, _, _ = layered128_oracle
    banner("layered128: GPU setup")
    h = amg.Hierarchy.from_problem(prob)
    compare_hierarchies(h, orc, "layered128", values=True, spread=load_spread("layered128"))
    banner("layered128: level SpMV row by row")
    rng = np.random.default_rng(6)
    for l in range(orc.nlev):
        n = orc.info(l)["n"]
        ratio, same = level_spmv_rowwise(h, orc, l, rng.standard_normal(n))
        print(f"layered128 level {l} (n={n}): SpMV worst row {ratio:.1e} of sum|a x|, {same:.1%} rows bitwise")
    banner("layered128: V-cycle")
    r = np.random.default_rng(5).standard_normal(prob.n)
    zo = orc.vcycle(r)
    rt = torch.from_numpy(r).cuda()
    zt = torch.zeros_like(rt)
    h.vcycle(rt, zt)
    torch.cuda.synchronize()
    z = zt.cpu().numpy()
    rel = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    # A-norm: the norm in which CG sees the preconditioner
    dz = z - zo
    rel_a = math.sqrt(abs(dz @ oracle.spmv(prob.rowptr, prob.col, prob.val, dz)) /
                      (zo @ oracle.spmv(prob.rowptr, prob.col, prob.val, zo)))
    # rounding differences in the coarse operator's entries reach the output
    # through the coarsest solve amplified by up to cond(A_L); on this stack
    # the deep levels themselves move with rounding (the oracle's own V-cycle
    # output on the same r moves by the recorded spread under a 1-ulp
    # rescaling of the input), and the larger of the two bounds the agreement
    rp, ci, va = orc.level_csr(orc.nlev - 1, "A")
    nL = len(rp) - 1
    AL = np.zeros((nL, nL))
    AL[np.repeat(np.arange(nL), np.diff(rp)), ci] = va
    spread = load_spread("layered128")["vcycle"]
    bound = max(1e-9, 10 * np.finfo(float).eps * np.linalg.cond(AL), SAFETY * spread)
    print(f"layered128 V-cycle rel diff {rel:.2e} (bound {bound:.2e}; the oracle's own spread {spread:.2e}), "
          f"in the A-norm {rel_a:.2e}")
    assert rel <= bound


GOLDEN128 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "layered128_oracle_exits.json")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_layered128_solve(amg, layered128, layered128_oracle, precision):
    """PCG from x0 = 0 in the configuration the benchmark times.

    The oracle's exit depends on rounding-level changes of the data: with b
    as generated it stops after 103 iterations, and with every nonzero of b
    moved by one ulp after 108, 103, 108, 103 or 108
    (tests/golden/layered128_oracle_exits.json, written by the script beside
    it from the oracle alone); all of these lie 2.7e-4 to 5.1e-4 from the
    exact discrete solution, the accuracy a relative residual of 1e-8 buys on
    a 1e10 contrast.  The FP64 form must stop within one iteration of an exit
    the oracle takes on b or on one of those perturbations, and be at least
    half as accurate against the exact solution as the least accurate of the
    oracle's exits there; both forms must reach a true relative residual of
    1e-8."""
    prob = layered128
    _, xo, io = layered128_oracle
    with open(GOLDEN128) as f:
        gold = json.load(f)
    assert gold["input_sha256"] == problem_digest(prob), "the generated stack differs from the recorded one"
    exits = [c for c in gold["cases"] if c["case"] in ("b", "ulp")]
    assert io["iterations"] == exits[0]["iterations"], "the oracle's exit on this host differs from the record"
    banner(f"layered128: {precision} PCG")
    h = amg.Hierarchy.from_problem(prob, precision=precision)
    x, info = h.solve(prob.b)
    r = prob.b - oracle.spmv(prob.rowptr, prob.col, prob.val, x)
    rel = np.linalg.norm(r) / np.linalg.norm(prob.b)
    ex = layered_exact(prob)
    eg = np.linalg.norm(x - ex) / np.linalg.norm(ex)
    eo = np.linalg.norm(xo - ex) / np.linalg.norm(ex)
    d = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    near = [c for c in exits if abs(c["iterations"] - info["iterations"]) <= 1]
    worst = max((c["err_vs_exact"] for c in near), default=float("nan"))
    print(f"layered128 {precision}: iterations {info['iterations']} (oracle {io['iterations']}; under 1-ulp "
          f"changes of b {[c['iterations'] for c in exits[1:]]}) true rel-res {rel:.2e}; error vs exact {eg:.3e} "
          f"(oracle {eo:.3e}, least accurate oracle exit within one iteration {worst:.3e}); vs the oracle's "
          f"solution {d:.2e}; solve {info['t_solve_s'] * 1e3:.1f} ms")
    assert info["status"] == "OK" and rel <= 1e-8
    if precision == "fp64":
        assert near, "the exit is not within one iteration of any of the oracle's"
        assert eg <= 2.0 * worst


def test_layered128_seeded_start(amg, layered128):
    """PCG (FP64 form) from the seeded start x0 = seeded_start(n, 0).  From
    this start the oracle stops after 114 iterations on b as generated and
    under one-ulp changes of b, and after 105, 115 or 116 once A's values are
    scaled by 1 + j 2^-52 (every rounding of its setup changes;
    tests/golden/layered128_oracle_exits.json, cases x0 seed 0, x0ulp and
    x0scale).  The GPU must stop within one iteration of one of these exits
    at a true relative residual of 1e-8.  From a random start the error
    against the exact solution keeps the start's floating-cluster modes,
    which the residual hardly sees, so it varies with the exit (the
    oracle's: 0.25% to 0.79%): the GPU must be at least half as accurate
    as the least accurate of the oracle's seven exits."""
    from workloads.q1 import seeded_start

    prob = layered128
    with open(GOLDEN128) as f:
        gold = json.load(f)
    assert gold["input_sha256"] == problem_digest(prob), "the generated stack differs from the recorded one"
    exits = [c for c in gold["cases"]
             if (c["case"] == "x0" and c["seed"] == 0) or c["case"] in ("x0ulp", "x0scale")]
    assert len(exits) == 7
    banner("layered128: fp64 PCG from seeded start 0")
    h = amg.Hierarchy.from_problem(prob)
    x, info = h.solve(prob.b, x0=seeded_start(prob.n, 0))
    h.close()
    r = prob.b - oracle.spmv(prob.rowptr, prob.col, prob.val, x)
    rel = np.linalg.norm(r) / np.linalg.norm(prob.b)
    ex = layered_exact(prob)
    eg = np.linalg.norm(x - ex) / np.linalg.norm(ex)
    near = [c for c in exits if abs(c["iterations"] - info["iterations"]) <= 1]
    worst = max(c["err_vs_exact"] for c in exits)
    print(f"layered128 seeded start: iterations {info['iterations']} (oracle {[c['iterations'] for c in exits]}) "
          f"true rel-res {rel:.2e}; error vs exact {eg:.3e} (least accurate oracle exit {worst:.3e})")
    assert info["status"] == "OK" and rel <= 1e-8
    assert near, "the exit is not within one iteration of any of the oracle's"
    assert eg <= 2.0 * worst


def test_aniso96_parity(amg):
    prob = rotated_anisotropic_3d(n=96, block=8)
    banner("aniso96: oracle setup + PCG")
    orc = oracle.Hierarchy(prob)
    xo, io = orc.pcg(prob.b)
    banner("aniso96: GPU")
    h = amg.Hierarchy.from_problem(prob)
    compare_hierarchies(h, orc, "aniso96", values=True, spread=load_spread("aniso96"))
    rng = np.random.default_rng(7)
    for l in range(orc.nlev):
        n = orc.info(l)["n"]
        ratio, same = level_spmv_rowwise(h, orc, l, rng.standard_normal(n))
        print(f"aniso96 level {l} (n={n}): SpMV worst row {ratio:.1e} of sum|a x|, {same:.1%} rows bitwise")
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


def test_layered192_hierarchy_and_solves(amg):
    """192^3 stack (7,189,057 DOF, 50 repeats, 20:1).  The paper's cap of 10
    levels stagnates above 5000 unknowns (150 thin layers coarsen in z only),
    so it runs with 16: every level of the hierarchy against the oracle's
    (patterns, masks, aggregates, coordinates and tensors bitwise, values to
    round-off), then PCG to a true relative residual of 1e-8 in both
    precision forms.  Each form's error against the series-resistor profile
    must be no worse than the oracle's own solve gives (to 1%; recorded by
    tests/golden/make_layered192_oracle_solve.py, the oracle's solve takes
    hours on one core), and its distance from the oracle's solution at the
    recorded sample positions is reported."""
    banner("generating layered stack 192^3")
    prob = layered_stack_3d(n=192, repeats=50, stretch=20.0, config_id=4)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "layered192_oracle_solve.json")) as f:
        rec = json.load(f)
    assert rec["input_sha256"] == problem_digest(prob), "the generated stack differs from the recorded one"
    sidx = np.asarray(rec["sample_index"])
    sx = np.asarray(rec["sample_x"])
    banner("layered192: GPU setup with the paper's 10 levels")
    with pytest.raises(amg.AmgError) as e:
        amg.Hierarchy.from_problem(prob, precision="fp32")
    assert e.value.status == "COARSENING_STAGNATED"
    banner("layered192: oracle setup, 16 levels (about a minute)")
    t = time.time()
    orc = oracle.Hierarchy(prob, max_levels=16)
    print(f"oracle setup {time.time() - t:.1f}s levels {orc.stats()['n']}", flush=True)
    banner("layered192: GPU FP32-hierarchy setup, 16 levels")
    h = amg.Hierarchy.from_problem(prob, precision="fp32", max_levels=16)
    st = compare_hierarchies(h, orc, "layered192", values=True, spread=load_spread("layered192"))
    del orc
    exact = layered_exact(prob)
    banner("layered192: FP32-hierarchy PCG")
    x, info = h.solve(prob.b, max_iter=4000)
    h.close()
    r = prob.b - oracle.spmv(prob.rowptr, prob.col, prob.val, x)
    rel32 = np.linalg.norm(r) / np.linalg.norm(prob.b)
    err32 = np.linalg.norm(x - exact) / np.linalg.norm(exact)
    d32 = np.linalg.norm(x[sidx] - sx) / np.linalg.norm(sx)
    print(f"layered192 fp32: levels {st['n']} iterations {info['iterations']} (oracle {rec['iterations']}) true "
          f"rel-res {rel32:.2e} error vs exact {err32:.2e} (oracle {rec['err_vs_exact']:.2e}); vs the oracle's "
          f"solution at the samples {d32:.2e}; setup {st['t_setup_s'] * 1e3:.0f} ms solve "
          f"{info['t_solve_s'] * 1e3:.0f} ms")
    assert info["status"] == "OK" and rel32 <= 1e-8
    assert err32 <= 1.01 * rec["err_vs_exact"]
    banner("layered192: FP64 PCG")
    h64 = amg.Hierarchy.from_problem(prob, precision="fp64", max_levels=16)
    x64, i64 = h64.solve(prob.b, max_iter=4000)
    h64.close()
    r = prob.b - oracle.spmv(prob.rowptr, prob.col, prob.val, x64)
    rel64 = np.linalg.norm(r) / np.linalg.norm(prob.b)
    err64 = np.linalg.norm(x64 - exact) / np.linalg.norm(exact)
    d = np.linalg.norm(x - x64) / np.linalg.norm(x64)
    d64 = np.linalg.norm(x64[sidx] - sx) / np.linalg.norm(sx)
    print(f"layered192 fp64: iterations {i64['iterations']} (oracle {rec['iterations']}) true rel-res {rel64:.2e} "
          f"error vs exact {err64:.2e} (oracle {rec['err_vs_exact']:.2e}); vs the oracle's solution at the samples "
          f"{d64:.2e}; solve {i64['t_solve_s'] * 1e3:.0f} ms; fp32-hierarchy vs fp64 form {d:.2e}")
    assert i64["status"] == "OK" and rel64 <= 1e-8
    assert err64 <= 1.01 * rec["err_vs_exact"]


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
