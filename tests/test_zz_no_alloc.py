"""The allocation-free PCG entry point (amg_pcg_solve_noalloc) against
amg_pcg_solve with device pointers: bitwise equal solutions and equal
iteration counts, in both precision forms, on two calls in a row whose
second problem is smaller than the first (the library's fixed workspace
keeps the first call's contents), plus the oracle's bar for the FP64 form
(iterations +-1, solution within 1e-6)."""

import sys

import numpy as np
import pytest

import oracle
from workloads.q1 import config1_checkerboard_2d, rotated_anisotropic_3d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amg():
    import torch

    import paper_2602_05686_amd as amg

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    amg.load()
    return amg


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_solve_equals_pcg_solve(amg, precision):
    import torch

    cases = [("aniso16", rotated_anisotropic_3d(n=16, block=8), dict(max_coarse=100)),
             ("checker64", config1_checkerboard_2d(), dict(max_coarse=100))]
    assert cases[1][1].n < cases[0][1].n
    for name, prob, kw in cases:
        print(f"[gpu-case] no-alloc solve: {name} n={prob.n} {precision}", flush=True)
        sys.stdout.flush()
        h = amg.Hierarchy.from_problem(prob, precision=precision, **kw)
        b = torch.from_numpy(prob.b).cuda()
        x_ref = torch.zeros_like(b)
        _, i_ref = h.solve(b, x_ref)
        # a nonzero start in the caller's buffer, then the same solve from zero
        x_na = torch.ones_like(b)
        h.solve_noalloc(b, x_na, max_iter=3, raise_on_error=False)
        x_na.zero_()
        _, i_na = h.solve_noalloc(b, x_na)
        torch.cuda.synchronize()
        assert i_na["status"] == "OK" and i_na["iterations"] == i_ref["iterations"], (i_na, i_ref)
        assert i_na["rel_res"] == i_ref["rel_res"]
        assert torch.equal(x_na, x_ref), f"{name} {precision}: solutions differ"
        if precision == "fp64":
            orc = oracle.Hierarchy(prob, **kw)
            xo, io = orc.pcg(prob.b)
            x = x_na.cpu().numpy()
            assert abs(i_na["iterations"] - io["iterations"]) <= 1
            assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-6
        h.close()
