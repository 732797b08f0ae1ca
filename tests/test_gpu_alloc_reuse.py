"""GPU: device buffers kept for reuse (a freed hierarchy's idle buffers, a
setup's released temporaries) never change a result: setups of the same
problem give bitwise the same hierarchy and solve whatever was built and
freed before them, and hierarchies alive at the same time do not share
memory."""

import sys

import numpy as np
import pytest

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


def run(amg, prob, **kw):
    h = amg.Hierarchy.from_problem(prob, **kw)
    x, info = h.solve(prob.b)
    mats = [h.level_csr(l, "A") for l in range(h.stats()["levels"])]
    return h, x, info, mats


def same(a, b):
    return all(np.array_equal(u, v) for u, v in zip(a, b))


def test_reused_buffers_give_bitwise_the_same_setup_and_solve(amg):
    p1 = layered_stack_3d(n=24, repeats=4, stretch=10.0)
    p2 = rotated_anisotropic_3d(n=16, block=4, seed=3)
    banner(f"alloc reuse: layered24 n={p1.n}, aniso16 n={p2.n}")
    h, x1, i1, m1 = run(amg, p1, max_coarse=100)
    h.close()
    for prob in (p2, config1_checkerboard_2d(), p2):
        hh, _, _, _ = run(amg, prob, max_coarse=100)
        hh.close()
    h, x2, i2, m2 = run(amg, p1, max_coarse=100)
    assert i2["iterations"] == i1["iterations"]
    assert np.array_equal(x2, x1)
    assert len(m2) == len(m1) and all(same(a, b) for a, b in zip(m1, m2))
    # a second hierarchy of the same problem while the first is alive
    g, x3, i3, m3 = run(amg, p1, max_coarse=100)
    assert np.array_equal(x3, x1) and all(same(a, b) for a, b in zip(m1, m3))
    # the first still solves as before after the second was built
    x4, i4 = h.solve(p1.b)
    assert np.array_equal(x4, x1) and i4["iterations"] == i1["iterations"]
    g.close()
    h.close()
    # the kept buffers go back to the pool; a setup after that still agrees
    assert amg.trim_cache() > 0
    assert amg.trim_cache() == 0
    h, x5, i5, m5 = run(amg, p1, max_coarse=100)
    assert np.array_equal(x5, x1) and all(same(a, b) for a, b in zip(m1, m5))
    h.close()


def test_fp32_form_after_fp64_frees(amg):
    p = layered_stack_3d(n=20, repeats=4, stretch=10.0)
    banner(f"alloc reuse fp32: layered20 n={p.n}")
    h, x1, i1, _ = run(amg, p, max_coarse=100, precision="fp32")
    h.close()
    for _ in range(2):
        hh, _, _, _ = run(amg, p, max_coarse=100)
        hh.close()
    h, x2, i2, _ = run(amg, p, max_coarse=100, precision="fp32")
    assert i2["iterations"] == i1["iterations"] and np.array_equal(x2, x1)
    h.close()
