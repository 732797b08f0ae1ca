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
