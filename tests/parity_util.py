"""Element-wise comparison helpers shared by the GPU parity tests."""

import numpy as np

import oracle

U = np.finfo(np.float64).eps / 2  # unit round-off of FP64


def level_spmv_rowwise(amg_h, orc, level, x):
    """y = A_level x from the library's streaming kernel against the oracle's
    serial row sums of its own A_level, row by row.

    The library's coarse operators equal the oracle's in pattern and to
    round-off in value (checked elsewhere), so row i may differ by
        4 k_i u sum_j |o_ij x_j|        (two summation orders of k_i terms
                                         differ by at most 2(k_i - 1)u of it)
      + sum_j |g_ij - o_ij| |x_j|       (the measured value differences)
    with g the library's and o the oracle's values; on the finest level g = o
    (the input) and only the first term remains.  Returns (max ratio of the
    difference to sum_j |o_ij x_j|, fraction of rows equal bitwise)."""
    import scipy.sparse as sp
    import torch

    rp, ci, va = orc.level_csr(level, "A")
    grp, gci, gva = amg_h.level_csr(level, "A")
    assert np.array_equal(grp, rp) and np.array_equal(gci, ci), f"level {level}: pattern differs"
    n = rp.shape[0] - 1
    y_or = oracle.spmv(rp, ci, va, x)
    ax = np.abs(x)
    scale = sp.csr_matrix((np.abs(va), ci, rp), shape=(n, n)) @ ax
    vdiff = sp.csr_matrix((np.abs(gva - va), ci, rp), shape=(n, n)) @ ax
    if level == 0:
        assert not vdiff.any(), "finest operator differs from the input"
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    yt = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    amg_h.level_spmv(level, xt, yt)
    torch.cuda.synchronize()
    y = yt.cpu().numpy()
    assert np.all(np.isfinite(y)), f"level {level}: non-finite or unwritten rows"
    d = np.abs(y - y_or)
    bound = 4.0 * np.diff(rp) * U * scale + vdiff
    bad = d > bound
    assert not bad.any(), (f"level {level}: {int(bad.sum())} rows beyond the bound, worst "
                           f"{float((d[bad] / np.maximum(bound[bad], 1e-300)).max()):.2f}x")
    nzs = scale > 0
    ratio = float((d[nzs] / scale[nzs]).max()) if nzs.any() else 0.0
    return ratio, float(np.mean(d == 0))


def row_scaled_diff(rp, va, ova):
    """max over rows of max_j |va_ij - ova_ij| / max_j |ova_ij| (rows of zeros: absolute)."""
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    rmax = np.zeros(n)
    np.maximum.at(rmax, rows, np.abs(ova))
    dmax = np.zeros(n)
    np.maximum.at(dmax, rows, np.abs(va - ova))
    scale = np.where(rmax > 0, rmax, 1.0)
    return float((dmax / scale).max()) if n else 0.0
