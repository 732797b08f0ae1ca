"""Structured Q1 (bilinear / trilinear) finite elements for -div(sigma grad u) = f.

The model problem and its variational form are those of the paper's introduction
(eq. model_problem): sigma is symmetric positive definite, Dirichlet data g on part
of the boundary and homogeneous Neumann data elsewhere. Meshes are tensor-product
boxes, so every element is an axis-aligned box and 2-point Gauss quadrature per
direction integrates the Q1 stiffness exactly.

Conventions
-----------
* Node (ix, iy[, iz]) has id ix + N0*(iy + N1*iz) with N_k = n_k + 1.
* Element (ex, ey[, ez]) has id ex + n0*(ey + n1*ez); its local vertex a has
  bits (a&1, (a>>1)&1, (a>>2)&1) giving the node (ex+a0, ey+a1, ez+a2).
* The matrix pattern is the full 3^d-point element connectivity, with structural
  zeros kept (the isotropic cube's axis couplings assemble to round-off zero).
* Dirichlet nodes are eliminated symmetrically: b_f -= A_fD g_D, every
  off-diagonal in a Dirichlet row or column is removed from the pattern, the
  assembled diagonal A_dd is kept and b_d = A_dd g_d.  Every node stays an
  unknown, so Dirichlet rows are diagonal-only rows.

All random draws come from numpy's SeedSequence([config_id, seed, ...]).
"""

from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
import threading

import numpy as np

__all__ = [
    "Problem",
    "box_mesh",
    "assemble_q1",
    "config1_checkerboard_2d",
    "layered_stack_3d",
    "rotated_anisotropic_3d",
    "two_domain_2d",
    "poisson_box",
    "structured_hex_nodes",
    "assemble_hex",
    "annulus_3d",
    "serving_stream",
    "problem_from_request",
]


@dataclasses.dataclass
class Problem:
    """One linear system A u = b plus the auxiliary data the setup needs."""

    name: str
    dim: int
    shape: tuple            # elements per direction
    lengths: tuple          # domain extent per direction
    rowptr: np.ndarray      # int32 [n+1]
    col: np.ndarray         # int32 [nnz], ascending per row
    val: np.ndarray         # float64 [nnz]
    b: np.ndarray           # float64 [n]
    coords: np.ndarray      # float64 [n, dim]
    elem_nodes: np.ndarray  # int32 [nelem, 2^dim]
    elem_sigma: np.ndarray  # float64 [nelem, dim, dim]
    dirichlet: np.ndarray   # bool [n]
    g: np.ndarray           # float64 [n], Dirichlet values (0 elsewhere)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def nelem(self) -> int:
        return int(self.elem_nodes.shape[0])

    def dense(self) -> np.ndarray:
        n = self.n
        a = np.zeros((n, n))
        rows = np.repeat(np.arange(n), np.diff(self.rowptr))
        a[rows, self.col] = self.val
        return a


def _rng(*key) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def box_mesh(shape, lengths):
    """Nodes and element connectivity of a tensor-product box mesh."""
    dim = len(shape)
    nn = [s + 1 for s in shape]
    axes = [np.linspace(0.0, float(L), s + 1) for s, L in zip(shape, lengths)]
    # node id = ix + N0*(iy + N1*iz): x fastest
    grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
    coords = np.stack([g.reshape(-1) for g in grids], axis=1).astype(np.float64)
    ne = [np.arange(s) for s in shape]
    egrid = np.meshgrid(*ne[::-1], indexing="ij")[::-1]  # element index per dim
    ecomp = [g.reshape(-1).astype(np.int64) for g in egrid]
    stride = [1] * dim
    for k in range(1, dim):
        stride[k] = stride[k - 1] * nn[k - 1]
    nloc = 1 << dim
    elem_nodes = np.empty((ecomp[0].shape[0], nloc), dtype=np.int32)
    for a in range(nloc):
        node = np.zeros_like(ecomp[0])
        for k in range(dim):
            node += (ecomp[k] + ((a >> k) & 1)) * stride[k]
        elem_nodes[:, a] = node
    return coords, elem_nodes


def _reference_gradients(h):
    """G[p, q, a, b] = integral over one box element of d_p phi_a * d_q phi_b."""
    dim = len(h)
    nloc = 1 << dim
    gp = np.array([0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)])
    gw = np.array([0.5, 0.5])
    vol = float(np.prod(h))
    G = np.zeros((dim, dim, nloc, nloc))
    for qidx in np.ndindex(*([2] * dim)):
        t = np.array([gp[i] for i in qidx])
        w = float(np.prod([gw[i] for i in qidx])) * vol
        grad = np.zeros((nloc, dim))
        for a in range(nloc):
            bits = [(a >> k) & 1 for k in range(dim)]
            vals = [t[k] if bits[k] else 1.0 - t[k] for k in range(dim)]
            ders = [1.0 / h[k] if bits[k] else -1.0 / h[k] for k in range(dim)]
            for p in range(dim):
                prod = ders[p]
                for k in range(dim):
                    if k != p:
                        prod *= vals[k]
                grad[a, p] = prod
        G += w * np.einsum("ap,bq->pqab", grad, grad)
    return G


# ----------------------------------------------------------------------------
# row-streamed C assembler for 3D (same operations in the same order as the
# numpy loops below, so the results are identical)
# ----------------------------------------------------------------------------
class _Q1Input(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("iso", ctypes.c_int), ("kiso", ctypes.c_void_p), ("sig", ctypes.c_void_p),
                ("G", ctypes.c_void_p), ("Gsum", ctypes.c_void_p), ("fg", ctypes.c_void_p),
                ("dmask", ctypes.c_void_p), ("g", ctypes.c_void_p)]


class _HexInput(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int64), ("n1", ctypes.c_int64), ("n2", ctypes.c_int64),
                ("periodic1", ctypes.c_int32), ("X", ctypes.c_void_p), ("sig", ctypes.c_void_p),
                ("fe", ctypes.c_void_p), ("dmask", ctypes.c_void_p), ("g", ctypes.c_void_p)]


_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "q1asm.c"), os.path.join(_HERE, "q1hex.c")]
_SO = os.path.join(_HERE, "_q1asm.so")
_lib_cache = []
_lib_lock = threading.Lock()


def build_fast(force=False):
    """Compile q1asm.c and q1hex.c into workloads/_q1asm.so (gcc, no contraction)."""
    stale = not os.path.exists(_SO) or any(os.path.getmtime(_SO) < os.path.getmtime(src) for src in _SRCS)
    if force or stale:
        tmp = _SO + f".{os.getpid()}.tmp"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", *_SRCS, "-lm", "-o", tmp],
                       check=True)
        os.replace(tmp, _SO)
    return _SO


def _fast_lib():
    with _lib_lock:
        if not _lib_cache:
            lib = None
            try:
                lib = ctypes.CDLL(build_fast())
                lib.q1_rowptr_3d.restype = ctypes.c_int64
                lib.q1_rowptr_3d.argtypes = [ctypes.POINTER(_Q1Input), ctypes.c_void_p]
                lib.q1_fill_3d.restype = None
                lib.q1_fill_3d.argtypes = [ctypes.POINTER(_Q1Input), ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
                lib.hex_elements.restype = ctypes.c_int
                lib.hex_elements.argtypes = [ctypes.POINTER(_HexInput), ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_void_p]
                lib.hex_rowptr.restype = ctypes.c_int64
                lib.hex_rowptr.argtypes = [ctypes.POINTER(_HexInput), ctypes.c_void_p]
                lib.hex_fill.restype = None
                lib.hex_fill.argtypes = [ctypes.POINTER(_HexInput), ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
            except (OSError, subprocess.CalledProcessError, FileNotFoundError):
                lib = None
            _lib_cache.append(lib)
        return _lib_cache[0]


def _assemble_3d_fast(shape, G, vol, elem_sigma, f_elem, dmask, g, threads=None):
    lib = _fast_lib()
    nx, ny, nz = shape
    n = (nx + 1) * (ny + 1) * (nz + 1)
    sig = np.ascontiguousarray(elem_sigma, dtype=np.float64).reshape(-1, 9)
    offdiag_zero = not np.any(sig[:, [1, 2, 3, 5, 6, 7]])
    iso = offdiag_zero and np.array_equal(sig[:, 0], sig[:, 4]) and np.array_equal(sig[:, 0], sig[:, 8])
    kiso = np.ascontiguousarray(sig[:, 0])
    Gc = np.ascontiguousarray(G.reshape(9, 64))
    Gsum = np.ascontiguousarray(sum(G[k, k] for k in range(3)).reshape(64))
    fg = np.ascontiguousarray(np.asarray(f_elem, dtype=np.float64) * (vol / 8))
    dm = np.ascontiguousarray(dmask.astype(np.uint8))
    gg = np.ascontiguousarray(g, dtype=np.float64)
    inp = _Q1Input(nx, ny, nz, int(iso), kiso.ctypes.data, sig.ctypes.data, Gc.ctypes.data, Gsum.ctypes.data,
                   fg.ctypes.data, dm.ctypes.data, gg.ctypes.data)
    rp = np.empty(n + 1, dtype=np.int64)
    nnz = lib.q1_rowptr_3d(ctypes.byref(inp), rp.ctypes.data)
    if nnz >= 2**31:
        raise ValueError("nnz exceeds int32 indexing")
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    b = np.empty(n, dtype=np.float64)
    threads = threads or min(8, os.cpu_count() or 1)
    cuts = np.linspace(0, n, threads + 1).astype(np.int64)

    def work(t):
        lib.q1_fill_3d(ctypes.byref(inp), rp.ctypes.data, int(cuts[t]), int(cuts[t + 1]), col.ctypes.data,
                       val.ctypes.data, b.ctypes.data)

    if threads == 1 or n < 100000:
        lib.q1_fill_3d(ctypes.byref(inp), rp.ctypes.data, 0, n, col.ctypes.data, val.ctypes.data, b.ctypes.data)
    else:
        ths = [threading.Thread(target=work, args=(t,)) for t in range(threads)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
    return rp.astype(np.int32), col, val, b


def assemble_q1(name, shape, lengths, elem_sigma, f_elem, dirichlet_fn, meta=None, fast=True):
    """Assemble A and b on a box mesh and eliminate the Dirichlet nodes.

    elem_sigma: [nelem, dim, dim] SPD tensors; f_elem: [nelem] element-constant
    source; dirichlet_fn(coords) -> (mask[n] bool, g[n] float).  In 3D the
    row-streamed C assembler (q1asm.c, identical results) is used when it
    builds, unless fast=False.
    """
    dim = len(shape)
    shape = tuple(int(s) for s in shape)
    lengths = tuple(float(L) for L in lengths)
    coords, elem_nodes = box_mesh(shape, lengths)
    nn = [s + 1 for s in shape]
    n = int(np.prod(nn))
    h = [L / s for L, s in zip(lengths, shape)]
    G = _reference_gradients(h)
    vol = float(np.prod(h))
    nloc = 1 << dim
    nslot = 3 ** dim
    if dim == 3 and fast and _fast_lib() is not None:
        dmask, g = dirichlet_fn(coords)
        dmask = np.asarray(dmask, dtype=bool)
        g = np.where(dmask, np.asarray(g, dtype=np.float64), 0.0)
        rowptr, col, val, b = _assemble_3d_fast(shape, G, vol, elem_sigma, f_elem, dmask, g)
        return Problem(
            name=name, dim=dim, shape=shape, lengths=lengths, rowptr=rowptr, col=col, val=val, b=b,
            coords=coords, elem_nodes=elem_nodes,
            elem_sigma=np.ascontiguousarray(elem_sigma, dtype=np.float64),
            dirichlet=dmask, g=g, meta=dict(meta or {}),
        )

    # element arrays viewed on the element grid (z, y, x order for reshaping);
    # V is stored slot-major so every sliced update writes contiguous planes
    egshape = tuple(shape[::-1])
    ngshape = tuple(nn[::-1])
    sig = elem_sigma.reshape(egshape + (dim, dim))
    V = np.zeros((nslot,) + ngshape)
    offdiag_zero = all(not np.any(sig[..., p, q]) for p in range(dim) for q in range(dim) if p != q)
    iso = offdiag_zero and all(np.array_equal(sig[..., 0, 0], sig[..., k, k]) for k in range(1, dim))
    kiso = np.ascontiguousarray(sig[..., 0, 0]) if iso else None
    Gsum = sum(G[k, k] for k in range(dim))

    def slot_of(off):
        s = 0
        for k in reversed(range(dim)):
            s = s * 3 + (off[k] + 1)
        return s

    for a in range(nloc):
        abits = [(a >> k) & 1 for k in range(dim)]
        sl = tuple(slice(abits[k], abits[k] + shape[k]) for k in reversed(range(dim)))
        for bb in range(nloc):
            bbits = [(bb >> k) & 1 for k in range(dim)]
            off = [bbits[k] - abits[k] for k in range(dim)]
            if iso:
                ke = kiso * Gsum[a, bb]
            else:
                ke = np.zeros(egshape)
                for p in range(dim):
                    for q in range(dim):
                        gpq = G[p, q, a, bb]
                        if gpq != 0.0:
                            ke += sig[..., p, q] * gpq
            V[(slot_of(off),) + sl] += ke

    # load vector: integral of phi_a over a box is vol / 2^dim
    bgrid = np.zeros(ngshape)
    fg = f_elem.reshape(egshape) * (vol / nloc)
    for a in range(nloc):
        abits = [(a >> k) & 1 for k in range(dim)]
        sl = tuple(slice(abits[k], abits[k] + shape[k]) for k in reversed(range(dim)))
        bgrid[sl] += fg
    V = np.ascontiguousarray(V.reshape(nslot, n).T)
    b = bgrid.reshape(n)

    # structural validity of each slot and the linear column offset
    idx = [np.arange(m) for m in nn]
    node_comp = np.meshgrid(*idx[::-1], indexing="ij")[::-1]
    node_comp = [c.reshape(-1) for c in node_comp]
    valid = np.ones((n, nslot), dtype=bool)
    lin = np.zeros(nslot, dtype=np.int64)
    stride = [1] * dim
    for k in range(1, dim):
        stride[k] = stride[k - 1] * nn[k - 1]
    for s in range(nslot):
        off = [((s // (3 ** k)) % 3) - 1 for k in range(dim)]
        for k in range(dim):
            if off[k] < 0:
                valid[:, s] &= node_comp[k] > 0
            elif off[k] > 0:
                valid[:, s] &= node_comp[k] < nn[k] - 1
        lin[s] = sum(off[k] * stride[k] for k in range(dim))
    center = slot_of([0] * dim)

    dmask, g = dirichlet_fn(coords)
    dmask = np.asarray(dmask, dtype=bool)
    g = np.where(dmask, np.asarray(g, dtype=np.float64), 0.0)
    rows = np.arange(n, dtype=np.int64)
    # symmetric elimination: b_f -= A_fD g_D, in slot order
    if dmask.any():
        for s in range(nslot):
            if s == center:
                continue
            j = np.clip(rows + lin[s], 0, n - 1)
            hit = valid[:, s] & dmask[j] & ~dmask
            if hit.any():
                b[hit] -= V[hit, s] * g[j[hit]]
        for s in range(nslot):
            if s == center:
                continue
            j = np.clip(rows + lin[s], 0, n - 1)
            valid[:, s] &= ~(dmask | dmask[j])
        b[dmask] = V[dmask, center] * g[dmask]

    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 indexing")
    colfull = (np.arange(n, dtype=np.int32)[:, None] + lin.astype(np.int32)[None, :])
    col = colfull[valid].astype(np.int32)
    del colfull
    val = V[valid].astype(np.float64)
    del V
    prob = Problem(
        name=name, dim=dim, shape=shape, lengths=lengths,
        rowptr=rowptr.astype(np.int32), col=col, val=val, b=b,
        coords=coords, elem_nodes=elem_nodes,
        elem_sigma=np.ascontiguousarray(elem_sigma, dtype=np.float64),
        dirichlet=dmask, g=g, meta=dict(meta or {}),
    )
    return prob


def _split_run(fn, count, threads, serial_below=100000):
    """fn(lo, hi) over [0, count) in `threads` contiguous ranges (ctypes calls release the GIL)."""
    threads = max(1, min(threads or min(8, os.cpu_count() or 1), count))
    if threads == 1 or count < serial_below:
        return [fn(0, count)]
    cuts = np.linspace(0, count, threads + 1).astype(np.int64)
    out = [None] * threads

    def work(t):
        out[t] = fn(int(cuts[t]), int(cuts[t + 1]))

    ths = [threading.Thread(target=work, args=(t,)) for t in range(threads)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    return out


def structured_hex_nodes(shape, periodic1=False):
    """Element connectivity [nelem, 8] of a structured hex index space whose
    second direction may wrap around (node j = n1 is node 0)."""
    n0, n1, n2 = (int(v) for v in shape)
    N0, N1 = n0 + 1, (n1 if periodic1 else n1 + 1)
    e2, e1, e0 = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    e0, e1, e2 = (v.reshape(-1).astype(np.int64) for v in (e0, e1, e2))
    nodes = np.empty((e0.shape[0], 8), dtype=np.int32)
    for a in range(8):
        j = e1 + ((a >> 1) & 1)
        if periodic1:
            j = j % n1
        nodes[:, a] = e0 + (a & 1) + N0 * (j + N1 * (e2 + ((a >> 2) & 1)))
    return nodes


def assemble_hex(name, shape, coords, elem_sigma, f_elem, dmask, g, periodic1=False, lengths=None, meta=None,
                 threads=None):
    """Q1 on a structured mesh of general (trilinear) hexahedra, assembled by
    q1hex.c: 2x2x2 Gauss quadrature, symmetric Dirichlet elimination as in
    assemble_q1.  coords [n, 3] in the node order of structured_hex_nodes;
    f_elem [nelem] or None (no source)."""
    lib = _fast_lib()
    if lib is None:
        raise RuntimeError("the C assembler (workloads/q1hex.c) did not build")
    n0, n1, n2 = (int(v) for v in shape)
    if min(n0, n1, n2) < 1 or (periodic1 and n1 < 3):
        raise ValueError("need at least one element per direction (three around a periodic direction)")
    N1 = n1 if periodic1 else n1 + 1
    n = (n0 + 1) * N1 * (n2 + 1)
    nelem = n0 * n1 * n2
    X = np.ascontiguousarray(coords, dtype=np.float64)
    sig = np.ascontiguousarray(elem_sigma, dtype=np.float64).reshape(nelem, 9)
    if X.shape != (n, 3):
        raise ValueError("coords must be [n, 3]")
    dm = np.ascontiguousarray(np.asarray(dmask, dtype=bool).astype(np.uint8))
    gg = np.ascontiguousarray(np.where(dm != 0, np.asarray(g, dtype=np.float64), 0.0))
    fe = None if f_elem is None else np.ascontiguousarray(f_elem, dtype=np.float64)
    inp = _HexInput(n0, n1, n2, int(bool(periodic1)), X.ctypes.data, sig.ctypes.data,
                    None if fe is None else fe.ctypes.data, dm.ctypes.data, gg.ctypes.data)
    Ke = np.empty((nelem, 64))
    Le = None if fe is None else np.empty((nelem, 8))
    rcs = _split_run(lambda lo, hi: lib.hex_elements(ctypes.byref(inp), lo, hi, Ke.ctypes.data,
                                                      None if Le is None else Le.ctypes.data),
                     nelem, threads, serial_below=20000)
    if any(rc != 0 for rc in rcs):
        raise ValueError("degenerate hexahedron (zero or non-finite Jacobian)")
    rp = np.empty(n + 1, dtype=np.int64)
    nnz = lib.hex_rowptr(ctypes.byref(inp), rp.ctypes.data)
    if nnz >= 2**31:
        raise ValueError("nnz exceeds int32 indexing")
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    b = np.empty(n, dtype=np.float64)
    _split_run(lambda lo, hi: lib.hex_fill(ctypes.byref(inp), Ke.ctypes.data,
                                           None if Le is None else Le.ctypes.data, rp.ctypes.data, lo, hi,
                                           col.ctypes.data, val.ctypes.data, b.ctypes.data), n, threads)
    del Ke, Le
    return Problem(
        name=name, dim=3, shape=(n0, n1, n2), lengths=tuple(lengths) if lengths else (0.0, 0.0, 0.0),
        rowptr=rp.astype(np.int32), col=col, val=val, b=b, coords=X,
        elem_nodes=structured_hex_nodes(shape, periodic1), elem_sigma=sig.reshape(nelem, 3, 3),
        dirichlet=dm.astype(bool), g=gg, meta=dict(meta or {}),
    )


ANNULUS_BASE = (20, 150, 1)


def annulus_3d(refine=0, kappa=1e4, r_in=0.5, r_out=1.0, thickness=0.1, base=ANNULUS_BASE, g_in=0.0, g_out=1.0,
               g_cos=0.5, threads=None):
    """The paper's anisotropic thermal-diffusion annulus (section "Anisotropic
    thermal diffusion"): r_in < r < r_out, 0 < z < thickness, base mesh
    base = (radial, circumferential, thickness) hexahedra, each direction
    refined 2^refine times.  Nodes lie on the circles r_i = r_in + (r_out -
    r_in) i / n_r at angles 2 pi j / n_phi; elements are the trilinear hexes
    through them.  sigma_e = kappa t t^T + r r^T + z z^T with t the
    circumferential and r the radial unit vector at the element's centre
    angle (high conductivity around the ring).  Dirichlet u = g_in on the
    inner and u = g_out + g_cos cos(phi) on the outer surface, natural
    conditions on the two flat faces, no source."""
    f = 1 << int(refine)
    n0, n1, n2 = base[0] * f, base[1] * f, base[2] * f
    N0, N1, N2 = n0 + 1, n1, n2 + 1
    k, j, i = np.meshgrid(np.arange(N2), np.arange(N1), np.arange(N0), indexing="ij")
    i, j, k = (v.reshape(-1) for v in (i, j, k))
    r = r_in + (r_out - r_in) * (i / n0)
    phi = (2.0 * math.pi) * (j / n1)
    coords = np.stack([r * np.cos(phi), r * np.sin(phi), thickness * (k / n2)], axis=1)
    del k, j, r
    e1 = np.tile(np.repeat(np.arange(n1), n0), n2)
    pc = (2.0 * math.pi) * ((e1 + 0.5) / n1)
    c, s = np.cos(pc), np.sin(pc)
    sig = np.zeros((e1.shape[0], 3, 3))
    sig[:, 0, 0] = kappa * (s * s) + c * c
    sig[:, 1, 1] = kappa * (c * c) + s * s
    sig[:, 0, 1] = (1.0 - kappa) * (c * s)
    sig[:, 1, 0] = sig[:, 0, 1]
    sig[:, 2, 2] = 1.0
    del e1, pc, c, s
    dmask = (i == 0) | (i == n0)
    g = np.where(i == n0, float(g_out) + float(g_cos) * np.cos(phi), float(g_in))
    return assemble_hex("annulus3d", (n0, n1, n2), coords, sig, None, dmask, g, periodic1=True,
                        lengths=(r_out - r_in, 2.0 * math.pi, thickness),
                        meta=dict(refine=int(refine), kappa=float(kappa), r_in=r_in, r_out=r_out,
                                  thickness=thickness, base=tuple(base), g_in=g_in, g_out=g_out, g_cos=g_cos),
                        threads=threads)


def _iso(kvals, dim):
    kvals = np.asarray(kvals, dtype=np.float64)
    return kvals[:, None, None] * np.eye(dim)[None, :, :]


def _elem_centers(shape, lengths):
    dim = len(shape)
    h = [L / s for L, s in zip(lengths, shape)]
    ne = [np.arange(s) for s in shape]
    eg = np.meshgrid(*ne[::-1], indexing="ij")[::-1]
    return [((eg[k].reshape(-1) + 0.5) * h[k]) for k in range(dim)], [g.reshape(-1) for g in eg]


def config1_checkerboard_2d(n=64, cells=8, k_low=1.0, k_high=1e6):
    """2D Q1 on the unit square with an 8x8 checkerboard of two isotropic materials.

    Element (I, J) lies in cell (I // (n/cells), J // (n/cells)); even cell parity
    takes k_low, odd parity k_high.  u = 0 on x = 0, homogeneous Neumann elsewhere,
    f = 1.
    """
    shape = (n, n)
    _, eg = _elem_centers(shape, (1.0, 1.0))
    w = n // cells
    parity = ((eg[0] // w) + (eg[1] // w)) % 2
    k = np.where(parity == 0, k_low, k_high)
    sigma = _iso(k, 2)
    f = np.ones(n * n)

    def dir_fn(x):
        m = np.isclose(x[:, 0], 0.0)
        return m, np.zeros(x.shape[0])

    return assemble_q1("checkerboard2d", shape, (1.0, 1.0), sigma, f, dir_fn,
                       meta=dict(config_id=1, k_low=k_low, k_high=k_high, cells=cells))


LAYER_RANGES = ((1e-5, 1e-2), (1e-10, 1e-8), (1e-1, 1e0))


def layered_stack_3d(n=128, repeats=20, stretch=10.0, seed=0, config_id=2, shape=None):
    """Battery-like stack: `repeats` repeats of three isotropic layers along z.

    The domain is [0, stretch]^2 x [0, 1], so elements are `stretch` times wider
    than tall.  Element z-index k lies in layer floor((k + 1/2) * 3R / nz); the
    layer's type t = layer % 3 draws one log-uniform conductivity per (repeat, type)
    from LAYER_RANGES[t].  u = 0 on z = 0, u = 1 on z = 1, Neumann on the sides,
    f = 0.
    """
    if shape is None:
        shape = (n, n, n)
    nz = shape[2]
    lengths = (float(stretch), float(stretch), 1.0)
    rng = _rng(config_id, seed)
    logk = np.empty((repeats, 3))
    for r in range(repeats):
        for t in range(3):
            lo, hi = LAYER_RANGES[t]
            logk[r, t] = rng.uniform(math.log(lo), math.log(hi))
    kz = np.empty(nz)
    for kk in range(nz):
        lam = int(math.floor((kk + 0.5) * 3 * repeats / nz))
        kz[kk] = math.exp(logk[lam // 3, lam % 3])
    _, eg = _elem_centers(shape, lengths)
    k = kz[eg[2]]
    sigma = _iso(k, 3)
    f = np.zeros(k.shape[0])

    def dir_fn(x):
        lo = np.isclose(x[:, 2], 0.0)
        hi = np.isclose(x[:, 2], 1.0)
        return lo | hi, np.where(hi, 1.0, 0.0)

    return assemble_q1("layered3d", shape, lengths, sigma, f, dir_fn,
                       meta=dict(config_id=config_id, seed=seed, repeats=repeats,
                                 stretch=stretch, layer_k=kz))


def _quat_rotation(qv):
    q = qv / np.linalg.norm(qv)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def rotated_anisotropic_3d(n=96, block=8, k_iso=1e-4, eps=1e-3, seed=0, config_id=3):
    """Unit cube with 3D-checkerboard blocks of rotated anisotropy and an isotropic fill.

    Block (bx, by, bz) of block^3 elements with even bx+by+bz has
    K = R diag(1, eps, eps) R^T with R a uniformly random rotation (normalised
    Gaussian quaternion, one per block); odd blocks have K = k_iso I.  Element
    sources f_e ~ U(-1, 1); homogeneous Dirichlet on all six faces.
    """
    shape = (n, n, n)
    rng = _rng(config_id, seed)
    nb = (n + block - 1) // block
    quats = rng.normal(size=(nb, nb, nb, 4))
    f = rng.uniform(-1.0, 1.0, size=n * n * n)
    _, eg = _elem_centers(shape, (1.0, 1.0, 1.0))
    bx, by, bz = eg[0] // block, eg[1] // block, eg[2] // block
    sigma = np.empty((n * n * n, 3, 3))
    aniso = ((bx + by + bz) % 2) == 0
    sigma[~aniso] = k_iso * np.eye(3)
    d = np.diag([1.0, eps, eps])
    Kb = np.empty((nb, nb, nb, 3, 3))
    for ib in np.ndindex(nb, nb, nb):
        R = _quat_rotation(quats[ib])
        Kb[ib] = R @ d @ R.T
    Kb = 0.5 * (Kb + np.swapaxes(Kb, -1, -2))
    sigma[aniso] = Kb[bx[aniso], by[aniso], bz[aniso]]

    def dir_fn(x):
        m = np.zeros(x.shape[0], dtype=bool)
        for k in range(3):
            m |= np.isclose(x[:, k], 0.0) | np.isclose(x[:, k], 1.0)
        return m, np.zeros(x.shape[0])

    return assemble_q1("aniso3d", shape, (1.0, 1.0, 1.0), sigma, f, dir_fn,
                       meta=dict(config_id=config_id, seed=seed, block=block))


def two_domain_2d(n=32, kappa=100.0):
    """The paper's two-domain problem on (-1, 1)^2: sigma = I for x < 0 and
    diag(kappa, 1) for x >= 0 (element centres decide), homogeneous Dirichlet
    on the whole boundary, f = 1."""
    shape = (n, n)
    cen, _ = _elem_centers(shape, (2.0, 2.0))
    x = cen[0] - 1.0
    sigma = np.repeat(np.eye(2)[None], n * n, axis=0)
    sigma[x >= 0.0, 0, 0] = kappa
    f = np.ones(n * n)

    def dir_fn(xc):
        m = np.zeros(xc.shape[0], dtype=bool)
        for k in range(2):
            m |= np.isclose(xc[:, k], 0.0) | np.isclose(xc[:, k], 2.0)
        return m, np.zeros(xc.shape[0])

    return assemble_q1("two_domain2d", shape, (2.0, 2.0), sigma, f, dir_fn,
                       meta=dict(kappa=kappa))


def poisson_box(shape, lengths=None, k=1.0, f=1.0, dirichlet="all"):
    """Homogeneous Q1 Poisson on a box; dirichlet in {"all", "none", "x0"}."""
    dim = len(shape)
    if lengths is None:
        lengths = tuple(1.0 for _ in shape)
    ne = int(np.prod(shape))
    sigma = _iso(np.full(ne, k), dim)
    fe = np.full(ne, float(f))

    def dir_fn(x):
        m = np.zeros(x.shape[0], dtype=bool)
        if dirichlet == "all":
            for kk in range(dim):
                m |= np.isclose(x[:, kk], 0.0) | np.isclose(x[:, kk], lengths[kk])
        elif dirichlet == "x0":
            m |= np.isclose(x[:, 0], 0.0)
        return m, np.zeros(x.shape[0])

    return assemble_q1("poisson", tuple(shape), tuple(lengths), sigma, fe, dir_fn)


def serving_stream(num=256, rate=20.0, nmin=32, nmax=128, seed=0, config_id=5):
    """Request stream: Poisson arrivals, log-uniform mesh size, layered or
    anisotropic material with a per-request seed."""
    rng = _rng(config_id, seed)
    gaps = rng.exponential(1.0 / rate, size=num)
    t = np.cumsum(gaps)
    sizes = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=num))).astype(int)
    kinds = np.where(rng.uniform(size=num) < 0.5, "layered", "aniso")
    seeds = rng.integers(0, 2**31 - 1, size=num)
    return [dict(id=i, t_arrival=float(t[i]), n=int(sizes[i]), kind=str(kinds[i]),
                 seed=int(seeds[i])) for i in range(num)]


def problem_from_request(req):
    if req["kind"] == "layered":
        return layered_stack_3d(n=req["n"], repeats=20, stretch=10.0, seed=req["seed"], config_id=5)
    return rotated_anisotropic_3d(n=req["n"], seed=req["seed"], config_id=5)


def ulp_perturbed(b, seed):
    """b with every nonzero entry moved by one unit in the last place, up or
    down by a fair coin from default_rng(1000 + seed); zeros stay zero.  Used
    to probe how a solver's exit depends on rounding-level changes of the data."""
    b = np.array(b, dtype=np.float64, copy=True)
    nz = np.nonzero(b)[0]
    sgn = np.random.default_rng(1000 + seed).choice([-1.0, 1.0], size=nz.size)
    b[nz] = np.nextafter(b[nz], np.where(sgn > 0, np.inf, -np.inf))
    return b


def seeded_start(n, seed):
    """Initial guess x0 ~ U(0, 1)^n from default_rng(1000 + seed)."""
    return np.random.default_rng(1000 + seed).uniform(0.0, 1.0, n)


def problem_digest(prob):
    """SHA-256 of a problem's arrays (CSR, load vector, element tensors,
    coordinates): equal digests mean bitwise equal inputs, e.g. on two hosts."""
    import hashlib

    h = hashlib.sha256()
    for a in (prob.rowptr, prob.col, prob.val, prob.b, prob.elem_sigma, prob.coords):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()
