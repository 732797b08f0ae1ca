"""CPU oracle for material-aware SA-AMG-PCG (test infrastructure).

A plain serial FP64 C implementation (saamg_oracle.c) loaded through ctypes.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
it; the HIP library never does.  `build()` compiles it with gcc
(-O2 -ffp-contract=off) next to the source.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "saamg_oracle.c")
_LIB = os.path.join(_HERE, "libsaamg_oracle.so")
_lib = None

OK, INVALID_ARG, OUT_OF_MEMORY, NOT_SPD, STAGNATED, NOT_CONVERGED, BREAKDOWN = 0, 1, 2, 4, 5, 6, 7
SOC = {"material": 0, "distance": 1, "sa": 2}
DROP = {"pointwise": 0, "cut": 1}
SMOOTHER = {"chebyshev": 0, "jacobi": 1, "jacobi_scaled": 2}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("theta", ctypes.c_double),
        ("soc", ctypes.c_int32),
        ("drop", ctypes.c_int32),
        ("smoother", ctypes.c_int32),
        ("max_coarse", ctypes.c_int32),
        ("max_levels", ctypes.c_int32),
        ("cheb_degree", ctypes.c_int32),
        ("cheb_ratio", ctypes.c_double),
        ("cheb_boost", ctypes.c_double),
        ("power_iters", ctypes.c_int32),
        ("omega_sym", ctypes.c_double),
        ("jacobi_omega", ctypes.c_double),
        ("jacobi_sweeps", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle shared library in place."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    """The loaded oracle library: SAAMG_ORACLE_LIB names a prebuilt one (the
    sanitizer test's instrumented build), else the in-tree build."""
    global _lib
    if _lib is None:
        path = os.environ.get("SAAMG_ORACLE_LIB")
        if not path:
            build(force=False)
            path = _LIB
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, f64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        L.orc_clement.argtypes = [i32, i32, i32, i32, P, P, P]
        L.orc_detect_dirichlet.argtypes = [i32, P, P, P, P]
        L.orc_strength.argtypes = [i32, P, P, P, i32, P, P, P, i32, i32, f64, P, P, P, P]
        L.orc_aggregate.argtypes = [i32, P, P, P, P, u64, i32, P, P, P, P]
        L.orc_setup.argtypes = [i32, P, P, P, i32, i32, P, P, P, ctypes.POINTER(Options), ctypes.POINTER(P)]
        L.orc_setup_reuse.argtypes = [P, P, P, P, ctypes.POINTER(P)]
        L.orc_free.argtypes = [P]
        L.orc_free.restype = None
        L.orc_num_levels.argtypes = [P]
        L.orc_level_info.argtypes = [P, i32, P, P]
        L.orc_level_get.argtypes = [P, i32, i32, P]
        L.orc_vcycle.argtypes = [P, P, P]
        L.orc_pcg.argtypes = [P, P, P, f64, i32, P, P]
        L.orc_spmv.argtypes = [i32, P, P, P, P, P]
        L.orc_dense_cholesky.argtypes = [i32, P]
        L.orc_dense_cholesky_solve.argtypes = [i32, P, P, P]
        L.orc_dense_cholesky_solve.restype = None
        L.orc_power_method.argtypes = [i32, P, P, P, P, i32, u64, i32, i32, P]
        L.orc_smooth.argtypes = [P, i32, P, P, i32]
        L.orc_splitmix64.argtypes = [u64]
        L.orc_splitmix64.restype = u64
        L.orc_default_options.argtypes = [ctypes.POINTER(Options)]
        L.orc_default_options.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(code, what):
    if code != OK:
        raise OracleError(code, what)


def default_options(**kw) -> Options:
    o = Options()
    lib().orc_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "soc" and isinstance(v, str):
            v = SOC[v]
        if k == "smoother" and isinstance(v, str):
            v = SMOOTHER[v]
        if k == "drop" and isinstance(v, str):
            v = DROP[v]
        setattr(o, k, v)
    return o


def splitmix64(x: int) -> int:
    return int(lib().orc_splitmix64(ctypes.c_uint64(x & (2**64 - 1))))


def clement(n, dim, elem_nodes, elem_sigma):
    en = np.ascontiguousarray(elem_nodes, dtype=np.int32)
    es = np.ascontiguousarray(elem_sigma, dtype=np.float64)
    out = np.zeros((n, dim * (dim + 1) // 2))
    _check(lib().orc_clement(n, dim, en.shape[0], en.shape[1], _p(en), _p(es), _p(out)), "clement")
    return out


def detect_dirichlet(rowptr, col, val):
    n = rowptr.shape[0] - 1
    d = np.zeros(n, dtype=np.uint8)
    lib().orc_detect_dirichlet(n, _p(rowptr), _p(col), _p(val), _p(d))
    return d.astype(bool)


def strength(rowptr, col, val, dim, x, sig, dirichlet=None, soc="material", theta=0.08, drop="pointwise"):
    """Returns (lval, ldiag, S, mask) over A's stored pattern."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    sig = np.ascontiguousarray(sig, dtype=np.float64)
    n = rowptr.shape[0] - 1
    nnz = col.shape[0]
    lv = np.zeros(nnz)
    ld = np.zeros(n)
    S = np.zeros(nnz)
    mask = np.zeros(nnz, dtype=np.uint8)
    dp = None
    if dirichlet is not None:
        dd = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        dp = _p(dd)
    socv = SOC[soc] if isinstance(soc, str) else int(soc)
    dropv = DROP[drop] if isinstance(drop, str) else int(drop)
    _check(lib().orc_strength(n, _p(rowptr), _p(col), _p(val), dim, _p(x), _p(sig), dp, socv, dropv, float(theta),
                              _p(lv), _p(ld), _p(S), _p(mask)), "strength")
    return lv, ld, S, mask.astype(bool)


def aggregate(rowptr, col, mask, dirichlet=None, seed=0, level=0):
    """Returns (agg, nagg, rounds, roots)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    n = rowptr.shape[0] - 1
    agg = np.zeros(n, dtype=np.int32)
    roots = np.zeros(n, dtype=np.uint8)
    nagg = ctypes.c_int32()
    rounds = ctypes.c_int32()
    dp = None
    if dirichlet is not None:
        dd = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        dp = _p(dd)
    _check(lib().orc_aggregate(n, _p(rowptr), _p(col), _p(m), dp, ctypes.c_uint64(seed), level, _p(agg),
                               ctypes.byref(nagg), ctypes.byref(rounds), _p(roots)), "aggregate")
    return agg, nagg.value, rounds.value, roots.astype(bool)


def spmv(rowptr, col, val, x):
    n = rowptr.shape[0] - 1
    y = np.zeros(n)
    x = np.ascontiguousarray(x, dtype=np.float64)
    lib().orc_spmv(n, _p(rowptr), _p(col), _p(val), _p(x), _p(y))
    return y


def power_method(rowptr, col, val, dscale, iters=10, seed=0, purpose="cheb", level=0):
    n = rowptr.shape[0] - 1
    lam = ctypes.c_double()
    ds = np.ascontiguousarray(dscale, dtype=np.float64)
    _check(lib().orc_power_method(n, _p(rowptr), _p(col), _p(val), _p(ds), iters, ctypes.c_uint64(seed),
                                  0 if purpose == "pf" else 1, level, ctypes.byref(lam)), "power_method")
    return lam.value


def dense_cholesky(a):
    a = np.array(a, dtype=np.float64, order="C", copy=True)
    _check(lib().orc_dense_cholesky(a.shape[0], _p(a)), "cholesky")
    return a


class Hierarchy:
    """Oracle AMG hierarchy for one problem."""

    _WHAT = dict(A_rowptr=0, A_col=1, A_val=2, P_rowptr=3, P_col=4, P_val=5, R_rowptr=6, R_col=7, R_val=8,
                 agg=9, mask=10, x=11, sig=12, ldiag=13, S=14, dirichlet=15, dinv=16, lval=17, chol=18)

    def __init__(self, prob=None, *, rowptr=None, col=None, val=None, elem_nodes=None, elem_sigma=None,
                 coords=None, options=None, reuse=None, **kw):
        """reuse: an oracle Hierarchy on the same sparsity pattern whose
        coordinates, tensors, masks, aggregates and depth are kept; only the
        value-dependent steps run on the new values (its options apply)."""
        if reuse is not None:
            if prob is not None:
                rowptr, col, val = prob.rowptr, prob.col, prob.val
            rp = np.ascontiguousarray(rowptr, dtype=np.int32)
            ci = np.ascontiguousarray(col, dtype=np.int32)
            va = np.ascontiguousarray(val, dtype=np.float64)
            h = ctypes.c_void_p()
            code = lib().orc_setup_reuse(reuse._h, _p(rp), _p(ci), _p(va), ctypes.byref(h))
            self._h = h
            _check(code, "setup_reuse")
            self.options = reuse.options
            self.nlev = lib().orc_num_levels(h)
            self.n = rp.shape[0] - 1
            return
        if prob is not None:
            rowptr, col, val = prob.rowptr, prob.col, prob.val
            elem_nodes, elem_sigma, coords = prob.elem_nodes, prob.elem_sigma, prob.coords
            kw.setdefault("dim", prob.dim)
        self.options = options if options is not None else default_options(**kw)
        self._keep = [np.ascontiguousarray(a) for a in (rowptr, col, val, elem_nodes, elem_sigma, coords)]
        rp, ci, va, en, es, xc = self._keep
        rp = rp.astype(np.int32, copy=False)
        ci = ci.astype(np.int32, copy=False)
        en = en.astype(np.int32, copy=False)
        self._keep = [rp, ci, va, en, es, xc]
        n = rp.shape[0] - 1
        h = ctypes.c_void_p()
        code = lib().orc_setup(n, _p(rp), _p(ci), _p(va), en.shape[0], en.shape[1], _p(en), _p(es), _p(xc),
                               ctypes.byref(self.options), ctypes.byref(h))
        self._h = h
        _check(code, "setup")
        self.nlev = lib().orc_num_levels(h)
        self.n = n
        self._keep = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_free(h)
            self._h = None

    def info(self, level):
        sizes = np.zeros(5, dtype=np.int64)
        sc = np.zeros(3)
        _check(lib().orc_level_info(self._h, level, _p(sizes), _p(sc)), "level_info")
        return dict(n=int(sizes[0]), nnz=int(sizes[1]), nc=int(sizes[2]), nnz_p=int(sizes[3]),
                    mis_rounds=int(sizes[4]), omega=float(sc[0]), lam_pf=float(sc[1]), lam_cheb=float(sc[2]))

    def get(self, level, what):
        inf = self.info(level)
        n, nnz, nc, nnzp = inf["n"], inf["nnz"], inf["nc"], inf["nnz_p"]
        dim = self.options.dim
        shapes = dict(A_rowptr=(n + 1, np.int32), A_col=(nnz, np.int32), A_val=(nnz, np.float64),
                      P_rowptr=(n + 1, np.int32), P_col=(nnzp, np.int32), P_val=(nnzp, np.float64),
                      R_rowptr=(nc + 1, np.int32), R_col=(nnzp, np.int32), R_val=(nnzp, np.float64),
                      agg=(n, np.int32), mask=(nnz, np.uint8), x=(n * dim, np.float64),
                      sig=(n * dim * (dim + 1) // 2, np.float64), ldiag=(n, np.float64), S=(nnz, np.float64),
                      dirichlet=(n, np.uint8), dinv=(n, np.float64), lval=(nnz, np.float64),
                      chol=(n * n, np.float64))
        size, dt = shapes[what]
        out = np.zeros(size, dtype=dt)
        _check(lib().orc_level_get(self._h, level, self._WHAT[what], _p(out)), f"get {what}")
        if what == "x":
            out = out.reshape(n, dim)
        elif what == "sig":
            out = out.reshape(n, -1)
        elif what == "chol":
            out = out.reshape(n, n)
        elif what in ("mask", "dirichlet"):
            out = out.astype(bool)
        return out

    def level_csr(self, level, which="A"):
        return (self.get(level, f"{which}_rowptr"), self.get(level, f"{which}_col"), self.get(level, f"{which}_val"))

    def vcycle(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.n)
        _check(lib().orc_vcycle(self._h, _p(r), _p(z)), "vcycle")
        return z

    def smooth(self, level, b, x0=None):
        """One smoother application on `level` (pre-smoother when x0 is None)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(b.shape[0]) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        _check(lib().orc_smooth(self._h, level, _p(b), _p(x), 1 if x0 is None else 0), "smooth")
        return x

    def pcg(self, b, x0=None, tol=1e-8, maxit=1000):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        it = ctypes.c_int32()
        rr = ctypes.c_double()
        code = lib().orc_pcg(self._h, _p(b), _p(x), float(tol), int(maxit), ctypes.byref(it), ctypes.byref(rr))
        return x, dict(status=code, iterations=it.value, rel_res=rr.value)

    def stats(self):
        infos = [self.info(l) for l in range(self.nlev)]
        nnz = [i["nnz"] for i in infos]
        return dict(levels=self.nlev, n=[i["n"] for i in infos], nnz=nnz,
                    op_complexity=sum(nnz) / nnz[0])
