"""ctypes binding of libmatamg.so (the C ABI declared in include/amg.h).

Argument marshalling only: every step of setup and solve runs in the HIP
library.  torch is imported before the library is loaded so that both share
one HIP runtime; it is used for device memory (tensors) and streams.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmatamg.so")

AMG_OK = 0
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "HIP", 4: "NOT_SPD", 5: "COARSENING_STAGNATED",
          6: "NOT_CONVERGED", 7: "BREAKDOWN", 8: "BUDGET"}
PTR_HOST, PTR_DEVICE = 0, 1
SOC = {"material": 0, "distance": 1, "sa": 2}
SMOOTHER = {"chebyshev": 0, "jacobi": 1, "jacobi_scaled": 2}
PRECISION = {"fp64": 0, "fp32": 1}
DROP = {"pointwise": 0, "cut": 1}

EXPORTED = [
    "amg_options_default", "amg_setup", "amg_pcg_solve", "amg_pcg_solve_noalloc", "amg_update_values", "amg_vcycle", "amg_level_spmv",
    "amg_hierarchy_info",
    "amg_get_aggregates", "amg_get_soc_mask", "amg_get_level_csr", "amg_get_level_aux", "amg_time_smoother",
    "amg_free", "amg_trim_cache", "amg_status_string", "amg_last_error",
    "amg_server_create", "amg_server_submit", "amg_server_poll", "amg_server_result", "amg_server_info",
    "amg_server_set_batch_wait", "amg_server_destroy",
]


class AmgError(RuntimeError):
    def __init__(self, code, where, detail=""):
        super().__init__(f"{where}: {STATUS.get(code, code)} {detail}".strip())
        self.code = code
        self.status = STATUS.get(code, str(code))


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
        ("precision", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
    ]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("rel_res_true", ctypes.c_double), ("t_solve_s", ctypes.c_double),
                ("status", ctypes.c_int32)]


class HierStats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("n", ctypes.c_int64 * 16),
        ("nnz", ctypes.c_int64 * 16),
        ("nnz_p", ctypes.c_int64 * 16),
        ("mis_rounds", ctypes.c_int32 * 16),
        ("omega", ctypes.c_double * 16),
        ("lam_pf", ctypes.c_double * 16),
        ("lam_cheb", ctypes.c_double * 16),
        ("op_complexity", ctypes.c_double),
        ("vcycle_alg_bytes", ctypes.c_double),
        ("t_setup_s", ctypes.c_double),
        ("device_bytes", ctypes.c_int64),
        ("device_peak_bytes", ctypes.c_int64),
        ("t_update_s", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
        ("rejected", ctypes.c_int64), ("budget_bytes", ctypes.c_int64), ("reserved_bytes", ctypes.c_int64),
        ("peak_reserved_bytes", ctypes.c_int64), ("active", ctypes.c_int32), ("waiting", ctypes.c_int64),
        ("steps", ctypes.c_int64), ("launches", ctypes.c_int64), ("mean_batch", ctypes.c_double),
        ("max_batch", ctypes.c_int64), ("estimate_exceeded", ctypes.c_int64),
    ]


class RequestStats(ctypes.Structure):
    _fields_ = [
        ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_setup_done", ctypes.c_double),
        ("t_done", ctypes.c_double), ("est_bytes", ctypes.c_int64), ("setup_peak_bytes", ctypes.c_int64),
        ("resident_bytes", ctypes.c_int64), ("levels", ctypes.c_int32), ("max_batch", ctypes.c_int32),
        ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
    ]


_lib = None


def load():
    """Load the library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.amg_options_default.argtypes = [ctypes.POINTER(Options)]
    L.amg_setup.argtypes = [i64, P, P, P, i64, i32, P, P, P, ctypes.POINTER(Options), i32, P, ctypes.POINTER(P)]
    L.amg_pcg_solve.argtypes = [P, P, P, f64, i32, i32, P, ctypes.POINTER(SolveInfo)]
    L.amg_pcg_solve_noalloc.argtypes = [P, P, P, f64, i32, P, ctypes.POINTER(SolveInfo)]
    L.amg_vcycle.argtypes = [P, P, P, P]
    L.amg_update_values.argtypes = [P, P, i32, P]
    L.amg_level_spmv.argtypes = [P, i32, P, P, P]
    L.amg_hierarchy_info.argtypes = [P, ctypes.POINTER(HierStats)]
    L.amg_get_aggregates.argtypes = [P, i32, P]
    L.amg_get_soc_mask.argtypes = [P, i32, P]
    L.amg_get_level_csr.argtypes = [P, i32, i32, P, P, P]
    L.amg_get_level_aux.argtypes = [P, i32, i32, P]
    L.amg_time_smoother.argtypes = [P, i32, i32, P, ctypes.POINTER(f64), ctypes.POINTER(f64)]
    L.amg_free.argtypes = [P]
    L.amg_free.restype = None
    L.amg_trim_cache.argtypes = [ctypes.POINTER(ctypes.c_int64)]
    L.amg_server_create.argtypes = [ctypes.POINTER(Options), i64, i32, i32, ctypes.POINTER(P)]
    L.amg_server_submit.argtypes = [P, i64, P, P, P, i64, i32, P, P, P, P, P, f64, i32,
                                    ctypes.POINTER(ctypes.c_uint64)]
    L.amg_server_poll.argtypes = [P, f64, P, i32, ctypes.POINTER(i32)]
    L.amg_server_result.argtypes = [P, ctypes.c_uint64, P, ctypes.POINTER(SolveInfo), ctypes.POINTER(RequestStats)]
    L.amg_server_info.argtypes = [P, ctypes.POINTER(ServerStats)]
    L.amg_server_set_batch_wait.argtypes = [P, f64]
    L.amg_server_destroy.argtypes = [P]
    L.amg_server_destroy.restype = None
    L.amg_status_string.argtypes = [i32]
    L.amg_status_string.restype = ctypes.c_char_p
    L.amg_last_error.argtypes = []
    L.amg_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("amg_free", "amg_status_string", "amg_last_error", "amg_server_destroy"):
            getattr(L, name).restype = ctypes.c_int32
    _lib = L
    return L


def check(code, where):
    if code != AMG_OK:
        detail = load().amg_last_error().decode(errors="replace")
        raise AmgError(code, where, detail)


def options(dim=3, **kw) -> Options:
    o = Options()
    load().amg_options_default(ctypes.byref(o))
    o.dim = dim
    for k, v in kw.items():
        if k == "soc" and isinstance(v, str):
            v = SOC[v]
        elif k == "smoother" and isinstance(v, str):
            v = SMOOTHER[v]
        elif k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        elif k == "drop" and isinstance(v, str):
            v = DROP[v]
        setattr(o, k, v)
    return o


def trim_cache() -> int:
    """Hand the device buffers kept by freed hierarchies back to the pool; returns their bytes."""
    n = ctypes.c_int64(0)
    check(load().amg_trim_cache(ctypes.byref(n)), "amg_trim_cache")
    return int(n.value)


def _hp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dp(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Hierarchy:
    """A multigrid hierarchy owned by the library (one GPU)."""

    def __init__(self, rowptr, col, val, elem_nodes, elem_sigma, coords, opts: Options, stream=None):
        L = load()
        self.opts = opts
        h = ctypes.c_void_p()
        if isinstance(rowptr, np.ndarray):
            rp = np.ascontiguousarray(rowptr, dtype=np.int32)
            ci = np.ascontiguousarray(col, dtype=np.int32)
            va = np.ascontiguousarray(val, dtype=np.float64)
            en = np.ascontiguousarray(elem_nodes, dtype=np.int32)
            es = np.ascontiguousarray(elem_sigma, dtype=np.float64)
            xc = np.ascontiguousarray(coords, dtype=np.float64)
            n = rp.shape[0] - 1
            code = L.amg_setup(n, _hp(rp), _hp(ci), _hp(va), en.shape[0], en.shape[1] if en.ndim == 2 else 0,
                               _hp(en), _hp(es), _hp(xc), ctypes.byref(opts), PTR_HOST, _stream(stream),
                               ctypes.byref(h))
        else:
            n = rowptr.shape[0] - 1
            code = L.amg_setup(n, _dp(rowptr), _dp(col), _dp(val), elem_nodes.shape[0], elem_nodes.shape[1],
                               _dp(elem_nodes), _dp(elem_sigma), _dp(coords), ctypes.byref(opts), PTR_DEVICE,
                               _stream(stream), ctypes.byref(h))
        check(code, "amg_setup")
        self._h = h
        self.n = n

    @classmethod
    def from_problem(cls, prob, stream=None, **kw):
        opts = options(dim=prob.dim, **kw)
        return cls(prob.rowptr, prob.col, prob.val, prob.elem_nodes, prob.elem_sigma, prob.coords, opts, stream)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().amg_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- solves
    def solve(self, b, x0=None, tol=1e-8, max_iter=1000, stream=None, raise_on_error=True):
        """PCG solve.  numpy inputs -> numpy output; torch device tensors -> in place."""
        L = load()
        info = SolveInfo()
        if isinstance(b, np.ndarray):
            bb = np.ascontiguousarray(b, dtype=np.float64)
            x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
            code = L.amg_pcg_solve(self._h, _hp(bb), _hp(x), float(tol), int(max_iter), PTR_HOST, _stream(stream),
                                   ctypes.byref(info))
        else:
            x = torch.zeros_like(b) if x0 is None else x0
            code = L.amg_pcg_solve(self._h, _dp(b), _dp(x), float(tol), int(max_iter), PTR_DEVICE, _stream(stream),
                                   ctypes.byref(info))
        if raise_on_error and code != AMG_OK:
            check(code, "amg_pcg_solve")
        return x, dict(status=STATUS[code], iterations=info.iterations, rel_res=info.rel_res_true,
                       t_solve_s=info.t_solve_s)

    def solve_noalloc(self, b, x, tol=1e-8, max_iter=1000, stream=None, raise_on_error=True):
        """amg_pcg_solve_noalloc: device tensors b and x (x iterated in place,
        holding the initial guess); the library allocates nothing."""
        info = SolveInfo()
        code = load().amg_pcg_solve_noalloc(self._h, _dp(b), _dp(x), float(tol), int(max_iter), _stream(stream),
                                            ctypes.byref(info))
        if raise_on_error and code != AMG_OK:
            check(code, "amg_pcg_solve_noalloc")
        return x, dict(status=STATUS[code], iterations=info.iterations, rel_res=info.rel_res_true,
                       t_solve_s=info.t_solve_s)

    def update_values(self, val, stream=None):
        """New values of A on the setup's pattern (numpy array or device
        tensor): masks, aggregates, coordinates and tensors are kept, the
        value-dependent parts of the setup are recomputed."""
        if isinstance(val, np.ndarray):
            va = np.ascontiguousarray(val, dtype=np.float64)
            code = load().amg_update_values(self._h, _hp(va), PTR_HOST, _stream(stream))
        else:
            code = load().amg_update_values(self._h, _dp(val), PTR_DEVICE, _stream(stream))
        check(code, "amg_update_values")

    def vcycle(self, r, z, stream=None):
        check(load().amg_vcycle(self._h, _dp(r), _dp(z), _stream(stream)), "amg_vcycle")

    def level_spmv(self, level, x, y, stream=None):
        check(load().amg_level_spmv(self._h, level, _dp(x), _dp(y), _stream(stream)), "amg_level_spmv")

    def time_smoother(self, level=0, reps=50, stream=None):
        """Average duration (ms) of the level's fused smoother step and its algorithmic bytes."""
        ms, b = ctypes.c_double(), ctypes.c_double()
        check(load().amg_time_smoother(self._h, level, reps, _stream(stream), ctypes.byref(ms), ctypes.byref(b)),
              "amg_time_smoother")
        return dict(avg_ms=ms.value, bytes_per_launch=b.value)

    # ------------------------------------------------------------ queries
    def stats(self):
        s = HierStats()
        check(load().amg_hierarchy_info(self._h, ctypes.byref(s)), "amg_hierarchy_info")
        L = s.levels
        return dict(levels=L, n=list(s.n[:L]), nnz=list(s.nnz[:L]), nnz_p=list(s.nnz_p[:L]),
                    mis_rounds=list(s.mis_rounds[:L]), omega=list(s.omega[:L]), lam_pf=list(s.lam_pf[:L]),
                    lam_cheb=list(s.lam_cheb[:L]), op_complexity=s.op_complexity,
                    vcycle_alg_bytes=s.vcycle_alg_bytes, t_setup_s=s.t_setup_s, device_bytes=s.device_bytes,
                    device_peak_bytes=s.device_peak_bytes, t_update_s=s.t_update_s)

    def aggregates(self, level):
        n = self.stats()["n"][level]
        out = np.zeros(n, dtype=np.int32)
        check(load().amg_get_aggregates(self._h, level, _hp(out)), "amg_get_aggregates")
        return out

    def soc_mask(self, level):
        nnz = self.stats()["nnz"][level]
        out = np.zeros(nnz, dtype=np.uint8)
        check(load().amg_get_soc_mask(self._h, level, _hp(out)), "amg_get_soc_mask")
        return out.astype(bool)

    def level_csr(self, level, which="A"):
        st = self.stats()
        w = {"A": 0, "P": 1, "R": 2}[which]
        if w == 0:
            rows, nnz = st["n"][level], st["nnz"][level]
        elif w == 1:
            rows, nnz = st["n"][level], st["nnz_p"][level]
        else:
            rows, nnz = st["n"][level + 1], st["nnz_p"][level]
        rp = np.zeros(rows + 1, dtype=np.int32)
        ci = np.zeros(nnz, dtype=np.int32)
        va = np.zeros(nnz, dtype=np.float64)
        check(load().amg_get_level_csr(self._h, level, w, _hp(rp), _hp(ci), _hp(va)), "amg_get_level_csr")
        return rp, ci, va

    def level_aux(self, level, which):
        st = self.stats()
        n, dim = st["n"][level], self.opts.dim
        size = {"x": n * dim, "sig": n * dim * (dim + 1) // 2, "dirichlet": n, "S": st["nnz"][level]}[which]
        out = np.zeros(size)
        w = {"x": 0, "sig": 1, "dirichlet": 2, "S": 3}[which]
        check(load().amg_get_level_aux(self._h, level, w, _hp(out)), "amg_get_level_aux")
        if which == "x":
            return out.reshape(n, dim)
        if which == "sig":
            return out.reshape(n, -1)
        if which == "dirichlet":
            return out.astype(bool)
        return out


class Server:
    """Solve server (amg_server_*): continuous batching of many solves on one GPU.

    submit() copies a problem into the server and returns its id; poll()
    returns ids of finished requests; result() hands one over as
    (x, info, timeline).
    """

    def __init__(self, budget_bytes=8 << 30, max_active=32, setup_workers=2, dim=3, batch_wait_s=0.0, **kw):
        L = load()
        self.opts = options(dim=dim, **kw)
        s = ctypes.c_void_p()
        check(L.amg_server_create(ctypes.byref(self.opts), int(budget_bytes), int(max_active), int(setup_workers),
                                  ctypes.byref(s)), "amg_server_create")
        self._s = s
        self._n = {}
        if batch_wait_s:
            check(L.amg_server_set_batch_wait(s, float(batch_wait_s)), "amg_server_set_batch_wait")

    def submit(self, prob, b=None, x0=None, tol=1e-8, max_iter=1000):
        """Submit a workloads.Problem (right-hand side prob.b unless b is given)."""
        L = load()
        rp = np.ascontiguousarray(prob.rowptr, dtype=np.int32)
        ci = np.ascontiguousarray(prob.col, dtype=np.int32)
        va = np.ascontiguousarray(prob.val, dtype=np.float64)
        en = np.ascontiguousarray(prob.elem_nodes, dtype=np.int32)
        es = np.ascontiguousarray(prob.elem_sigma, dtype=np.float64)
        xc = np.ascontiguousarray(prob.coords, dtype=np.float64)
        bb = np.ascontiguousarray(prob.b if b is None else b, dtype=np.float64)
        x0p = None
        if x0 is not None:
            x0a = np.ascontiguousarray(x0, dtype=np.float64)
            x0p = _hp(x0a)
        n = rp.shape[0] - 1
        rid = ctypes.c_uint64()
        code = L.amg_server_submit(self._s, n, _hp(rp), _hp(ci), _hp(va), en.shape[0], en.shape[1], _hp(en), _hp(es),
                                   _hp(xc), _hp(bb), x0p, float(tol), int(max_iter), ctypes.byref(rid))
        check(code, "amg_server_submit")
        self._n[rid.value] = n
        return rid.value

    def poll(self, timeout_s=0.0, cap=256):
        ids = (ctypes.c_uint64 * cap)()
        nd = ctypes.c_int32()
        check(load().amg_server_poll(self._s, float(timeout_s), ids, cap, ctypes.byref(nd)), "amg_server_poll")
        return [int(ids[i]) for i in range(nd.value)]

    def result(self, rid):
        n = self._n.pop(rid)
        x = np.empty(n)
        info = SolveInfo()
        rs = RequestStats()
        L = load()
        check(L.amg_server_result(self._s, ctypes.c_uint64(rid), _hp(x), ctypes.byref(info), ctypes.byref(rs)),
              "amg_server_result")
        detail = L.amg_last_error().decode(errors="replace") if info.status != AMG_OK else ""
        out = dict(status=STATUS[info.status], iterations=info.iterations, rel_res=info.rel_res_true,
                   t_solve_s=info.t_solve_s, error=detail)
        tl = {f: getattr(rs, f) for f, _ in RequestStats._fields_}
        return x, out, tl

    def stats(self):
        s = ServerStats()
        check(load().amg_server_info(self._s, ctypes.byref(s)), "amg_server_info")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_s", None) is not None and self._s.value:
            load().amg_server_destroy(self._s)
        self._s = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
