"""ctypes binding of libduq.so (include/duq.h).  Argument marshalling only.

Host inputs are NumPy arrays; device inputs are torch tensors on the HIP
device (PyTorch is used for device memory and streams, nothing else).  The
library must be built (python -m paper_1504_05708_amd.build); loading fails
loudly otherwise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from collections.abc import Sequence
from ctypes import POINTER, Structure, c_char_p, c_double, c_int32, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libduq.so")

DUQ_OK, DUQ_EINVAL, DUQ_ENOMEM, DUQ_EDEVICE, DUQ_EMAXITER, DUQ_ENUMERIC, DUQ_EAGAIN, DUQ_ENOTFOUND = \
    0, -1, -2, -3, -4, -5, -6, -7
DUQ_EINFEASIBLE = -8
# outcomes of a solve that still write x and the multipliers
SOLVE_OUTCOMES = (DUQ_OK, DUQ_EMAXITER, DUQ_EINFEASIBLE)
F64, F32 = 0, 1
HOST, DEVICE = 0, 1
DGM, DFGM = 0, 1
LAST, AVG = 0, 1
CERT, FIXED = 0, 1
INNER_AUTO, INNER_GM, INNER_FGM, INNER_FGM_SIGMA = 0, 1, 2, 3
ACC_F64, ACC_F32 = 0, 1
ENGINE_AUTO, ENGINE_BLOCK, ENGINE_GRID, ENGINE_TILE = 0, 1, 2, 3
SPX_AUTO, SPX_LDS, SPX_IN_PLACE = 0, 1, 2
LB_AUTO, LB_SIGMA, LB_SIGMA_FREE = 0, 1, 2
TRACE_SCALARS = 16

BATCH_UNEVEN, BATCH_SHARED = 0, 1

SERVE_BATCH_NMAX = 1536

EXPORTS = ["duq_default_options", "duq_setup", "duq_max_n", "duq_solve", "duq_get_trace", "duq_get_constants",
           "duq_destroy", "duq_last_error", "duq_strerror", "duq_solve_batch", "duq_server_create",
           "duq_register_shared", "duq_submit", "duq_poll", "duq_server_destroy", "duq_solve_static",
           "duq_plan_params", "duq_solve_planned", "duq_tune_batch", "duq_tune_save", "duq_tune_load",
           "duq_setup_csr"]
STATIC_SCRATCH_BYTES = 64 << 20


class DuqProblem(Structure):
    _fields_ = [("n", c_int32), ("p", c_int32), ("dtype", c_int32), ("memspace", c_int32),
                ("Q", c_void_p), ("G", c_void_p), ("q", c_void_p), ("g", c_void_p),
                ("lb", c_void_p), ("ub", c_void_p), ("rlo", c_void_p), ("rhi", c_void_p)]


class DuqCsr(Structure):
    _fields_ = [("rows", c_int32), ("cols", c_int32), ("rowptr", c_void_p), ("col", c_void_p), ("val", c_void_p)]


class DuqOptions(Structure):
    _fields_ = [("method", c_int32), ("output", c_int32), ("inner_rule", c_int32),
                ("inner_variant", c_int32), ("accumulate", c_int32), ("engine", c_int32),
                ("max_outer", c_int32), ("max_inner", c_int32), ("lanczos_steps", c_int32),
                ("trace_outer", c_int32), ("eps_out", c_double), ("eps_in", c_double),
                ("rho", c_double), ("lam_min", c_double), ("lam_max", c_double),
                ("G_norm2", c_double), ("safety", c_double), ("switch_factor", c_double),
                ("switch_stall", c_int32), ("serve_slice", c_int32), ("out_memspace", c_int32),
                ("batch_wpc", c_int32), ("sigma_in", c_double), ("sparse_x", c_int32), ("lb_cert", c_int32)]


class DuqResult(Structure):
    _fields_ = [("status", c_int32), ("outer_iters", c_int32), ("inner_iters", c_int64),
                ("gt_rows", c_int64), ("f", c_double), ("lb_dual", c_double), ("gap", c_double),
                ("feas", c_double), ("time_ms", c_double), ("f64_outer_iters", c_int32),
                ("engine", c_int32), ("lam_min", c_double), ("lam_max", c_double),
                ("G_norm2", c_double), ("reserved", c_double * 4)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Results(Sequence):
    """Per-instance results of a batch: entry i is converted to a dict when
    it is read, so returning a large batch costs nothing up front."""

    def __init__(self, arr):
        self._arr = arr

    def __len__(self):
        return len(self._arr)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self._arr[j].as_dict() for j in range(*i.indices(len(self._arr)))]
        return self._arr[i].as_dict()


class DuqBatch(Structure):
    _fields_ = [("kind", c_int32), ("B", c_int32), ("dtype", c_int32), ("memspace", c_int32),
                ("n_shared", c_int32), ("p_shared", c_int32),
                ("n", c_void_p), ("p", c_void_p), ("qoff", c_void_p), ("goff", c_void_p),
                ("voff", c_void_p), ("coff", c_void_p), ("Q", c_void_p), ("G", c_void_p),
                ("q", c_void_p), ("g", c_void_p), ("lb", c_void_p), ("ub", c_void_p),
                ("lam_min", c_void_p), ("lam_max", c_void_p), ("G_norm2", c_void_p)]


class DuqPlan(Structure):
    _fields_ = [("eps_in", c_double), ("k_out", c_int64), ("rho_star", c_double), ("k_in", c_int64),
                ("k_total", c_int64)]


class DuqRequest(Structure):
    _fields_ = [("shared_id", c_int32), ("reserved", c_int32), ("prob", DuqProblem)]


class DuqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"duq error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load libduq.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1504_05708_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    L.duq_default_options.argtypes = [POINTER(DuqOptions)]
    L.duq_default_options.restype = None
    L.duq_setup.argtypes = [POINTER(DuqProblem), POINTER(DuqOptions), c_void_p, POINTER(c_void_p)]
    L.duq_setup.restype = c_int32
    L.duq_setup_csr.argtypes = [POINTER(DuqProblem), POINTER(DuqCsr), POINTER(DuqCsr), POINTER(DuqOptions), c_void_p,
                                POINTER(c_void_p)]
    L.duq_setup_csr.restype = c_int32
    L.duq_solve.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(DuqResult)]
    L.duq_solve.restype = c_int32
    L.duq_max_n.argtypes = [c_int32, c_int32, POINTER(c_int32)]
    L.duq_max_n.restype = c_int32
    L.duq_get_trace.argtypes = [c_void_p, c_void_p, c_int32, POINTER(c_int32)]
    L.duq_get_trace.restype = c_int32
    L.duq_get_constants.argtypes = [c_void_p] + [POINTER(c_double)] * 6
    L.duq_get_constants.restype = c_int32
    L.duq_destroy.argtypes = [c_void_p]
    L.duq_destroy.restype = None
    L.duq_last_error.argtypes = []
    L.duq_last_error.restype = c_char_p
    L.duq_strerror.argtypes = [c_int32]
    L.duq_strerror.restype = c_char_p
    L.duq_solve_batch.argtypes = [POINTER(DuqBatch), POINTER(DuqOptions), c_void_p, c_void_p, c_void_p,
                                  POINTER(DuqResult)]
    L.duq_solve_batch.restype = c_int32
    L.duq_server_create.argtypes = [ctypes.c_size_t, POINTER(DuqOptions), POINTER(c_void_p)]
    L.duq_server_create.restype = c_int32
    L.duq_register_shared.argtypes = [c_void_p, POINTER(DuqProblem), POINTER(c_int32)]
    L.duq_register_shared.restype = c_int32
    L.duq_submit.argtypes = [c_void_p, POINTER(DuqRequest), POINTER(ctypes.c_uint64)]
    L.duq_submit.restype = c_int32
    L.duq_poll.argtypes = [c_void_p, ctypes.c_uint64, c_void_p, c_void_p, POINTER(DuqResult)]
    L.duq_poll.restype = c_int32
    L.duq_server_destroy.argtypes = [c_void_p]
    L.duq_server_destroy.restype = None
    L.duq_solve_static.argtypes = [POINTER(DuqProblem), POINTER(DuqOptions), c_void_p, c_void_p, c_void_p,
                                   POINTER(DuqResult)]
    L.duq_solve_static.restype = c_int32
    L.duq_tune_batch.argtypes = [POINTER(DuqBatch), POINTER(DuqOptions), c_void_p, POINTER(c_int32),
                                 POINTER(c_double)]
    L.duq_tune_batch.restype = c_int32
    L.duq_tune_save.argtypes = [c_char_p]
    L.duq_tune_save.restype = c_int32
    L.duq_tune_load.argtypes = [c_char_p]
    L.duq_tune_load.restype = c_int32
    L.duq_plan_params.argtypes = [c_int32, c_double, c_double, c_double, c_double, c_double, c_double,
                                  POINTER(DuqPlan)]
    L.duq_plan_params.restype = c_int32
    L.duq_solve_planned.argtypes = [c_void_p, c_double, c_double, c_int32, c_void_p, c_void_p, POINTER(DuqResult),
                                    POINTER(c_double), POINTER(c_int32)]
    L.duq_solve_planned.restype = c_int32
    _lib = L
    return L


def last_error() -> str:
    return lib().duq_last_error().decode()


def max_n(p: int, engine: int = 2) -> int:
    """duq_max_n: largest n duq_setup accepts for p rows of G on `engine`
    (default DUQ_ENGINE_GRID) on the current device."""
    v = c_int32()
    rc = lib().duq_max_n(p, engine, ctypes.byref(v))
    if rc != DUQ_OK:
        raise DuqError(rc, last_error())
    return v.value


def default_options(**kw) -> DuqOptions:
    o = DuqOptions()
    lib().duq_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(c_void_p)


def _stream_of(t):
    if t is not None and hasattr(t, "data_ptr"):
        import torch
        return c_void_p(torch.cuda.current_stream(t.device).cuda_stream)
    return c_void_p(None)


def _csr_parts(M, dtype=None):
    """(rows, cols, row offsets int64, column indices int32, values) of a
    compressed-row matrix: an object with rowptr/col/val/rows/cols, or one
    with indptr/indices/data/shape (scipy's CSR layout)."""
    if hasattr(M, "rowptr"):
        rows, cols, rp, ci, v = M.rows, M.cols, M.rowptr, M.col, M.val
    else:
        (rows, cols), rp, ci, v = M.shape, M.indptr, M.indices, M.data
    v = np.ascontiguousarray(v, dtype=dtype if dtype is not None else v.dtype)
    return (int(rows), int(cols), np.ascontiguousarray(rp, dtype=np.int64), np.ascontiguousarray(ci, dtype=np.int32), v)


def _is_csr(M) -> bool:
    return hasattr(M, "rowptr") or hasattr(M, "indptr")


class Solver:
    """One QP set up on the device (duq_setup) and solved with duq_solve.

    Q, G: NumPy float64/float32 arrays (copied) or torch tensors on the GPU
    (borrowed: they must outlive the solver), or both compressed-row matrices
    on the host (duq_setup_csr; see _csr_parts for the accepted forms).
    q, g, lb, ub: float64 of the same kind.  rlo, rhi (optional, both or
    neither): row bounds rlo <= G u + g <= rhi (equality where rlo = rhi,
    +-inf for no side)."""

    def __init__(self, Q, q, G, g, lb, ub, rlo=None, rhi=None, **opts):
        self._keep = []
        if _is_csr(Q):
            self._setup_csr(Q, q, G, g, lb, ub, rlo, rhi, opts)
            return
        dev = hasattr(Q, "data_ptr")
        if dev:
            import torch
            dt = {torch.float64: F64, torch.float32: F32}[Q.dtype]
            for t in (q, g, lb, ub):
                assert t.dtype == torch.float64 and t.is_contiguous()
            Q = Q.contiguous()
            G = G.contiguous()
        else:
            Q = np.ascontiguousarray(Q)
            dt = {np.dtype(np.float64): F64, np.dtype(np.float32): F32}[Q.dtype]
            G = np.ascontiguousarray(G, dtype=Q.dtype)
            q, g, lb, ub = (np.ascontiguousarray(v, dtype=np.float64) for v in (q, g, lb, ub))
            if rlo is not None:
                rlo, rhi = (np.ascontiguousarray(v, dtype=np.float64) for v in (rlo, rhi))
        self._keep = [Q, G, q, g, lb, ub, rlo, rhi]
        n, p = int(Q.shape[0]), int(G.shape[0])
        self.n, self.p = n, p
        self.rows = rlo is not None
        prob = DuqProblem(n, p, dt, DEVICE if dev else HOST, _ptr(Q), _ptr(G) if p else None,
                          _ptr(q), _ptr(g) if p else None, _ptr(lb), _ptr(ub), _ptr(rlo), _ptr(rhi))
        self.opts = default_options(**opts)
        h = c_void_p()
        rc = lib().duq_setup(ctypes.byref(prob), ctypes.byref(self.opts), _stream_of(Q if dev else None),
                             ctypes.byref(h))
        if rc != DUQ_OK:
            raise DuqError(rc, last_error())
        self._h = h
        if not dev:
            self._keep = []   # host data was copied

    def _setup_csr(self, Q, q, G, g, lb, ub, rlo, rhi, opts):
        nq, qcols, qrp, qci, qv = _csr_parts(Q)
        if qv.dtype not in (np.float64, np.float32):
            qv = qv.astype(np.float64)
        dt = F64 if qv.dtype == np.float64 else F32
        cg = None
        p = 0
        if G is not None:
            p, gcols, grp, gci, gv = _csr_parts(G, qv.dtype)
            cg = DuqCsr(p, gcols, _ptr(grp), _ptr(gci), _ptr(gv))
        g = np.zeros(0) if g is None else g
        q, g, lb, ub = (np.ascontiguousarray(v, dtype=np.float64) for v in (q, g, lb, ub))
        if rlo is not None:
            rlo, rhi = (np.ascontiguousarray(v, dtype=np.float64) for v in (rlo, rhi))
        self.n, self.p = nq, p
        self.rows = rlo is not None
        cq = DuqCsr(nq, qcols, _ptr(qrp), _ptr(qci), _ptr(qv))
        prob = DuqProblem(nq, p, dt, HOST, None, None, _ptr(q), _ptr(g) if p else None, _ptr(lb), _ptr(ub),
                          _ptr(rlo), _ptr(rhi))
        self.opts = default_options(**opts)
        h = c_void_p()
        rc = lib().duq_setup_csr(ctypes.byref(prob), ctypes.byref(cq), ctypes.byref(cg) if cg is not None else None,
                                 ctypes.byref(self.opts),
                                 c_void_p(None), ctypes.byref(h))
        if rc != DUQ_OK:
            raise DuqError(rc, last_error())
        self._h = h

    def solve(self, x0=None, lam0=None, check=True):
        x = np.empty(self.n)
        lam = np.empty(self.p)
        res = DuqResult()
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        l0a = None if lam0 is None else np.ascontiguousarray(lam0, dtype=np.float64)
        rc = lib().duq_solve(self._h, _ptr(x0a), _ptr(l0a), _ptr(x), _ptr(lam) if self.p else None,
                             ctypes.byref(res))
        if check and rc not in SOLVE_OUTCOMES:
            raise DuqError(rc, last_error())
        return x, lam, res.as_dict()

    def trace(self, max_records: int):
        per = TRACE_SCALARS + (4 if self.rows else 2) * self.p + self.n
        out = np.zeros((max_records, per))
        nrec = c_int32()
        rc = lib().duq_get_trace(self._h, _ptr(out), max_records, ctypes.byref(nrec))
        if rc != DUQ_OK:
            raise DuqError(rc, last_error())
        out = out[:nrec.value]
        p, n = self.p, self.n
        S = TRACE_SCALARS
        tr = dict(scalars=out[:, :S], lam=out[:, S:S + p], mu=out[:, S + p:S + 2 * p],
                  u=out[:, S + 2 * p:S + 2 * p + n])
        if self.rows:   # lower sides of the row bounds
            tr.update(lam_lo=out[:, S + 2 * p + n:S + 3 * p + n], mu_lo=out[:, S + 3 * p + n:S + 4 * p + n])
        return tr

    def solve_planned(self, eps: float, R0: float, max_rounds: int = 12, check=True):
        """duq_solve_planned: eps_in and max_outer from eq. choose_ein for a
        guess R of R_d, doubled per round until the test at eps passes.
        Returns (x, lam, result dict with 'R' and 'rounds')."""
        x = np.empty(self.n)
        lam = np.empty(max(self.p, 1))
        res = DuqResult()
        R, rounds = c_double(), c_int32()
        rc = lib().duq_solve_planned(self._h, eps, R0, max_rounds, _ptr(x), _ptr(lam), ctypes.byref(res),
                                     ctypes.byref(R), ctypes.byref(rounds))
        if check and rc not in SOLVE_OUTCOMES:
            raise DuqError(rc, last_error())
        d = res.as_dict()
        d.update(R=R.value, rounds=rounds.value)
        return x, lam[:self.p], d

    def constants(self) -> dict:
        vals = [c_double() for _ in range(6)]
        rc = lib().duq_get_constants(self._h, *[ctypes.byref(v) for v in vals])
        if rc != DUQ_OK:
            raise DuqError(rc, last_error())
        return dict(zip(["lam_min", "lam_max", "G_norm2", "Ld", "L_in", "sigma_in"], [v.value for v in vals]))

    def close(self):
        if getattr(self, "_h", None):
            lib().duq_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_params(method: int, eps: float, Ld: float, Rd: float, L_in: float = 0.0, sigma_in: float = 0.0,
                D_U: float = 0.0) -> dict:
    """duq_plan_params: eq. choose_ein (eps_in, k_out), rho* and k_in."""
    out = DuqPlan()
    rc = lib().duq_plan_params(method, eps, Ld, Rd, L_in, sigma_in, D_U, ctypes.byref(out))
    if rc != DUQ_OK:
        raise DuqError(rc, last_error())
    return {k: getattr(out, k) for k, _ in out._fields_}


def solve_static(Q, q, G, g, lb, ub, x_out, lam_out, check=True, **opts):
    """duq_solve_static: one solve with the workspace in the library's static
    device scratch (no allocation in the call).  Every array is a torch tensor
    on the GPU (Q, G float64 or float32; the rest float64); x_out (n) and
    lam_out (p) receive the answer.  lam_min, lam_max, G_norm2 must be given.
    Returns (status, result dict)."""
    import torch
    dt = {torch.float64: F64, torch.float32: F32}[Q.dtype]
    for t in (q, g, lb, ub, x_out, lam_out):
        assert t.dtype == torch.float64 and t.is_contiguous()
    assert Q.is_contiguous() and G.is_contiguous()
    n, p = int(Q.shape[0]), int(G.shape[0])
    prob = DuqProblem(n, p, dt, DEVICE, _ptr(Q), _ptr(G) if p else None, _ptr(q), _ptr(g) if p else None,
                      _ptr(lb), _ptr(ub))
    o = default_options(**opts)
    res = DuqResult()
    rc = lib().duq_solve_static(ctypes.byref(prob), ctypes.byref(o), _stream_of(Q), _ptr(x_out),
                                _ptr(lam_out) if p else None, ctypes.byref(res))
    if check and rc not in SOLVE_OUTCOMES:
        raise DuqError(rc, last_error())
    return rc, res.as_dict()


def solve_batch_uneven(batch, constants=None, check=True, **opts):
    """duq_solve_batch on a packed gen.UnevenBatch (host arrays or torch
    device tensors).

    constants: optional (lam_min, lam_max, G_norm2) arrays of length B.
    device_out=True keeps X, Lam in device memory (torch tensors).
    Returns (X, Lam, results) with X, Lam packed like q and g."""
    B = batch.B
    n = np.ascontiguousarray(batch.n, dtype=np.int32)
    p = np.ascontiguousarray(batch.p, dtype=np.int32)
    offs = [np.ascontiguousarray(v, dtype=np.int64) for v in (batch.qoff, batch.goff, batch.voff, batch.coff)]
    dev = hasattr(batch.Q, "data_ptr")
    if dev:   # torch tensors on the GPU: borrowed
        import torch
        Q, G = batch.Q, batch.G
        dt = {torch.float64: F64, torch.float32: F32}[Q.dtype]
        vecs = [batch.q, batch.g, batch.lb, batch.ub]
    else:
        Q = np.ascontiguousarray(batch.Q)
        G = np.ascontiguousarray(batch.G, dtype=Q.dtype)
        dt = {np.dtype(np.float64): F64, np.dtype(np.float32): F32}[Q.dtype]
        vecs = [np.ascontiguousarray(v, dtype=np.float64) for v in (batch.q, batch.g, batch.lb, batch.ub)]
    cs = [None, None, None] if constants is None else [np.ascontiguousarray(c, dtype=np.float64)
                                                       for c in constants]
    b = DuqBatch(BATCH_UNEVEN, B, dt, DEVICE if dev else HOST, 0, 0, _ptr(n), _ptr(p), *[_ptr(o) for o in offs],
                 _ptr(Q), _ptr(G), *[_ptr(v) for v in vecs], *[_ptr(c) for c in cs])
    return _run_batch(b, B, int(batch.q.shape[0]), int(batch.g.shape[0]), check, opts)


def tune_batch(batch, **opts):
    """duq_tune_batch on a packed gen.UnevenBatch (host arrays): returns
    (best workgroups per CU, device ms per candidate 1..3)."""
    n = np.ascontiguousarray(batch.n, dtype=np.int32)
    p = np.ascontiguousarray(batch.p, dtype=np.int32)
    offs = [np.ascontiguousarray(v, dtype=np.int64) for v in (batch.qoff, batch.goff, batch.voff, batch.coff)]
    Q = np.ascontiguousarray(batch.Q)
    dt = {np.dtype(np.float64): F64, np.dtype(np.float32): F32}[Q.dtype]
    G = np.ascontiguousarray(batch.G, dtype=Q.dtype)
    vecs = [np.ascontiguousarray(v, dtype=np.float64) for v in (batch.q, batch.g, batch.lb, batch.ub)]
    b = DuqBatch(BATCH_UNEVEN, batch.B, dt, HOST, 0, 0, _ptr(n), _ptr(p), *[_ptr(o) for o in offs],
                 _ptr(Q), _ptr(G), *[_ptr(v) for v in vecs], None, None, None)
    o = default_options(**opts)
    best = c_int32()
    ms = (c_double * 3)()
    rc = lib().duq_tune_batch(ctypes.byref(b), ctypes.byref(o), c_void_p(None), ctypes.byref(best), ms)
    if rc != DUQ_OK:
        raise DuqError(rc, last_error())
    return best.value, list(ms)


def tune_save(path: str):
    rc = lib().duq_tune_save(path.encode())
    if rc != DUQ_OK:
        raise DuqError(rc, last_error())


def tune_load(path: str):
    rc = lib().duq_tune_load(path.encode())
    if rc != DUQ_OK:
        raise DuqError(rc, last_error())


def solve_batch_shared(Q, G, lb, ub, q, g, constants=None, check=True, **opts):
    """duq_solve_batch on B instances sharing Q, G, lb, ub; q is B x n, g is B x p.

    constants: optional (lam_min, lam_max, G_norm2) scalars.  device_out=True
    keeps X, Lam in device memory (torch tensors)."""
    dev = hasattr(Q, "data_ptr")
    if dev:   # torch tensors on the GPU: borrowed
        import torch
        dt = {torch.float64: F64, torch.float32: F32}[Q.dtype]
    else:
        Q = np.ascontiguousarray(Q)
        dt = {np.dtype(np.float64): F64, np.dtype(np.float32): F32}[Q.dtype]
        G = np.ascontiguousarray(G, dtype=Q.dtype)
        q = np.ascontiguousarray(q, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        lb = np.ascontiguousarray(lb, dtype=np.float64)
        ub = np.ascontiguousarray(ub, dtype=np.float64)
    B, n = int(q.shape[0]), int(q.shape[1])
    p = int(g.shape[1])
    cs = [None, None, None] if constants is None else [np.array([c], dtype=np.float64) for c in constants]
    b = DuqBatch(BATCH_SHARED, B, dt, DEVICE if dev else HOST, n, p, None, None, None, None, None, None,
                 _ptr(Q), _ptr(G), _ptr(q), _ptr(g), _ptr(lb), _ptr(ub), *[_ptr(c) for c in cs])
    X, Lam, res = _run_batch(b, B, B * n, B * p, check, opts)
    return X.reshape(B, n), Lam.reshape(B, p), res


def _run_batch(b, B, nx, nl, check, opts):
    device_out = opts.pop("device_out", False)
    o = default_options(**opts)
    if device_out:   # outputs stay in device memory (torch tensors)
        import torch
        o.out_memspace = DEVICE
        X = torch.empty(max(nx, 1), dtype=torch.float64, device="cuda")
        Lam = torch.empty(max(nl, 1), dtype=torch.float64, device="cuda")
    else:
        X = np.empty(max(nx, 1))
        Lam = np.empty(max(nl, 1))
    res = (DuqResult * B)()
    rc = lib().duq_solve_batch(ctypes.byref(b), ctypes.byref(o), c_void_p(None), _ptr(X), _ptr(Lam), res)
    if check and rc not in SOLVE_OUTCOMES:
        raise DuqError(rc, last_error())
    return X[:nx], Lam[:nl], Results(res)


class Server:
    """Serving loop (duq_server_*): submit QPs, poll for their results.

    Requests are host NumPy data.  Own problems are (Q, q, G, g, lb, ub);
    requests against a registered system (register_shared) give q and g."""

    def __init__(self, hbm_budget_bytes: int = 0, **opts):
        self.opts = default_options(**opts)
        s = c_void_p()
        rc = lib().duq_server_create(hbm_budget_bytes, ctypes.byref(self.opts), ctypes.byref(s))
        if rc != DUQ_OK:
            raise DuqError(rc, last_error())
        self._s = s
        self._sizes = {}     # ticket -> (n, p)
        self._shared = {}    # id -> (n, p)

    @staticmethod
    def _problem(Q, q, G, g, lb, ub):
        Q = np.ascontiguousarray(Q)
        dt = {np.dtype(np.float64): F64, np.dtype(np.float32): F32}[Q.dtype]
        n = int(Q.shape[0])
        G = np.ascontiguousarray(G, dtype=Q.dtype).reshape(-1, n)
        p = int(G.shape[0])
        vecs = [None if v is None else np.ascontiguousarray(v, dtype=np.float64) for v in (q, g, lb, ub)]
        keep = [Q, G] + vecs
        prob = DuqProblem(n, p, dt, HOST, _ptr(Q), _ptr(G) if p else None, _ptr(vecs[0]),
                          _ptr(vecs[1]) if p else None, _ptr(vecs[2]), _ptr(vecs[3]))
        return prob, keep, n, p

    def register_shared(self, Q, G, lb, ub) -> int:
        prob, keep, n, p = self._problem(Q, None, G, None, lb, ub)
        sid = c_int32()
        rc = lib().duq_register_shared(self._s, ctypes.byref(prob), ctypes.byref(sid))
        if rc != DUQ_OK:
            raise DuqError(rc, last_error())
        self._shared[sid.value] = (n, p)
        return sid.value

    def submit(self, Q=None, q=None, G=None, g=None, lb=None, ub=None, shared_id: int = -1) -> int:
        if shared_id >= 0:
            qa = np.ascontiguousarray(q, dtype=np.float64)
            ga = np.ascontiguousarray(g, dtype=np.float64)
            n, p = self._shared.get(shared_id, (qa.size, ga.size))   # the library checks the id
            keep = [qa, ga]
            prob = DuqProblem(n, p, F64, HOST, None, None, _ptr(qa), _ptr(ga) if p else None, None, None)
        else:
            prob, keep, n, p = self._problem(Q, q, G, g, lb, ub)
        req = DuqRequest(shared_id, 0, prob)
        t = ctypes.c_uint64()
        rc = lib().duq_submit(self._s, ctypes.byref(req), ctypes.byref(t))
        del keep
        if rc != DUQ_OK:
            raise DuqError(rc, last_error())
        self._sizes[t.value] = (n, p)
        return t.value

    def poll(self, ticket: int):
        """None while pending; else (status, x, lam, result dict)."""
        n, p = self._sizes.get(ticket, (0, 0))
        x = np.empty(max(n, 1))
        lam = np.empty(max(p, 1))
        res = DuqResult()
        rc = lib().duq_poll(self._s, ticket, _ptr(x), _ptr(lam), ctypes.byref(res))
        if rc == DUQ_EAGAIN:
            return None
        if rc == DUQ_ENOTFOUND:
            raise DuqError(rc, last_error())
        self._sizes.pop(ticket, None)
        return rc, x[:n], lam[:p], res.as_dict()

    def wait(self, ticket: int, timeout: float = 60.0, interval: float = 1e-4):
        import time
        t0 = time.perf_counter()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError(f"ticket {ticket} not finished after {timeout} s")
            time.sleep(interval)

    def close(self):
        if getattr(self, "_s", None):
            lib().duq_server_destroy(self._s)
            self._s = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
