"""Python binding of libsrot (include/srot.h): argument marshalling only.

Every function below has the name of the C entry point it calls and does no
arithmetic of the method: tensors are passed by device pointer, the stream is
torch's current stream, and the library's status codes become exceptions.
The library must be built (`__graft_entry__.build()`); without it every call
raises -- there is no fallback path.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrot.so")

SROT_OK = 0
SROT_NOT_CONVERGED = 1
SROT_EINVAL = -1
SROT_ENOMEM = -2
SROT_ENONFINITE = -3
SROT_EHIP = -4
SROT_ECAPACITY = -5

SROT_ELS = 0
SROT_DEC = 1
SROT_STEP_AWAY = 1
SROT_STEP_PAIRWISE = 2
SROT_UNIFORM = 0
SROT_PERMUTE = 1
SROT_COST_F32 = 0
SROT_COST_F64 = 1
SROT_COST_SQEUCLID = 2
SROT_GA_INIT = 2.0 ** 300
SROT_CHAIN_PREFETCH = 1
SROT_CHAIN_SCREENED = 2
SROT_CHAIN_GLOBAL = 3
SROT_CHAIN_WIDE = 4
SROT_CHAIN_TEAM = 5
SROT_NOALLOC_SCRATCH_BYTES = 8 << 20


class SrotError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"srot status {status}: {msg}")
        self.status = status


class srot_options(ctypes.Structure):
    _fields_ = [("w", ctypes.c_double), ("step_rule", ctypes.c_int32),
                ("sampling", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("eps", ctypes.c_double), ("max_passes", ctypes.c_int64),
                ("gap_every", ctypes.c_int32), ("cost", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64


def load():
    """Loads libsrot.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    L.srot_default_options.argtypes = [ctypes.POINTER(srot_options)]
    L.srot_default_options.restype = None
    L.srot_workspace_size.argtypes = [_i64, _i64, ctypes.POINTER(srot_options)]
    L.srot_workspace_size.restype = ctypes.c_size_t
    L.srot_init.argtypes = [ctypes.POINTER(_vp), _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp,
                            ctypes.c_size_t, ctypes.POINTER(srot_options), _vp]
    L.srot_init.restype = ctypes.c_int
    L.srot_step.argtypes = [_vp, _i64, _vp, _vp, _vp]
    L.srot_step.restype = ctypes.c_int
    L.srot_gap.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), _vp, _vp]
    L.srot_gap.restype = ctypes.c_int
    L.srot_gap_async.argtypes = [_vp, _vp]
    L.srot_gap_async.restype = ctypes.c_int
    L.srot_solve.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]
    L.srot_solve.restype = ctypes.c_int
    L.srot_get_plan.argtypes = [_vp, _vp, _vp]
    L.srot_get_plan.restype = ctypes.c_int
    L.srot_get_plan_csr.argtypes = [_vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64)]
    L.srot_get_plan_csr.restype = ctypes.c_int
    L.srot_get_state.argtypes = [_vp, ctypes.POINTER(_i64)]
    L.srot_get_state.restype = ctypes.c_int
    L.srot_set_state.argtypes = [_vp, _vp, _vp, _i64]
    L.srot_set_state.restype = ctypes.c_int
    L.srot_chain_stats.argtypes = [_vp, _vp]
    L.srot_chain_stats.restype = ctypes.c_int
    L.srot_backward.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]
    L.srot_backward.restype = ctypes.c_int
    L.srot_backward_noalloc.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]
    L.srot_backward_noalloc.restype = ctypes.c_int
    L.srot_workspace_size_batched.argtypes = [ctypes.c_int32, _vp, _vp, ctypes.POINTER(srot_options)]
    L.srot_workspace_size_batched.restype = ctypes.c_size_t
    L.srot_init_batched.argtypes = [ctypes.POINTER(_vp), ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                    ctypes.c_size_t, ctypes.POINTER(srot_options), ctypes.c_int32, _vp]
    L.srot_init_batched.restype = ctypes.c_int
    L.srot_solve_batched.argtypes = [_vp, _vp, _vp, _vp]
    L.srot_solve_batched.restype = ctypes.c_int
    L.srot_get_plan_batched.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
    L.srot_get_plan_batched.restype = ctypes.c_int
    L.srot_get_tiles_batched.argtypes = [_vp, _vp, _vp]
    L.srot_get_tiles_batched.restype = ctypes.c_int
    L.srot_destroy_batched.argtypes = [_vp]
    L.srot_destroy_batched.restype = None
    L.srot_fw_steps.argtypes = [_vp, _i64, _vp]
    L.srot_fw_steps.restype = ctypes.c_int
    L.srot_fw_solve.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]
    L.srot_fw_solve.restype = ctypes.c_int
    L.srot_step_variant.argtypes = [_vp, ctypes.c_int, _i64, _vp, _vp, _vp, _vp]
    L.srot_step_variant.restype = ctypes.c_int
    L.srot_solve_variant.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]
    L.srot_solve_variant.restype = ctypes.c_int
    L.srot_ga_reset.argtypes = [_vp, ctypes.c_double]
    L.srot_ga_reset.restype = ctypes.c_int
    L.srot_ga_refresh.argtypes = [_vp]
    L.srot_ga_refresh.restype = ctypes.c_int
    L.srot_ga_weights.argtypes = [_vp, _vp]
    L.srot_ga_weights.restype = ctypes.c_int
    L.srot_step_ga.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp, _vp]
    L.srot_step_ga.restype = ctypes.c_int
    L.srot_solve_ga.argtypes = [_vp, ctypes.c_double, _i64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]
    L.srot_solve_ga.restype = ctypes.c_int
    L.srot_barycentric.argtypes = [_vp, _vp]
    L.srot_barycentric.restype = ctypes.c_int
    L.srot_destroy.argtypes = [_vp]
    L.srot_destroy.restype = None
    L.srot_strerror.argtypes = [ctypes.c_int]
    L.srot_strerror.restype = ctypes.c_char_p
    L.srot_last_error.argtypes = []
    L.srot_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status, allow=(SROT_OK,)):
    if status in allow:
        return status
    L = load()
    raise SrotError(status, f"{L.srot_strerror(status).decode()}: {L.srot_last_error().decode()}")


def _ptr(t, dtype=None, numel=0, pinned_ok=False):
    """Device pointer of a contiguous CUDA tensor (or None).  The library
    dereferences it on the GPU, so anything else is refused here: a host
    pointer would fault the device."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise SrotError(SROT_EINVAL, f"expected a torch tensor, got {type(t).__name__}")
    if not (t.is_cuda or (pinned_ok and t.is_pinned())):
        raise SrotError(SROT_EINVAL, "expected a CUDA tensor" + (" or pinned host tensor" if pinned_ok else ""))
    if not t.is_contiguous():
        raise SrotError(SROT_EINVAL, "expected a contiguous tensor")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise SrotError(SROT_EINVAL, f"expected dtype {dtype}, got {t.dtype}")
    if t.numel() < numel:
        raise SrotError(SROT_EINVAL, f"tensor has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


_F32, _F64, _I32 = torch.float32, torch.float64, torch.int32


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def srot_default_options(**kw):
    opt = srot_options()
    load().srot_default_options(ctypes.byref(opt))
    for k, v in kw.items():
        setattr(opt, k, v)
    return opt


def srot_workspace_size(m, n, opt):
    return int(load().srot_workspace_size(m, n, ctypes.byref(opt)))


def srot_init(m, n, C, X, Y, a, b, workspace, opt):
    h = ctypes.c_void_p()
    cdt = _F64 if opt.cost == SROT_COST_F64 else _F32
    _check(load().srot_init(ctypes.byref(h), m, n, _ptr(C, cdt, m * n), _ptr(X, _F32, 3 * m), _ptr(Y, _F32, 3 * n),
                            _ptr(a, _F64, m), _ptr(b, _F64, n),
                            _ptr(workspace), workspace.numel() * workspace.element_size(),
                            ctypes.byref(opt), _stream()))
    return h


def srot_step(h, nsteps, idx=None, trace_j=None, trace_gamma=None):
    _check(load().srot_step(h, nsteps, _ptr(idx, _I32, nsteps), _ptr(trace_j, _I32, nsteps),
                            _ptr(trace_gamma, _F64, nsteps)))


def srot_gap(h, row_gap=None, row_argmin=None):
    out = (ctypes.c_double * 3)()
    _check(load().srot_gap(h, out, _ptr(row_gap, _F64), _ptr(row_argmin, _I32)))
    return out[0], out[1], out[2]


def srot_gap_async(h, out5):
    """Enqueues the gap sweep; out5 (5 doubles, device or pinned) receives
    {g, f, D, <T,C>, ||r||^2} when the stream gets there."""
    _check(load().srot_gap_async(h, _ptr(out5, _F64, 5, pinned_ok=True)))


def srot_solve(h):
    out = (ctypes.c_double * 3)()
    passes = _i64()
    st = _check(load().srot_solve(h, out, ctypes.byref(passes)), allow=(SROT_OK, SROT_NOT_CONVERGED))
    return st, (out[0], out[1], out[2]), passes.value


def srot_get_plan(h, T_out=None, r_out=None):
    _check(load().srot_get_plan(h, _ptr(T_out, _F64), _ptr(r_out, _F64)))


def srot_get_plan_csr(h, row_ptr, col=None, val=None):
    """Writes the plan's compressed sparse rows into row_ptr (m + 1 int32)
    and, when they hold enough entries, col (int32) and val (float64);
    returns the number of entries (SrotError with status SROT_ECAPACITY when
    col and val are too small; without them it only counts)."""
    count_only = col is None or val is None
    cap = 0 if count_only else min(col.numel(), val.numel())
    nnz = _i64()
    _check(load().srot_get_plan_csr(h, _ptr(row_ptr, _I32, 1), None if count_only else _ptr(col, _I32),
                                    None if count_only else _ptr(val, _F64), cap, ctypes.byref(nnz)),
           allow=(SROT_OK, SROT_ECAPACITY) if count_only else (SROT_OK,))
    return nnz.value


def srot_get_state(h):
    k = _i64()
    _check(load().srot_get_state(h, ctypes.byref(k)))
    return k.value


def srot_set_state(h, T_in, k, r_in=None):
    _check(load().srot_set_state(h, _ptr(T_in, _F64), _ptr(r_in, _F64), k))


def srot_chain_stats(h):
    out = (ctypes.c_int64 * 4)()
    _check(load().srot_chain_stats(h, out))
    return list(out)


def srot_backward(h, grad_out, dC=None, dX=None, dY=None, da=None, db=None):
    _check(load().srot_backward(h, float(grad_out), _ptr(dC, (_F32, _F64)), _ptr(dX, _F32), _ptr(dY, _F32),
                                _ptr(da, _F64), _ptr(db, _F64)))


def srot_backward_noalloc(h, grad_out, dC=None, dX=None, dY=None, da=None, db=None):
    """srot_backward with its scratch in the library's static device array
    (no allocation, no workspace scratch)."""
    _check(load().srot_backward_noalloc(h, float(grad_out), _ptr(dC, (_F32, _F64)), _ptr(dX, _F32),
                                        _ptr(dY, _F32), _ptr(da, _F64), _ptr(db, _F64)))


def srot_fw_steps(h, iters, trace_gamma=None):
    _check(load().srot_fw_steps(h, int(iters), _ptr(trace_gamma, _F64, iters)))


def srot_fw_solve(h):
    out = (ctypes.c_double * 3)()
    iters = _i64()
    st = _check(load().srot_fw_solve(h, out, ctypes.byref(iters)), allow=(SROT_OK, SROT_NOT_CONVERGED))
    return st, (out[0], out[1], out[2]), iters.value


def srot_step_variant(h, variant, nsteps, idx=None, trace_j=None, trace_away=None, trace_gamma=None):
    _check(load().srot_step_variant(h, int(variant), int(nsteps), _ptr(idx, _I32, nsteps),
                                    _ptr(trace_j, _I32, nsteps), _ptr(trace_away, _I32, nsteps),
                                    _ptr(trace_gamma, _F64, nsteps)))


def srot_solve_variant(h, variant):
    out = (ctypes.c_double * 3)()
    passes = _i64()
    st = _check(load().srot_solve_variant(h, int(variant), out, ctypes.byref(passes)),
                allow=(SROT_OK, SROT_NOT_CONVERGED))
    return st, (out[0], out[1], out[2]), passes.value


def srot_ga_reset(h, init=SROT_GA_INIT):
    _check(load().srot_ga_reset(h, float(init)))


def srot_ga_refresh(h):
    _check(load().srot_ga_refresh(h))


def srot_ga_weights(h, W_out):
    _check(load().srot_ga_weights(h, _ptr(W_out, _F64)))


def srot_step_ga(h, nsteps, u=None, trace_i=None, trace_j=None, trace_gamma=None, trace_g=None):
    _check(load().srot_step_ga(h, int(nsteps), _ptr(u, _F64, nsteps), _ptr(trace_i, _I32, nsteps),
                               _ptr(trace_j, _I32, nsteps), _ptr(trace_gamma, _F64, nsteps),
                               _ptr(trace_g, _F64, nsteps)))


def srot_solve_ga(h, init=0.0, period=1):
    out = (ctypes.c_double * 3)()
    passes = _i64()
    st = _check(load().srot_solve_ga(h, float(init), int(period), out, ctypes.byref(passes)),
                allow=(SROT_OK, SROT_NOT_CONVERGED))
    return st, (out[0], out[1], out[2]), passes.value


def srot_barycentric(h, Xhat):
    _check(load().srot_barycentric(h, _ptr(Xhat, _F32)))


def srot_destroy(h):
    if h:
        load().srot_destroy(h)


def _host_ptr(arr):
    return None if arr is None else ctypes.c_void_p(arr.ctypes.data)


def srot_workspace_size_batched(m, n, opt):
    import numpy as np
    m = np.ascontiguousarray(m, dtype=np.int64)
    n = np.ascontiguousarray(n, dtype=np.int64)
    return int(load().srot_workspace_size_batched(len(m), _host_ptr(m), _host_ptr(n), ctypes.byref(opt)))


def srot_init_batched(m, n, c_off, C, a, b, workspace, opt, tune=0):
    import numpy as np
    m = np.ascontiguousarray(m, dtype=np.int64)
    n = np.ascontiguousarray(n, dtype=np.int64)
    c_off = None if c_off is None else np.ascontiguousarray(c_off, dtype=np.int64)
    h = ctypes.c_void_p()
    _check(load().srot_init_batched(ctypes.byref(h), len(m), _host_ptr(m), _host_ptr(n), _host_ptr(c_off),
                                    _ptr(C, _F32), _ptr(a, _F64), _ptr(b, _F64), _ptr(workspace),
                                    workspace.numel() * workspace.element_size(), ctypes.byref(opt),
                                    int(tune), _stream()))
    return h


def srot_solve_batched(h, count):
    import numpy as np
    out3 = np.empty((count, 3), dtype=np.float64)
    passes = np.empty(count, dtype=np.int64)
    status = np.empty(count, dtype=np.int32)
    st = _check(load().srot_solve_batched(h, _host_ptr(out3), _host_ptr(passes), _host_ptr(status)),
                allow=(SROT_OK, SROT_NOT_CONVERGED))
    return st, out3, passes, status


def srot_get_plan_batched(h, p, T_out=None, r_out=None):
    _check(load().srot_get_plan_batched(h, int(p), _ptr(T_out, _F64), _ptr(r_out, _F64)))


def srot_get_tiles_batched(h, count):
    import numpy as np
    tiles = np.empty((count, 3), dtype=np.int32)
    ms = np.empty(count, dtype=np.float32)
    _check(load().srot_get_tiles_batched(h, _host_ptr(tiles), _host_ptr(ms)))
    return tiles, ms


def srot_destroy_batched(h):
    if h:
        load().srot_destroy_batched(h)


class BatchSolver:
    """Many independent problems with stored FP32 costs (srot_init_batched).

    Cs: list of (m_p, n_p) float32 CUDA tensors; As, Bs: lists of float64 CUDA
    tensors.  The costs are packed into one buffer with 16-byte aligned
    offsets; the weights back to back."""

    def __init__(self, Cs, As, Bs, tune=False, **options):
        import numpy as np
        options.setdefault("cost", SROT_COST_F32)
        self.opt = srot_default_options(**options)
        self.count = len(Cs)
        self.m = np.array([c.shape[0] for c in Cs], dtype=np.int64)
        self.n = np.array([c.shape[1] for c in Cs], dtype=np.int64)
        dev = Cs[0].device
        sizes = self.m * self.n
        padded = (sizes + 3) // 4 * 4
        self.c_off = np.concatenate([[0], np.cumsum(padded)[:-1]]).astype(np.int64)
        self.C = torch.zeros(int(padded.sum()), dtype=torch.float32, device=dev)
        for p, c in enumerate(Cs):
            self.C[int(self.c_off[p]):int(self.c_off[p] + sizes[p])] = c.reshape(-1)
        self.a = torch.cat([x.reshape(-1) for x in As]).to(torch.float64).contiguous()
        self.b = torch.cat([x.reshape(-1) for x in Bs]).to(torch.float64).contiguous()
        nbytes = srot_workspace_size_batched(self.m, self.n, self.opt)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.h = srot_init_batched(self.m, self.n, self.c_off, self.C, self.a, self.b, self.workspace,
                                   self.opt, tune=1 if tune else 0)

    def solve(self):
        """(status, out3 (count x 3: g, f, D), passes, per-problem status)."""
        return srot_solve_batched(self.h, self.count)

    def plan(self, p):
        dev = self.workspace.device
        T = torch.empty(int(self.m[p]), int(self.n[p]), dtype=torch.float64, device=dev)
        r = torch.empty(int(self.n[p]), dtype=torch.float64, device=dev)
        srot_get_plan_batched(self.h, p, T, r)
        return T, r

    def tiles(self):
        return srot_get_tiles_batched(self.h, self.count)

    def close(self):
        if self.h:
            srot_destroy_batched(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Owns the device workspace of one handle and keeps its inputs alive.

    C: (m, n) float32/float64 CUDA tensor, or None with X, Y (float32, N x 3)
    for the fused squared-Euclidean cost.  a, b: float64 CUDA tensors."""

    def __init__(self, a, b, C=None, X=None, Y=None, **options):
        m, n = a.shape[0], b.shape[0]
        if "cost" not in options:
            if C is None:
                options["cost"] = SROT_COST_SQEUCLID
            else:
                options["cost"] = SROT_COST_F64 if C.dtype == torch.float64 else SROT_COST_F32
        self.opt = srot_default_options(**options)
        self.m, self.n = m, n
        self._keep = (a, b, C, X, Y)
        nbytes = srot_workspace_size(m, n, self.opt)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=a.device)
        self.h = srot_init(m, n, C, X, Y, a, b, self.workspace, self.opt)

    def step(self, nsteps, idx=None, trace=False):
        if trace:
            tj = torch.empty(nsteps, dtype=torch.int32, device=self.workspace.device)
            tg = torch.empty(nsteps, dtype=torch.float64, device=self.workspace.device)
            srot_step(self.h, nsteps, idx, tj, tg)
            return tj, tg
        srot_step(self.h, nsteps, idx)
        return None

    def gap(self, per_row=False):
        if per_row:
            rg = torch.empty(self.m, dtype=torch.float64, device=self.workspace.device)
            rj = torch.empty(self.m, dtype=torch.int32, device=self.workspace.device)
            g, f, D = srot_gap(self.h, rg, rj)
            return (g, f, D), rg, rj
        return srot_gap(self.h)

    def solve(self):
        return srot_solve(self.h)

    def plan(self):
        T = torch.empty(self.m, self.n, dtype=torch.float64, device=self.workspace.device)
        r = torch.empty(self.n, dtype=torch.float64, device=self.workspace.device)
        srot_get_plan(self.h, T, r)
        return T, r

    def plan_csr(self):
        """The plan's support as (row_ptr, col, val) CUDA tensors."""
        dev = self.workspace.device
        row_ptr = torch.empty(self.m + 1, dtype=torch.int32, device=dev)
        nnz = srot_get_plan_csr(self.h, row_ptr)
        col = torch.empty(nnz, dtype=torch.int32, device=dev)
        val = torch.empty(nnz, dtype=torch.float64, device=dev)
        if nnz:
            srot_get_plan_csr(self.h, row_ptr, col, val)
        return row_ptr, col, val

    @property
    def k(self):
        return srot_get_state(self.h)

    def set_state(self, T, k, r=None):
        srot_set_state(self.h, T, k, r)

    def backward(self, grad_out=1.0, dC=False, dX=False, dY=False, da=False, db=False):
        """Gradients of the optimal value at the current plan (srot_backward),
        as a dict of the requested tensors."""
        dev = self.workspace.device
        m, n = self.m, self.n
        out = {}
        if dC:
            cdt = torch.float64 if self.opt.cost == SROT_COST_F64 else torch.float32
            out["dC"] = torch.empty(m, n, dtype=cdt, device=dev)
        if dX:
            out["dX"] = torch.empty(m, 3, dtype=torch.float32, device=dev)
        if dY:
            out["dY"] = torch.empty(n, 3, dtype=torch.float32, device=dev)
        if da:
            out["da"] = torch.empty(m, dtype=torch.float64, device=dev)
        if db:
            out["db"] = torch.empty(n, dtype=torch.float64, device=dev)
        srot_backward(self.h, grad_out, out.get("dC"), out.get("dX"), out.get("dY"),
                      out.get("da"), out.get("db"))
        return out

    def close(self):
        if self.h:
            srot_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
