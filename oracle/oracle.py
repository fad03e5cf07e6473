"""ctypes front end of the FP64 CPU oracle (srot_oracle.c).

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
CPU-baseline leg; the GPU library never imports it.

Orientation (same as the C file): T is m x n with exact row sums a, blocks are
rows, r = T^T 1 - b, w is the penalty weight (the paper's 1/lambda).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsrot_oracle.so")
_lib = None

ELS = 0
DEC = 1

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


class _Problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("C", _dp), ("X", _fp), ("Y", _fp),
                ("a", _dp), ("b", _dp), ("w", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build_oracle
        build_oracle.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(_Problem)
    lib.or_cost.argtypes = [P, ctypes.c_int64, ctypes.c_int64]
    lib.or_cost.restype = ctypes.c_double
    lib.or_cost_matrix.argtypes = [P, _dp]
    lib.or_residual.argtypes = [P, _dp, _dp]
    lib.or_objective.argtypes = [P, _dp, _dp]
    lib.or_objective.restype = ctypes.c_double
    lib.or_block_gradient.argtypes = [P, _dp, ctypes.c_int64, _dp]
    lib.or_lmo.argtypes = [ctypes.c_int64, _dp, _dp]
    lib.or_lmo.restype = ctypes.c_int64
    lib.or_step_dec.argtypes = [ctypes.c_int64, ctypes.c_int64]
    lib.or_step_dec.restype = ctypes.c_double
    lib.or_step_els.argtypes = [P, _dp, _dp, ctypes.c_int64, _dp]
    lib.or_step_els.restype = ctypes.c_double
    lib.or_gap.argtypes = [P, _dp, _dp, _i64p, _dp, _dp]
    lib.or_init_plan.argtypes = [P, _dp]
    lib.or_bcfw_steps.argtypes = [P, _dp, _dp, _i64p, ctypes.c_int, ctypes.c_int64,
                                  _i32p, _i32p, _dp, _dp, _i32p, _i32p, ctypes.c_double]
    lib.or_bcfw_steps.restype = ctypes.c_int
    lib.or_active_steps.argtypes = [P, _dp, _dp, _i64p, ctypes.c_int, ctypes.c_int64, _i32p, _i32p, _i32p,
                                    _dp, _dp, _i32p, _dp, _i32p, _dp, ctypes.c_double]
    lib.or_active_steps.restype = ctypes.c_int
    lib.or_fw_iteration.argtypes = [P, _dp, ctypes.c_int64, ctypes.c_int, _dp]
    lib.or_fw_iteration.restype = ctypes.c_double
    lib.or_row_gap.argtypes = [P, _dp, _dp, ctypes.c_int64]
    lib.or_row_gap.restype = ctypes.c_double
    lib.or_ga_draw.argtypes = [ctypes.c_int64, _dp, ctypes.c_double, _dp]
    lib.or_ga_draw.restype = ctypes.c_int64
    lib.or_ga_steps.argtypes = [P, _dp, _dp, _i64p, ctypes.c_int, ctypes.c_int64, _dp, _dp, _i32p, _dp,
                                _i32p, _dp, _dp, _i32p, _dp, ctypes.c_double]
    lib.or_ga_refresh.argtypes = [P, _dp, _dp]
    _lib = lib
    return lib


def _ptr(arr, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype)) if arr is not None else None


class Problem:
    """Holds the (double) cost or the (float) points, the weights and w.

    C, when given, is widened to float64 exactly; X, Y (float32, N x 3) give
    the squared Euclidean cost evaluated in double."""

    def __init__(self, a, b, w, C=None, X=None, Y=None):
        self.a = np.ascontiguousarray(a, dtype=np.float64)
        self.b = np.ascontiguousarray(b, dtype=np.float64)
        self.m, self.n = self.a.shape[0], self.b.shape[0]
        self.w = float(w)
        self.C = None if C is None else np.ascontiguousarray(C, dtype=np.float64)
        self.X = None if X is None else np.ascontiguousarray(X, dtype=np.float32)
        self.Y = None if Y is None else np.ascontiguousarray(Y, dtype=np.float32)
        if self.C is None and (self.X is None or self.Y is None):
            raise ValueError("need C or both X and Y")
        if self.C is not None and self.C.shape != (self.m, self.n):
            raise ValueError("C must be m x n")
        if self.C is None and (self.X.shape != (self.m, 3) or self.Y.shape != (self.n, 3)):
            raise ValueError("X must be m x 3 and Y n x 3")
        self._s = _Problem(self.m, self.n, _ptr(self.C, ctypes.c_double),
                           _ptr(self.X, ctypes.c_float), _ptr(self.Y, ctypes.c_float),
                           _ptr(self.a, ctypes.c_double), _ptr(self.b, ctypes.c_double),
                           self.w)

    @property
    def ref(self):
        return ctypes.byref(self._s)


def cost_matrix(P):
    out = np.empty((P.m, P.n), dtype=np.float64)
    _load().or_cost_matrix(P.ref, _ptr(out, ctypes.c_double))
    return out


def residual(P, T):
    T = np.ascontiguousarray(T, dtype=np.float64)
    r = np.empty(P.n, dtype=np.float64)
    _load().or_residual(P.ref, _ptr(T, ctypes.c_double), _ptr(r, ctypes.c_double))
    return r


def objective(P, T):
    T = np.ascontiguousarray(T, dtype=np.float64)
    return _load().or_objective(P.ref, _ptr(T, ctypes.c_double), None)


def block_gradient(P, r, i):
    r = np.ascontiguousarray(r, dtype=np.float64)
    g = np.empty(P.n, dtype=np.float64)
    _load().or_block_gradient(P.ref, _ptr(r, ctypes.c_double), int(i), _ptr(g, ctypes.c_double))
    return g


def lmo(grad):
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    margin = ctypes.c_double()
    j = _load().or_lmo(grad.shape[0], _ptr(grad, ctypes.c_double), ctypes.byref(margin))
    return int(j), margin.value


def step_dec(k, m):
    return _load().or_step_dec(int(k), int(m))


def step_els(P, t_i, s_i, i, r):
    t_i = np.ascontiguousarray(t_i, dtype=np.float64)
    s_i = np.ascontiguousarray(s_i, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    return _load().or_step_els(P.ref, _ptr(t_i, ctypes.c_double), _ptr(s_i, ctypes.c_double),
                               int(i), _ptr(r, ctypes.c_double))


def gap(P, T):
    """Returns dict(g, f, D, G (m), jstar (m), grow (m))."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    G = np.empty(P.m, dtype=np.float64)
    js = np.empty(P.m, dtype=np.int64)
    gr = np.empty(P.m, dtype=np.float64)
    out = np.empty(3, dtype=np.float64)
    _load().or_gap(P.ref, _ptr(T, ctypes.c_double), _ptr(G, ctypes.c_double),
                   _ptr(js, ctypes.c_int64), _ptr(gr, ctypes.c_double), _ptr(out, ctypes.c_double))
    return dict(g=float(out[0]), f=float(out[1]), D=float(out[2]), G=G, jstar=js, grow=gr)


def init_plan(P):
    T = np.empty((P.m, P.n), dtype=np.float64)
    _load().or_init_plan(P.ref, _ptr(T, ctypes.c_double))
    return T


class State:
    """Plan T, incremental residual r and the global block-step counter k."""

    def __init__(self, P, T=None):
        self.T = init_plan(P) if T is None else np.ascontiguousarray(T, dtype=np.float64).copy()
        self.r = residual(P, self.T)
        self.k = 0


class Trace(tuple):
    """(jstar, gamma, margin) per step, plus .runner (the runner-up vertex)
    and .near (steps x 4: columns within near_tol of the minimum, -1 padded)."""


def bcfw_steps(P, state, idx, rule=ELS, trace=True, near_tol=1e-12):
    """Runs len(idx) BCFW block steps (Alg. 1) in place on state.

    Returns (jstar, gamma, margin) traces (numpy arrays) when trace is set; the
    returned tuple also carries .runner and .near (see Trace)."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    ns = idx.shape[0]
    tj = np.empty(ns, dtype=np.int32) if trace else None
    tg = np.empty(ns, dtype=np.float64) if trace else None
    tm = np.empty(ns, dtype=np.float64) if trace else None
    tr = np.empty(ns, dtype=np.int32) if trace else None
    tn = np.empty((ns, 4), dtype=np.int32) if trace else None
    k = ctypes.c_int64(state.k)
    rc = _load().or_bcfw_steps(P.ref, _ptr(state.T, ctypes.c_double), _ptr(state.r, ctypes.c_double),
                               ctypes.byref(k), int(rule), ns, _ptr(idx, ctypes.c_int32),
                               _ptr(tj, ctypes.c_int32), _ptr(tg, ctypes.c_double),
                               _ptr(tm, ctypes.c_double), _ptr(tr, ctypes.c_int32),
                               _ptr(tn, ctypes.c_int32), float(near_tol))
    if rc != 0:
        raise ValueError("block index out of range")
    state.k = k.value
    if not trace:
        return None
    out = Trace((tj, tg, tm))
    out.runner = tr
    out.near = tn
    return out


AWAY = 0
PAIRWISE = 1


def active_steps(P, state, idx, variant, trace=True, near_tol=1e-12):
    """Runs len(idx) block steps with away steps (variant AWAY, Alg. A.2) or
    pairwise steps (PAIRWISE, Alg. A.3) in place on state.

    Returns dict(j, away, gamma, margin, near, amargin, anear, dslope) when
    trace is set; dslope is the FW slope minus the away slope of the BCAFW
    direction choice (NaN where no choice is made)."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    ns = idx.shape[0]
    out = None
    if trace:
        out = dict(j=np.empty(ns, np.int32), away=np.empty(ns, np.int32), gamma=np.empty(ns),
                   margin=np.empty(ns), near=np.empty((ns, 4), np.int32), amargin=np.empty(ns),
                   anear=np.empty((ns, 4), np.int32), dslope=np.empty(ns))
    g = (lambda key, ct: _ptr(out[key], ct)) if trace else (lambda key, ct: None)
    k = ctypes.c_int64(state.k)
    rc = _load().or_active_steps(P.ref, _ptr(state.T, ctypes.c_double), _ptr(state.r, ctypes.c_double),
                                 ctypes.byref(k), int(variant), ns, _ptr(idx, ctypes.c_int32),
                                 g("j", ctypes.c_int32), g("away", ctypes.c_int32), g("gamma", ctypes.c_double),
                                 g("margin", ctypes.c_double), g("near", ctypes.c_int32),
                                 g("amargin", ctypes.c_double), g("anear", ctypes.c_int32),
                                 g("dslope", ctypes.c_double), float(near_tol))
    if rc != 0:
        raise ValueError("block index out of range")
    state.k = k.value
    return out


def solve(P, index_source, rule=ELS, eps=0.0, max_passes=1, gap_every=1, state=None,
          trace=False, on_pass=None):
    """Passes of m block steps; the gap is measured every gap_every passes and
    the run stops at the first measured gap <= eps (Sec. 3.1 stopping rule).

    index_source(p) returns the m block indices of pass p.
    Returns (state, history) with history a list of dicts (pass, g, f, D)."""
    st = State(P) if state is None else state
    hist = []
    traces = []
    for p in range(max_passes):
        tr = bcfw_steps(P, st, index_source(p), rule=rule, trace=trace)
        if trace:
            traces.append(tr)
        if (p + 1) % gap_every == 0 or p + 1 == max_passes:
            gp = gap(P, st.T)
            rec = dict(passes=p + 1, g=gp["g"], f=gp["f"], D=gp["D"])
            hist.append(rec)
            if on_pass is not None:
                on_pass(rec)
            if gp["g"] <= eps:
                break
    if trace:
        out = Trace((np.concatenate([t[0] for t in traces]),
                     np.concatenate([t[1] for t in traces]),
                     np.concatenate([t[2] for t in traces])))
        out.runner = np.concatenate([t.runner for t in traces])
        out.near = np.concatenate([t.near for t in traces])
        return st, hist, out
    return st, hist


def fw_iteration(P, T, k, rule=ELS):
    """One full FW iteration (Alg. A.1) in place on T; returns (gap_before, gamma)."""
    gam = ctypes.c_double()
    g = _load().or_fw_iteration(P.ref, _ptr(T, ctypes.c_double), int(k), int(rule), ctypes.byref(gam))
    return g, gam.value


def barycentric(T, X, Y):
    """Barycentric projection (eq. barycentric_projection, Sec. 5):
    xhat_i = sum_j t_ij y_j / sum_j t_ij in FP64; a row without mass keeps x_i."""
    T = np.asarray(T, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    out = X.copy()
    for i in range(T.shape[0]):
        den = T[i].sum()
        if den > 0.0:
            out[i] = (T[i][:, None] * Y).sum(axis=0) / den
    return out


# BCFW with gap-adaptive sampling (Alg. A.4, Sec. 4.2.1).  Every stored block
# gap starts at a large constant; 2^300 is exact under addition of up to 2^53
# copies and absorbs any real block gap below 2^246, so blocks not yet
# visited are drawn (uniformly) before any visited one.
GA_INIT = 2.0 ** 300


def row_gap(P, T, r, i):
    """Gap of block i (eq. AppenEq:Gi) at plan T with residual r."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    return _load().or_row_gap(P.ref, _ptr(T, ctypes.c_double), _ptr(r, ctypes.c_double), int(i))


def ga_draw(W, u):
    """Block drawn from the stored gaps W with uniform u (see or_ga_draw);
    returns (i, margin relative to the sum of W)."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    mg = ctypes.c_double()
    i = _load().or_ga_draw(W.shape[0], _ptr(W, ctypes.c_double), float(u), ctypes.byref(mg))
    return int(i), mg.value


def ga_weights(P, init=GA_INIT):
    return np.full(P.m, float(init), dtype=np.float64)


def ga_refresh(P, T):
    """Global update of Alg. A.4: every block's gap at T (clamped at 0)."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    W = np.empty(P.m, dtype=np.float64)
    _load().or_ga_refresh(P.ref, _ptr(T, ctypes.c_double), _ptr(W, ctypes.c_double))
    return W


def ga_steps(P, state, W, u, rule=ELS, trace=True, near_tol=1e-12):
    """len(u) iterations of Alg. A.4 in place on state and on the stored
    gaps W (float64, length m): draw, BCFW block step, store the drawn
    block's new gap.  Returns dict(i, umargin, j, gamma, margin, near, g)
    when trace is set."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert W.dtype == np.float64 and W.flags.c_contiguous and W.shape == (P.m,)
    ns = u.shape[0]
    out = None
    if trace:
        out = dict(i=np.empty(ns, np.int32), umargin=np.empty(ns), j=np.empty(ns, np.int32),
                   gamma=np.empty(ns), margin=np.empty(ns), near=np.empty((ns, 4), np.int32),
                   g=np.empty(ns))
    g = (lambda key, ct: _ptr(out[key], ct)) if trace else (lambda key, ct: None)
    k = ctypes.c_int64(state.k)
    _load().or_ga_steps(P.ref, _ptr(state.T, ctypes.c_double), _ptr(state.r, ctypes.c_double),
                        ctypes.byref(k), int(rule), ns, _ptr(u, ctypes.c_double), _ptr(W, ctypes.c_double),
                        g("i", ctypes.c_int32), g("umargin", ctypes.c_double), g("j", ctypes.c_int32),
                        g("gamma", ctypes.c_double), g("margin", ctypes.c_double), g("near", ctypes.c_int32),
                        g("g", ctypes.c_double), float(near_tol))
    state.k = k.value
    return out


def solve_ga(P, u_source, period=1, init=GA_INIT, rule=ELS, eps=0.0, max_passes=1):
    """Outer iterations of Alg. A.4: passes of m inner iterations; after each
    pass the gap is measured (stop at g <= eps, Sec. 3.1), and after every
    `period` passes all stored block gaps are recomputed (global update).
    u_source(p) returns the m uniforms of pass p.  Returns (state, W, hist)."""
    st = State(P)
    W = ga_weights(P, init)
    hist = []
    for p in range(max_passes):
        ga_steps(P, st, W, u_source(p), rule=rule, trace=False)
        gp = gap(P, st.T)
        hist.append(dict(passes=p + 1, g=gp["g"], f=gp["f"], D=gp["D"]))
        if gp["g"] <= eps:
            break
        if (p + 1) % period == 0:
            W[:] = ga_refresh(P, st.T)
    return st, W, hist
