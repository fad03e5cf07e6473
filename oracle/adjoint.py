"""FP64 adjoint of the semi-relaxed OT value, and an exact-optimum polish.

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: used by the tests and
never by the GPU library.  Plain numpy, written to be read against the
formulas below; it shares nothing with the HIP path.

Orientation as in srot_oracle.c: T is m x n, T 1 = a exactly, r = T^T 1 - b,
w is the penalty weight (the paper's 1/lambda), and the value is

    V(C, a, b) = min { <T, C> + (w/2) ||T^T 1 - b||^2 : T >= 0, T 1 = a }

(the problem of Sec. 3).  The paper does not differentiate V.  Its
Lagrangian (App. D) has one multiplier mu_i per row-sum constraint; at an
optimal plan T* with residual r* the KKT conditions read

    c_ij + w r*_j - mu_i = 0  where t*_ij > 0,
    c_ij + w r*_j - mu_i >= 0 elsewhere,

so mu_i = min_j (c_ij + w r*_j), the row minimum of the block gradient
(eq. RelaxedGradient).  By the envelope theorem the derivatives of V are
the partial derivatives of the Lagrangian at (T*, mu):

    dV/dC_ij = t*_ij,    dV/db_j = -w r*_j,    dV/da_i = mu_i,

and with the squared Euclidean cost c_ij = ||x_i - y_j||^2

    dV/dx_i = 2 sum_j t*_ij (x_i - y_j),   dV/dy_j = 2 sum_i t*_ij (y_j - x_i).

`adjoint` evaluates these formulas at whatever plan it is given; they are
the gradient of V only at an optimum.  `kkt_polish` turns a feasible BCFW
iterate into an exact optimum with a primal active-set method: the KKT
equations above, restricted to a working support, are one linear system;
entries that would turn negative leave the support and columns with
negative reduced cost join it.  The result satisfies the KKT conditions to
FP64 rounding, which the oracle's duality-gap sweep (Thm 2) certifies.
"""
import numpy as np


def sqeuclid_cost(X, Y):
    """c_ij = ||x_i - y_j||^2 in double (points widened exactly)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    m, n = X.shape[0], Y.shape[0]
    C = np.zeros((m, n))
    for d in range(3):
        diff = X[:, d][:, None] - Y[:, d][None, :]
        C += diff * diff
    return C


def objective(C, b, w, T):
    r = T.sum(axis=0) - b
    return float(np.sum(T * C) + 0.5 * w * np.dot(r, r))


def adjoint(C, a, b, w, T, X=None, Y=None, grad_out=1.0):
    """Envelope-theorem derivatives of V at the plan T, scaled by grad_out.

    Returns dict(dC, da, db, dX, dY); dX and dY only when X and Y are given
    (the cost is then taken to be their squared Euclidean distance)."""
    T = np.asarray(T, dtype=np.float64)
    m, n = T.shape
    g = float(grad_out)
    r = T.sum(axis=0) - b
    grad_rows = np.asarray(C, dtype=np.float64) + w * r[None, :]
    mu = grad_rows.min(axis=1)
    out = dict(dC=g * T, da=g * mu, db=-g * w * r)
    if X is not None and Y is not None:
        X = np.asarray(X, dtype=np.float64)
        Y = np.asarray(Y, dtype=np.float64)
        dX = np.zeros((m, 3))
        dY = np.zeros((n, 3))
        for d in range(3):
            diff = X[:, d][:, None] - Y[:, d][None, :]      # x_i - y_j
            dX[:, d] = 2.0 * g * np.sum(T * diff, axis=1)
            dY[:, d] = 2.0 * g * np.sum(T * (-diff), axis=0)
        out["dX"] = dX
        out["dY"] = dY
    return out


def _kkt_system(C, a, b, w, S):
    """The KKT equations of the problem restricted to the support S.

    Unknowns: t_ij for (i, j) in S (row-major order) and mu_i for the rows
    with a nonempty support.
      (i, j) in S:  c_ij + w (sum_k t_kj - b_j) - mu_i = 0
      row i:        sum_{j in S_i} t_ij = a_i
    Returns (K, rhs, var, rows)."""
    m, n = C.shape
    var = [(i, j) for i in range(m) for j in range(n) if S[i, j]]
    rows = [i for i in range(m) if S[i].any()]
    rpos = {i: k for k, i in enumerate(rows)}
    nv, nr = len(var), len(rows)
    K = np.zeros((nv + nr, nv + nr))
    rhs = np.zeros(nv + nr)
    by_col = {}
    for e, (i, j) in enumerate(var):
        by_col.setdefault(j, []).append(e)
    for e, (i, j) in enumerate(var):
        for e2 in by_col[j]:
            K[e, e2] += w
        K[e, nv + rpos[i]] = -1.0
        rhs[e] = w * b[j] - C[i, j]
        K[nv + rpos[i], e] = 1.0
    for i in rows:
        rhs[nv + rpos[i]] = a[i]
    return K, rhs, var, rows


def _scatter(var, values, shape):
    M = np.zeros(shape)
    for e, (i, j) in enumerate(var):
        M[i, j] = values[e]
    return M


def _ratio_step(T, D, S):
    """Largest alpha in [0, 1] keeping T + alpha D >= 0 on S; the entry that
    blocks (if any) leaves the support."""
    alpha, block = 1.0, None
    for i, j in zip(*np.nonzero(S & (D < 0.0))):
        ratio = T[i, j] / (-D[i, j])
        if ratio < alpha:
            alpha, block = ratio, (i, j)
    T = T + alpha * D
    if block is not None:
        T[block] = 0.0
        S[block] = False
    T = np.where(S, np.maximum(T, 0.0), 0.0)
    return T, block


def kkt_polish(C, a, b, w, T0, tol=1e-13, max_iter=2000):
    """Exact optimum from a feasible plan T0 (T0 >= 0, T0 1 = a): a primal
    active-set method for the convex quadratic program.

    Each iteration solves the KKT equations on the working support S.  The
    Hessian w (column-sum)^T (column-sum) is only semidefinite: when S holds
    a cycle the system is singular and the objective is linear along the
    cycle direction (row and column sums unchanged), so the method moves
    along it downhill until an entry reaches zero.  Otherwise it moves toward
    the equality-constrained minimiser, stopping at the first entry that
    reaches zero; at the minimiser it adds the column of most negative
    reduced cost, or stops when none is negative.
    Returns (T*, mu, info)."""
    C = np.asarray(C, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = C.shape
    T = np.asarray(T0, dtype=np.float64).copy()
    S = T > 0.0
    scale = max(1.0, float(np.abs(C).max()), w)
    for it in range(max_iter):
        K, rhs, var, rows = _kkt_system(C, a, b, w, S)
        nv = len(var)
        U, sv, Vt = np.linalg.svd(K)
        singular = sv[-1] <= sv[0] * 1e-12
        if singular:
            d = _scatter(var, Vt[-1][:nv], (m, n))
            r = T.sum(axis=0) - b
            slope = float(np.sum((C + w * r[None, :]) * d))
            if abs(slope) > 1e-14 * scale * np.abs(d).sum():
                if slope > 0.0:
                    d = -d
                T, block = _ratio_step(T, d * 1e6 / max(np.abs(d).max(), 1e-300), S)
                if block is None:
                    raise RuntimeError("kkt_polish: unbounded cycle direction")
                continue
            sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
        else:
            sol = Vt.T @ ((U.T @ rhs) / sv)
        Tn = _scatter(var, sol[:nv], (m, n))
        D = Tn - T
        if np.any(S & (Tn < 0.0)):
            T, _ = _ratio_step(T, D, S)
            continue
        T = np.where(S, Tn, 0.0)
        r = T.sum(axis=0) - b
        mu = (C + w * r[None, :]).min(axis=1)
        for k, i in enumerate(rows):
            mu[i] = sol[nv + k]
        red = C + w * r[None, :] - mu[:, None]
        red_off = np.where(S, np.inf, red)
        k = np.unravel_index(np.argmin(red_off), red_off.shape)
        if red_off[k] < -tol * scale:
            S[k] = True
            continue
        return T, mu, dict(iters=it + 1, min_t=float(np.where(S, T, np.inf).min()),
                           min_reduced=float(red_off.min()) if np.isfinite(red_off).any() else 0.0)
    raise RuntimeError("kkt_polish: active set did not settle")
