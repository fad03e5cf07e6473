"""Independent checkers used to pin the oracle (no oracle code is used here).

* kkt_bruteforce: exact optimum of the quadratic semi-relaxed problem on tiny
  inputs by enumerating row supports and solving the KKT linear system.
* ot_lp / one_sided_lp: the Kantorovich LP (eq. FormulationOptimalTransport,
  Sec. 2.1) and the one-sided LP of Sec. 2.2 via scipy's HiGHS.
* objective_np: numpy evaluation of f(T) = <T,C> + (w/2)||T^T 1 - b||^2,
  an evaluation path separate from the oracle's C loops.
"""
import itertools

import numpy as np
from scipy.optimize import linprog


def objective_np(C, a, b, w, T):
    r = T.sum(axis=0) - b
    return float(np.sum(T * C) + 0.5 * w * np.dot(r, r))


def kkt_bruteforce(C, a, b, w, tol=1e-10):
    """Optimal value f* and one optimal plan by support enumeration.

    For supports P_i (non-empty subsets of columns) solve
        c_ij + w r_j - mu_i = 0   (j in P_i),   sum_{j in P_i} t_ij = a_i,
    with r = T^T 1 - b, and keep solutions with t >= 0 and
    c_ij + w r_j - mu_i >= 0 off the support.  For a convex problem every
    such KKT point is optimal."""
    m, n = C.shape
    subsets = [s for k in range(1, n + 1) for s in itertools.combinations(range(n), k)]
    best = None
    for sup in itertools.product(subsets, repeat=m):
        var = [(i, j) for i in range(m) for j in sup[i]]
        nv = len(var)
        A = np.zeros((nv + m, nv + m))
        rhs = np.zeros(nv + m)
        for e, (i, j) in enumerate(var):
            # c_ij + w (sum_k t_kj - b_j) - mu_i = 0
            for e2, (i2, j2) in enumerate(var):
                if j2 == j:
                    A[e, e2] += w
            A[e, nv + i] = -1.0
            rhs[e] = -C[i, j] + w * b[j]
        for i in range(m):
            for e, (i2, _) in enumerate(var):
                if i2 == i:
                    A[nv + i, e] = 1.0
            rhs[nv + i] = a[i]
        sol, *_ = np.linalg.lstsq(A, rhs, rcond=None)
        if np.max(np.abs(A @ sol - rhs)) > 1e-9:
            continue
        T = np.zeros((m, n))
        for e, (i, j) in enumerate(var):
            T[i, j] = sol[e]
        if T.min() < -tol:
            continue
        mu = sol[nv:]
        r = T.sum(axis=0) - b
        red = C + w * r[None, :] - mu[:, None]
        if red.min() < -1e-9:
            continue
        T = np.maximum(T, 0.0)
        fv = objective_np(C, a, b, w, T)
        if best is None or fv < best[0]:
            best = (fv, T)
    return best


def ot_lp(C, a, b):
    m, n = C.shape
    A_eq = []
    for i in range(m):
        row = np.zeros((m, n)); row[i, :] = 1.0; A_eq.append(row.ravel())
    for j in range(n):
        col = np.zeros((m, n)); col[:, j] = 1.0; A_eq.append(col.ravel())
    res = linprog(C.ravel(), A_eq=np.array(A_eq), b_eq=np.concatenate([a, b]),
                  bounds=(0, None), method="highs")
    assert res.status == 0
    return float(res.fun)


def one_sided_lp(C, a):
    m, n = C.shape
    A_eq = []
    for i in range(m):
        row = np.zeros((m, n)); row[i, :] = 1.0; A_eq.append(row.ravel())
    res = linprog(C.ravel(), A_eq=np.array(A_eq), b_eq=a, bounds=(0, None), method="highs")
    assert res.status == 0
    return float(res.fun)
