"""Pins of the oracle's adjoint (oracle/adjoint.py) to things other than itself.

* kkt_polish reaches the exact optimum: it agrees with brute-force support
  enumeration (tests/pins.py) on tiny inputs, and at m = n = 64 the oracle's
  own duality-gap sweep (Thm 2) certifies it to rounding.
* The envelope-theorem derivatives agree with FP64 central finite
  differences of the optimal value (computed by re-polishing the perturbed
  problem) for dV/dX, dV/dY, dV/db, dV/da and dV/dC (every support entry
  plus 256 random zeros): relative error <= 1e-5.  On a fixed optimal
  support the optimal plan is affine in (C, a, b), so V is quadratic there
  and central differences in those arguments carry no truncation error.
"""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import oracle as O
from paper_2103_05857_amd import inputs as I

from pins import kkt_bruteforce


def _bcfw_plan(C, a, b, w, passes, seed=0):
    m = C.shape[0]
    P = O.Problem(a, b, w, C=C)
    st, _ = O.solve(P, lambda p: I.philox_uniform_indices(seed, p * m, m, m),
                    max_passes=passes, gap_every=passes)
    return st.T


@pytest.mark.parametrize("seed,m,n,w", [(1, 2, 3, 1.0), (2, 3, 3, 0.5), (3, 3, 2, 4.0),
                                         (4, 3, 3, 20.0)])
def test_polish_matches_bruteforce(seed, m, n, w):
    rng = np.random.default_rng(seed)
    C = rng.random((m, n))
    a = rng.dirichlet(np.ones(m))
    b = rng.dirichlet(np.ones(n))
    T0 = _bcfw_plan(C, a, b, w, 200, seed)
    T, mu, info = A.kkt_polish(C, a, b, w, T0)
    fstar, Tb = kkt_bruteforce(C, a, b, w)
    assert abs(A.objective(C, b, w, T) - fstar) <= 1e-13
    np.testing.assert_allclose(T, Tb, atol=1e-12)
    assert T.min() >= 0.0
    np.testing.assert_allclose(T.sum(axis=1), a, rtol=0, atol=1e-14)


@pytest.fixture(scope="module")
def polished64():
    d = I.problem_mixture(0, 64, 64, cost_dtype=np.float64, with_cost=False)
    X = d["X"].astype(np.float64)
    Y = d["Y"].astype(np.float64)
    C = A.sqeuclid_cost(X, Y)
    a, b, w = d["a"], d["b"], 1.0
    T0 = _bcfw_plan(C, a, b, w, 1500)
    T, mu, info = A.kkt_polish(C, a, b, w, T0)
    return dict(X=X, Y=Y, C=C, a=a, b=b, w=w, T=T, mu=mu, T0=T0)


def test_polish_is_optimal_by_the_gap_certificate(polished64):
    p = polished64
    P = O.Problem(p["a"], p["b"], p["w"], C=p["C"])
    gp = O.gap(P, p["T"])
    g0 = O.gap(P, p["T0"])
    assert gp["g"] <= 1e-14 and gp["g"] >= -1e-15
    assert gp["f"] <= g0["f"]
    np.testing.assert_allclose(p["T"].sum(axis=1), p["a"], rtol=0, atol=1e-15)
    assert p["T"].min() >= 0.0
    # multipliers: the row minima of the gradient at the optimum
    np.testing.assert_allclose(p["mu"], gp["G"], rtol=0, atol=1e-14)


def _value(C, a, b, w, T_guess):
    T, _, _ = A.kkt_polish(C, a, b, w, T_guess)
    return A.objective(C, b, w, T)


def _rel_err(fd, an):
    return float(np.max(np.abs(fd - an)) / max(np.max(np.abs(fd)), 1e-300))


def test_adjoint_matches_finite_differences(polished64):
    p = polished64
    X, Y, C, a, b, w, T = p["X"], p["Y"], p["C"], p["a"], p["b"], p["w"], p["T"]
    adj = A.adjoint(C, a, b, w, T, X=X, Y=Y, grad_out=1.0)
    h = 1e-6

    fdX = np.zeros_like(X)
    for i in range(X.shape[0]):
        for d in range(3):
            Xp = X.copy(); Xp[i, d] += h
            Xm = X.copy(); Xm[i, d] -= h
            fdX[i, d] = (_value(A.sqeuclid_cost(Xp, Y), a, b, w, T)
                         - _value(A.sqeuclid_cost(Xm, Y), a, b, w, T)) / (2 * h)
    assert _rel_err(fdX, adj["dX"]) <= 1e-5

    fdY = np.zeros_like(Y)
    for j in range(Y.shape[0]):
        for d in range(3):
            Yp = Y.copy(); Yp[j, d] += h
            Ym = Y.copy(); Ym[j, d] -= h
            fdY[j, d] = (_value(A.sqeuclid_cost(X, Yp), a, b, w, T)
                         - _value(A.sqeuclid_cost(X, Ym), a, b, w, T)) / (2 * h)
    assert _rel_err(fdY, adj["dY"]) <= 1e-5

    fdb = np.zeros_like(b)
    for j in range(b.shape[0]):
        bp = b.copy(); bp[j] += h
        bm = b.copy(); bm[j] -= h
        fdb[j] = (_value(C, a, bp, w, T) - _value(C, a, bm, w, T)) / (2 * h)
    assert _rel_err(fdb, adj["db"]) <= 1e-5

    fda = np.zeros_like(a)
    for i in range(a.shape[0]):
        ap = a.copy(); ap[i] += h
        am = a.copy(); am[i] -= h
        fda[i] = (_value(C, ap, b, w, T) - _value(C, am, b, w, T)) / (2 * h)
    assert _rel_err(fda, adj["da"]) <= 1e-5

    rng = np.random.default_rng(5)
    sup = list(zip(*np.nonzero(T > 0)))
    zeros = list(zip(*np.nonzero(T == 0)))
    pick = [zeros[k] for k in rng.choice(len(zeros), 256, replace=False)]
    cells = sup + pick
    fdC = np.zeros(len(cells))
    for k, (i, j) in enumerate(cells):
        Cp = C.copy(); Cp[i, j] += h
        Cm = C.copy(); Cm[i, j] -= h
        fdC[k] = (_value(Cp, a, b, w, T) - _value(Cm, a, b, w, T)) / (2 * h)
    an = np.array([adj["dC"][i, j] for i, j in cells])
    assert _rel_err(fdC, an) <= 1e-5
    # the zeros of the plan have exactly zero derivative
    assert np.all(fdC[len(sup):] == 0.0)


def test_adjoint_scales_with_grad_out(polished64):
    p = polished64
    a1 = A.adjoint(p["C"], p["a"], p["b"], p["w"], p["T"], X=p["X"], Y=p["Y"], grad_out=1.0)
    a3 = A.adjoint(p["C"], p["a"], p["b"], p["w"], p["T"], X=p["X"], Y=p["Y"], grad_out=-2.5)
    for k in a1:
        np.testing.assert_allclose(a3[k], -2.5 * a1[k], rtol=1e-15, atol=0)
