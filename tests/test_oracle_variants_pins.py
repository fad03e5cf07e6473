"""Pins of the oracle's away-step (Alg. A.2) and pairwise (Alg. A.3) block
steps, against an independent numpy derivation and exact optima.

* Each step moves along the direction the algorithm prescribes (FW vertex
  = lowest-index gradient minimum, away vertex = largest gradient on the
  support) by the minimiser of f over [0, gamma_max], checked on a dense
  gamma grid; a step that reaches gamma_max empties the away atom exactly.
* f never increases; row sums stay a_i; T stays >= 0.
* While a row holds a single atom the variants coincide with BCFW + exact
  line search (the away direction is then zero and d_Pair = d_FW).
* Both reach the brute-force optimum (support enumeration) on tiny inputs.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2103_05857_amd import inputs as I

from pins import kkt_bruteforce, objective_np


def _state_after_bcfw(d, w, steps, seed=0):
    m = d["C"].shape[0]
    P = O.Problem(d["a"], d["b"], w, C=d["C"])
    st = O.State(P)
    O.bcfw_steps(P, st, I.philox_uniform_indices(seed, 0, steps, m), trace=False)
    return P, st


@pytest.mark.parametrize("variant", [O.AWAY, O.PAIRWISE])
@pytest.mark.parametrize("w", [0.5, 3.0])
def test_each_step_is_the_line_search_minimiser(variant, w):
    d = I.problem_mixture(11, 12, 9, cost_dtype=np.float64)
    C, a, b = d["C"], d["a"], d["b"]
    P, st = _state_after_bcfw(d, w, 60)
    # rows 0..5 get a small atom on their most expensive column: moving it
    # away pays all the way, so those steps end at gamma_max (a drop)
    for i in range(6):
        st.T[i] = 0.0
        st.T[i, int(np.argmin(C[i]))] = 0.97 * a[i]
        st.T[i, int(np.argmax(C[i]))] = 0.03 * a[i]
    st.r = O.residual(P, st.T)
    rng = np.random.default_rng(3)
    drops = 0
    order = list(range(6)) + [int(x) for x in rng.integers(0, 12, 74)]
    for i in order:
        T0 = st.T.copy()
        g = C[i] + w * (T0.sum(axis=0) - b)
        sup = np.nonzero(T0[i] > 0)[0]
        tr = O.active_steps(P, st, np.array([i], np.int32), variant)
        # the vertices must be the extreme gradient entries; the line search
        # makes a row's atoms equal in exact arithmetic, so a rounding-level
        # tie (1e-12) may be resolved either way: take the oracle's choice
        js = int(tr["j"][0])
        ja = int(tr["away"][0]) if tr["away"][0] >= 0 else -1 - int(tr["away"][0])
        assert g[js] - g.min() <= 1e-12
        assert ja in sup and g[sup].max() - g[ja] <= 1e-12
        alpha = T0[i, ja] / a[i]
        s = np.zeros(9); s[js] = a[i]
        v = np.zeros(9); v[ja] = a[i]
        if variant == O.PAIRWISE:
            dvec, gmax = s - v, alpha
        else:
            dfw, daw = s - T0[i], T0[i] - v
            if len(sup) == 1 or ja == js or -g @ dfw >= -g @ daw:
                dvec, gmax = dfw, 1.0
            else:
                dvec, gmax = daw, alpha / (1 - alpha)
        gam = tr["gamma"][0]
        assert 0.0 <= gam <= gmax + 1e-15
        T1 = T0.copy()
        T1[i] = T0[i] + gam * dvec
        if gam > 0 and gam == gmax and not (variant == O.AWAY and tr["away"][0] < 0):
            drops += 1
            assert st.T[i, ja] == 0.0
            T1[i, ja] = 0.0
        np.testing.assert_allclose(st.T, T1, rtol=1e-12, atol=1e-15)
        grid = np.linspace(0.0, gmax, 401)
        fgrid = [objective_np(C, a, b, w, np.where(np.arange(12)[:, None] == i, T0 + gg * dvec, T0)) for gg in grid]
        assert objective_np(C, a, b, w, st.T) <= min(fgrid) + 1e-14
        np.testing.assert_allclose(st.T.sum(axis=1), a, rtol=0, atol=1e-15)
        assert st.T.min() >= 0.0
    assert drops > 0


@pytest.mark.parametrize("variant", [O.AWAY, O.PAIRWISE])
def test_objective_never_increases(variant):
    d = I.problem_mixture(12, 40, 50, cost_dtype=np.float64)
    P = O.Problem(d["a"], d["b"], 1.0, C=d["C"])
    st = O.State(P)
    f_prev = O.objective(P, st.T)
    idx = I.philox_uniform_indices(1, 0, 40 * 30, 40)
    for q in range(0, len(idx), 40):
        O.active_steps(P, st, idx[q:q + 40], variant, trace=False)
        f = O.objective(P, st.T)
        assert f <= f_prev + 1e-15
        f_prev = f
    np.testing.assert_allclose(st.r, st.T.sum(axis=0) - d["b"], rtol=0, atol=1e-13)


@pytest.mark.parametrize("variant", [O.AWAY, O.PAIRWISE])
def test_single_atom_rows_match_bcfw(variant):
    d = I.problem_mixture(13, 30, 40, cost_dtype=np.float64)
    P = O.Problem(d["a"], d["b"], 1.0, C=d["C"])
    idx = np.random.default_rng(0).permutation(30).astype(np.int32)   # each row once, single atom
    s1 = O.State(P)
    t1 = O.bcfw_steps(P, s1, idx)
    s2 = O.State(P)
    t2 = O.active_steps(P, s2, idx, variant)
    np.testing.assert_array_equal(t2["j"], t1[0])
    np.testing.assert_allclose(t2["gamma"], t1[1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(s2.T, s1.T, rtol=0, atol=1e-15)


@pytest.mark.parametrize("variant", [O.AWAY, O.PAIRWISE])
@pytest.mark.parametrize("seed,m,n,w", [(1, 3, 3, 1.0), (2, 3, 2, 4.0), (5, 2, 4, 0.5)])
def test_reaches_the_bruteforce_optimum(variant, seed, m, n, w):
    rng = np.random.default_rng(seed)
    C = rng.random((m, n))
    a = rng.dirichlet(np.ones(m))
    b = rng.dirichlet(np.ones(n))
    P = O.Problem(a, b, w, C=C)
    st = O.State(P)
    O.active_steps(P, st, I.philox_uniform_indices(seed, 0, 400 * m, m), variant, trace=False)
    fstar, _ = kkt_bruteforce(C, a, b, w)
    assert O.objective(P, st.T) - fstar <= 1e-12


def test_away_direction_choice_margin_is_the_slope_difference():
    """BCAFW (Alg. A.2) takes the FW direction when its descent slope is at
    least the away direction's.  The oracle reports the margin of that choice,
    <-g, d_FW> - <-g, d_A>; here each slope is measured as a central
    difference of f along the direction (exact up to rounding, f being
    quadratic), and the direction taken must follow the sign of the margin."""
    d = I.problem_mixture(21, 10, 8, cost_dtype=np.float64)
    C, a, b, w = d["C"], d["a"], d["b"], 2.0
    P, st = _state_after_bcfw(d, w, 50)
    rng = np.random.default_rng(4)
    choices = set()
    checked = 0
    for i in rng.integers(0, 10, 120):
        i = int(i)
        T0 = st.T.copy()
        sup = np.nonzero(T0[i] > 0)[0]
        tr = O.active_steps(P, st, np.array([i], np.int32), O.AWAY)
        js = int(tr["j"][0])
        ja = int(tr["away"][0]) if tr["away"][0] >= 0 else -1 - int(tr["away"][0])
        if len(sup) == 1 or ja == js:
            assert np.isnan(tr["dslope"][0]) and tr["away"][0] < 0
            continue
        s = np.zeros(8); s[js] = a[i]
        v = np.zeros(8); v[ja] = a[i]
        h = 1e-3
        slopes = []
        for dvec in (s - T0[i], T0[i] - v):
            Tp, Tm = T0.copy(), T0.copy()
            Tp[i] += h * dvec
            Tm[i] -= h * dvec
            slopes.append(-(objective_np(C, a, b, w, Tp) - objective_np(C, a, b, w, Tm)) / (2 * h))
        assert abs(tr["dslope"][0] - (slopes[0] - slopes[1])) <= 1e-10
        took_fw = tr["away"][0] < 0
        assert took_fw == (tr["dslope"][0] >= 0.0)
        choices.add(took_fw)
        checked += 1
    assert checked >= 40 and choices == {True, False}
