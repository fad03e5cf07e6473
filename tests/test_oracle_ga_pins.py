"""Pins of the oracle's BCFW with gap-adaptive sampling (Alg. A.4, Sec. 4.2.1)
against independent numpy derivations, hand examples and exact optima.

* The draw is inversion of the distribution W / sum W: on a fine grid of u
  every block gets its share of the grid to one grid cell; zero weights are
  never drawn; hand examples fix the interval ends; all-zero weights give
  floor(u m).
* The block gap (eq. AppenEq:Gi) equals <t_i, grad_i f> - a_i min grad_i f
  computed in numpy from T alone; the gaps sum to the linearization gap
  (Thm 2), and the global update stores exactly those values.
* After each inner iteration the drawn block's stored gap is its gap at the
  new plan (numpy), every other stored value is unchanged, and the step is
  the BCFW step of Alg. 1 on the drawn block.
* With the large initial constant the first m draws visit every block once.
* The outer iterations reach the brute-force optimum on tiny inputs.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2103_05857_amd import inputs as I

from pins import kkt_bruteforce, objective_np


def _np_row_gaps(C, b, w, T):
    g = C + w * (T.sum(axis=0) - b)[None, :]
    return np.sum(T * g, axis=1) - T.sum(axis=1) * g.min(axis=1)


def test_draw_hand_examples():
    W = np.array([1.0, 0.0, 3.0])
    assert O.ga_draw(W, 0.0)[0] == 0
    assert O.ga_draw(W, 0.2)[0] == 0          # x = 0.8 in [0, 1)
    assert O.ga_draw(W, 0.25)[0] == 2         # x = 1.0: block 1 has an empty interval
    assert O.ga_draw(W, 0.999)[0] == 2
    i, mg = O.ga_draw(W, 0.5)                 # x = 2.0 in [1, 4): 1 from the lower end
    assert i == 2 and mg == pytest.approx(1.0 / 4.0)
    Z = np.zeros(5)
    assert [O.ga_draw(Z, u)[0] for u in (0.0, 0.19, 0.2, 0.99)] == [0, 0, 1, 4]
    # u just below 1 cannot run past the last positive weight
    assert O.ga_draw(np.array([0.5, 0.25, 0.0]), np.nextafter(1.0, 0.0))[0] == 1


@pytest.mark.parametrize("seed", [0, 1])
def test_draw_is_inversion_of_the_weights(seed):
    rng = np.random.default_rng(seed)
    W = rng.random(37)
    W[rng.integers(0, 37, 8)] = 0.0
    N = 200000
    u = (np.arange(N) + 0.5) / N
    cnt = np.bincount([O.ga_draw(W, x)[0] for x in u], minlength=37)
    assert np.all(cnt[W == 0.0] == 0)
    np.testing.assert_allclose(cnt / N, W / W.sum(), rtol=0, atol=1.0 / N + 1e-12)


@pytest.mark.parametrize("w", [0.5, 4.0])
def test_block_gaps_sum_to_the_linearization_gap(w):
    d = I.problem_mixture(21, 15, 11, cost_dtype=np.float64)
    C, a, b = d["C"], d["a"], d["b"]
    P = O.Problem(a, b, w, C=C)
    st = O.State(P)
    O.bcfw_steps(P, st, I.philox_uniform_indices(2, 0, 40, 15), trace=False)
    ref = _np_row_gaps(C, b, w, st.T)
    r = st.T.sum(axis=0) - b
    got = np.array([O.row_gap(P, st.T, r, i) for i in range(15)])
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-16)
    assert np.all(ref >= -1e-16)
    W = O.ga_refresh(P, st.T)
    np.testing.assert_allclose(W, np.maximum(ref, 0.0), rtol=1e-12, atol=1e-16)
    assert W.sum() == pytest.approx(O.gap(P, st.T)["g"], rel=1e-12)


@pytest.mark.parametrize("rule", [O.ELS, O.DEC])
def test_inner_iteration_updates_only_the_drawn_block(rule):
    m, n, w = 12, 9, 1.5
    d = I.problem_mixture(22, m, n, cost_dtype=np.float64)
    C, a, b = d["C"], d["a"], d["b"]
    P = O.Problem(a, b, w, C=C)
    st = O.State(P)
    W = O.ga_weights(P)
    u = I.philox_uniform_doubles(4, 0, 6 * m)
    for s in range(len(u)):
        T0, r0, W0, k0 = st.T.copy(), st.r.copy(), W.copy(), st.k
        tr = O.ga_steps(P, st, W, u[s:s + 1], rule=rule)
        i = int(tr["i"][0])
        assert i == O.ga_draw(W0, u[s])[0]
        # the block step is the one of Alg. 1 on block i
        ref = O.State(P, T0)
        ref.r, ref.k = r0, k0
        bt = O.bcfw_steps(P, ref, np.array([i], np.int32), rule=rule)
        assert bt[0][0] == tr["j"][0] and bt[1][0] == tr["gamma"][0]
        np.testing.assert_array_equal(ref.T, st.T)
        # only the drawn block's stored gap changes, to its gap at the new plan
        g_new = _np_row_gaps(C, b, w, st.T)[i]
        assert W[i] == pytest.approx(max(g_new, 0.0), rel=1e-10, abs=1e-16)
        assert tr["g"][0] == W[i]
        keep = np.arange(m) != i
        np.testing.assert_array_equal(W[keep], W0[keep])
        np.testing.assert_allclose(st.T.sum(axis=1), a, rtol=0, atol=1e-15)


def test_large_initial_constant_visits_every_block_first():
    m, n = 40, 25
    d = I.problem_mixture(23, m, n, cost_dtype=np.float64)
    P = O.Problem(d["a"], d["b"], 1.0, C=d["C"])
    st = O.State(P)
    W = O.ga_weights(P)
    tr = O.ga_steps(P, st, W, I.philox_uniform_doubles(9, 0, m))
    assert sorted(tr["i"].tolist()) == list(range(m))
    assert np.all(W < 1.0)                     # every stored value is now a real gap


def test_zero_gap_blocks_are_not_drawn():
    m, n = 30, 20
    d = I.problem_mixture(24, m, n, cost_dtype=np.float64)
    P = O.Problem(d["a"], d["b"], 1.0, C=d["C"])
    st = O.State(P)
    O.bcfw_steps(P, st, I.philox_uniform_indices(3, 0, 20 * m, m), trace=False)
    W = O.ga_refresh(P, st.T)
    W[::3] = 0.0                               # pretend these blocks are optimal
    zero = set(range(0, m, 3))
    drawn = [O.ga_draw(W, x)[0] for x in I.philox_uniform_doubles(5, 0, 5000)]
    assert not zero.intersection(drawn)


@pytest.mark.parametrize("period", [1, 3])
@pytest.mark.parametrize("seed,m,n,w", [(1, 3, 3, 1.0), (2, 3, 2, 4.0), (5, 2, 4, 0.5)])
def test_reaches_the_bruteforce_optimum(period, seed, m, n, w):
    rng = np.random.default_rng(seed)
    C = rng.random((m, n))
    a = rng.dirichlet(np.ones(m))
    b = rng.dirichlet(np.ones(n))
    P = O.Problem(a, b, w, C=C)
    st, W, hist = O.solve_ga(P, lambda p: I.philox_uniform_doubles(seed, p * m, m), period=period,
                             max_passes=600)
    fstar, _ = kkt_bruteforce(C, a, b, w)
    assert objective_np(C, a, b, w, st.T) - fstar <= 1e-12
    assert hist[-1]["g"] <= 1e-9
