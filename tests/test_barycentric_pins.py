"""Pins of the oracle's barycentric projection (eq. barycentric_projection).

* At zero penalty BCFW reaches the row-wise nearest-target plan t_i = a_i e_{j(i)}
  (the closed form of Sec. 2.2): the projection of x_i is exactly y_{j(i)}.
* A plan split over two targets gives their weighted mean (hand example).
* The projection is a convex combination: it lies in the targets' bounding box.
"""
import numpy as np

from oracle import oracle as O
from paper_2103_05857_amd import inputs as I


def test_zero_penalty_projects_onto_nearest_target():
    d = I.problem_mixture(3, 30, 40, cost_dtype=np.float64)
    P = O.Problem(d["a"], d["b"], 0.0, C=d["C"])
    st = O.State(P)
    O.bcfw_steps(P, st, np.arange(30, dtype=np.int32), trace=False)
    Xh = O.barycentric(st.T, d["X"], d["Y"])
    nearest = d["C"].argmin(axis=1)
    np.testing.assert_array_equal(Xh, d["Y"][nearest].astype(np.float64))


def test_two_target_split_is_the_weighted_mean():
    T = np.array([[0.25, 0.75, 0.0], [0.0, 0.0, 0.0]])
    X = np.array([[9.0, 9.0, 9.0], [1.0, 2.0, 3.0]])
    Y = np.array([[0.0, 0.0, 4.0], [4.0, 8.0, 0.0], [7.0, 7.0, 7.0]])
    Xh = O.barycentric(T, X, Y)
    np.testing.assert_allclose(Xh[0], [3.0, 6.0, 1.0], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(Xh[1], X[1])      # no mass: unchanged


def test_projection_is_a_convex_combination():
    d = I.problem_mixture(4, 50, 60, cost_dtype=np.float64)
    P = O.Problem(d["a"], d["b"], 1.0, C=d["C"])
    st, _ = O.solve(P, lambda p: I.philox_uniform_indices(0, p * 50, 50, 50), max_passes=20, gap_every=20)
    Xh = O.barycentric(st.T, d["X"], d["Y"])
    Y = d["Y"].astype(np.float64)
    assert np.all(Xh >= Y.min(axis=0) - 1e-15) and np.all(Xh <= Y.max(axis=0) + 1e-15)
