"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Both sides get the same seeded inputs from paper_2103_05857_amd.inputs and the
same block-index stream (given explicitly, or drawn by the library's Philox
sampler and by numpy's Philox on the oracle side).

Bar (floating point, FP64 arithmetic on both sides; C may be stored in FP32
and is widened exactly):
  * LMO vertex j* identical at every step, except that where the oracle's
    margin to its runner-up vertex is <= 1e-12 (a rounding-level tie; the
    two sides round r differently by ~1e-16) any column within 1e-12 of the
    oracle's minimum is accepted: exact line search makes the gradient equal
    on the atoms of the row it moves, so such ties recur by construction;
  * step sizes within 1e-9 absolute;
  * per-pass objective f within 1e-6 relative and gap g within
    1e-6 * max(g, 1e-9) + 1e-15 (the stated 1e-6 relative tolerance, with an absolute
    floor for FP64 rounding of a tiny difference).
"""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2103_05857_amd import inputs as I

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _S():
    from paper_2103_05857_amd import srot as S
    return S


def _gpu_problem(d, cost_mode, w, **opts):
    S = _S()
    a = torch.from_numpy(d["a"]).to(DEV)
    b = torch.from_numpy(d["b"]).to(DEV)
    if cost_mode == "sqeuclid":
        X = torch.from_numpy(d["X"]).to(DEV)
        Y = torch.from_numpy(d["Y"]).to(DEV)
        return S.Solver(a, b, X=X, Y=Y, w=w, **opts)
    C = torch.from_numpy(d["C"]).to(DEV)
    return S.Solver(a, b, C=C, w=w, **opts)


def _oracle_problem(d, cost_mode, w):
    if cost_mode == "sqeuclid":
        return O.Problem(d["a"], d["b"], w, X=d["X"], Y=d["Y"])
    return O.Problem(d["a"], d["b"], w, C=d["C"].astype(np.float64))


def _compare_traces(otr, gj, gg, tau=1e-12, gtol=1e-9):
    """Step-by-step parity of (j*, gamma).  At a near-tie of the oracle's LMO
    (margin to the runner-up <= tau) either vertex is a correct LMO answer:
    exact line search leaves the gradient equal on a row's atoms, so such
    rounding-level ties recur by construction.  Returns the number of
    steps decided at a near-tie."""
    oj, og, om = otr
    gj = gj.cpu().numpy()
    gg = gg.cpu().numpy()
    assert gj.shape == oj.shape
    # any column within 1e-12 of the oracle's minimum is an LMO answer
    ok_j = (gj == oj) | ((om <= tau) & (otr.near == gj[:, None]).any(axis=1))
    ok_g = np.abs(gg - og) <= gtol
    bad = np.nonzero(~(ok_j & ok_g))[0]
    assert len(bad) == 0, (bad[:5], gj[bad[:5]], oj[bad[:5]], otr.near[bad[:5]], om[bad[:5]],
                           gg[bad[:5]], og[bad[:5]])
    return int(np.sum(om <= tau))


def _close_fg(gpu, ref):
    g, f, D = gpu
    assert abs(f - ref["f"]) <= 1e-6 * abs(ref["f"]) + 1e-15
    assert abs(g - ref["g"]) <= 1e-6 * max(ref["g"], 1e-9) + 1e-15
    assert abs(D - ref["D"]) <= 1e-6 * abs(ref["D"]) + 1e-13


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cost_mode,dtype,m,n,w,dirichlet_b", [(*c, False)[:6] for c in [
    ("stored", np.float64, 256, 256, 1.0),     # uniform RGB, FP64 C (small config)
    ("stored", np.float32, 300, 700, 0.1),     # ragged, several tiles
    ("stored", np.float32, 333, 1500, 10.0),
    ("stored", np.float32, 97, 4096, 1.0),      # full row width of the 4096 config
    ("sqeuclid", None, 200, 777, 1.0),
    ("stored", np.float32, 41, 5000, 1.0),      # global-residual kernel
    ("sqeuclid", None, 37, 6001, 3.0),          # wide rows: FP32 screen, points in registers
    ("sqeuclid", None, 23, 12001, 1.0),         # wide rows, 32 columns per thread
    ("sqeuclid", None, 11, 20000, 0.5),         # wide rows, points streamed from L2
    ("sqeuclid", None, 5, 32768, 10.0),         # the widest screened row
    # target weights b ~ Dirichlet(1), as in the 32768-point fused workload
    ("sqeuclid", None, 9, 32768, 1.0, True),
    ("sqeuclid", None, 13, 9000, 1.0, True),
    ("stored", np.float32, 97, 4096, 1.0, True),
]])
def test_trace_parity_explicit_indices(cost_mode, dtype, m, n, w, dirichlet_b):
    _need_gpu()
    d = I.problem_mixture(5, m, n, cost_dtype=dtype or np.float32, dirichlet_b=dirichlet_b)
    passes = 6
    idx = I.philox_uniform_indices(21, 0, passes * m, m)
    P = _oracle_problem(d, cost_mode, w)
    st = O.State(P)
    otr = O.bcfw_steps(P, st, idx, rule=O.ELS)
    ref = O.gap(P, st.T)

    S = _S()
    sol = _gpu_problem(d, cost_mode, w)
    gj, gg = sol.step(len(idx), idx=torch.from_numpy(idx).to(DEV), trace=True)
    kind = S.srot_chain_stats(sol.h)[2]
    if n > 4096:
        assert kind == S.SROT_CHAIN_TEAM
    elif cost_mode == "stored" and dtype == np.float32 and n > 512 and n % 4 == 0:
        assert kind == S.SROT_CHAIN_SCREENED
    else:
        assert kind == S.SROT_CHAIN_PREFETCH
    _compare_traces(otr, gj, gg)
    _close_fg(sol.gap(), ref)
    T, r = sol.plan()
    T = T.cpu().numpy()
    np.testing.assert_allclose(T, st.T, rtol=1e-9, atol=1e-12)
    assert T.min() >= 0.0
    np.testing.assert_allclose(T.sum(axis=1), d["a"], rtol=1e-12)
    np.testing.assert_allclose(r.cpu().numpy(), T.sum(axis=0) - d["b"], rtol=0, atol=1e-13)


def _trace_case(d, cost_mode, w, idx, rule=O.ELS, **opts):
    """Runs idx on both sides and applies the block-step bar; returns the
    solver (open) and the oracle state."""
    S = _S()
    P = _oracle_problem(d, cost_mode, w)
    st = O.State(P)
    otr = O.bcfw_steps(P, st, idx, rule=rule)
    sol = _gpu_problem(d, cost_mode, w, step_rule=(S.SROT_DEC if rule == O.DEC else S.SROT_ELS), **opts)
    gj, gg = sol.step(len(idx), idx=torch.from_numpy(idx).to(DEV), trace=True)
    _compare_traces(otr, gj, gg)
    _close_fg(sol.gap(), O.gap(P, st.T))
    T, r = sol.plan()
    T = T.cpu().numpy()
    np.testing.assert_allclose(T, st.T, rtol=1e-9, atol=1e-12)
    assert T.min() >= 0.0
    np.testing.assert_allclose(T.sum(axis=1), d["a"], rtol=1e-12)
    np.testing.assert_allclose(r.cpu().numpy(), T.sum(axis=0) - d["b"], rtol=0, atol=1e-13)
    return sol, st


@pytest.mark.parametrize("cost_mode,dtype,m,n,w,rule,passes", [
    ("sqeuclid", None, 3, 9000, 1.0, O.ELS, 60),        # 3 rows: revisits inside the prefetch window
    ("stored", np.float32, 4, 4097, 2.0, O.ELS, 40),    # one column past 4096: a member with one live column
    ("stored", np.float64, 7, 6000, 0.5, O.ELS, 20),    # FP64 stored cost, ragged last member
    ("sqeuclid", None, 5, 65536, 1.0, O.ELS, 6),        # the widest team (64 members)
    ("sqeuclid", None, 17, 12000, 3.0, O.DEC, 8),       # decay rule
    ("stored", np.float32, 2, 5000, 10.0, O.ELS, 150),  # two rows, strong penalty: supports over members
])
def test_team_chain_traces_match_oracle(cost_mode, dtype, m, n, w, rule, passes):
    """Rows wider than 4096 columns take the team chain (workgroups of 1024
    columns exchanging one record per step): the block-step bar on its
    corner cases, and the support masks it maintains with atomics match
    the plan (the gap sweep reads the plan through them)."""
    _need_gpu()
    S = _S()
    d = I.problem_mixture(31, m, n, cost_dtype=dtype or np.float32, dirichlet_b=(m == 17))
    idx = I.philox_uniform_indices(13, 0, passes * m, m)
    sol, st = _trace_case(d, cost_mode, w, idx, rule=rule)
    assert S.srot_chain_stats(sol.h)[2] == S.SROT_CHAIN_TEAM
    if m <= 4:
        assert (st.T > 0).sum(axis=1).max() >= 3        # several atoms per row were exercised
    sol.close()


@pytest.mark.parametrize("cost_mode,dtype,m,n,w", [
    ("stored", np.float32, 41, 5000, 1.0),
    ("sqeuclid", None, 11, 20000, 0.5),
])
def test_one_workgroup_wide_chains(cost_mode, dtype, m, n, w):
    """SROT_TEAM_CHAIN=0 at init keeps the one-workgroup chains for wide rows
    (global residual for stored costs, FP32-screened for fused ones)."""
    _need_gpu()
    S = _S()
    d = I.problem_mixture(5, m, n, cost_dtype=dtype or np.float32)
    idx = I.philox_uniform_indices(21, 0, 4 * m, m)
    os.environ["SROT_TEAM_CHAIN"] = "0"
    try:
        sol, _ = _trace_case(d, cost_mode, w, idx)
    finally:
        del os.environ["SROT_TEAM_CHAIN"]
    assert S.srot_chain_stats(sol.h)[2] == (S.SROT_CHAIN_WIDE if cost_mode == "sqeuclid" else S.SROT_CHAIN_GLOBAL)
    sol.close()


def test_small_config_500_passes_internal_sampler():
    """m = n = 256 uniform RGB, FP64 C, w = 1, 500 passes, seed 0: the library
    draws its own Philox indices; the oracle uses numpy's Philox stream."""
    _need_gpu()
    m = n = 256
    d = I.problem_uniform_c1(0, m, n)
    P = O.Problem(d["a"], d["b"], 1.0, C=d["C"])
    st = O.State(P)
    idx = I.philox_uniform_indices(0, 0, 500 * m, m)
    otr = O.bcfw_steps(P, st, idx, rule=O.ELS)
    ref = O.gap(P, st.T)

    sol = _gpu_problem(d, "stored", 1.0, seed=0)
    gj, gg = sol.step(500 * m, trace=True)
    _compare_traces(otr, gj, gg)
    _close_fg(sol.gap(), ref)
    assert sol.k == 500 * m


def test_solve_stops_at_same_pass_as_oracle():
    _need_gpu()
    m, n, w = 512, 640, 1.0
    d = I.problem_mixture(2, m, n)
    P = O.Problem(d["a"], d["b"], w, C=d["C"].astype(np.float64))
    src = lambda p: I.philox_uniform_indices(4, p * m, m, m)
    st, hist = O.solve(P, src, eps=1e-6, max_passes=400)
    sol = _gpu_problem(d, "stored", w, seed=4, eps=1e-6, max_passes=400)
    status, (g, f, D), passes = sol.solve()
    assert status == _S().SROT_OK
    assert passes == hist[-1]["passes"]
    _close_fg((g, f, D), hist[-1])
    assert g <= 1e-6


@pytest.mark.parametrize("m,n,gap_every,max_passes", [(200, 300, 1, 400), (150, 256, 3, 400),
                                                       (96, 5000, 1, 400), (120, 700, 2, 13)])
def test_solve_leaves_the_state_of_its_stopping_pass(m, n, gap_every, max_passes):
    """The stop test runs on the device with passes queued ahead: the plan,
    residual and step counter left are those of the stopping pass (the same
    as stepping that many passes by hand), the reported (g, f, D) is the
    sweep of that state, and stepping on continues the same index stream.
    Covers gap_every > 1, a pass budget that ends mid-batch (13) and the
    team chain (5000 columns)."""
    _need_gpu()
    d = I.problem_mixture(5, m, n)
    opts = dict(seed=6, eps=1e-6, max_passes=max_passes, gap_every=gap_every)
    sol = _gpu_problem(d, "stored", 1.0, **opts)
    status, (g, f, D), passes = sol.solve()
    ref = _gpu_problem(d, "stored", 1.0, **opts)
    for _ in range(passes):
        ref.step(m)  # one launch per pass, as the solve (launch boundaries shape the chain's prefetch)
    T1, r1 = sol.plan()
    T2, r2 = ref.plan()
    assert torch.equal(T1, T2) and torch.equal(r1, r2)
    assert (g, f, D) == tuple(ref.gap())
    if status == _S().SROT_OK:
        assert g <= 1e-6 and passes % gap_every == 0
    else:
        assert passes == max_passes and g > 1e-6
    sol.step(m)
    ref.step(m)
    T1, _ = sol.plan()
    T2, _ = ref.plan()
    assert torch.equal(T1, T2)
    sol.close()
    ref.close()


@pytest.mark.parametrize("cost_mode,dtype", [("stored", np.float32), ("stored", np.float64),
                                             ("sqeuclid", np.float32)])
def test_gap_sweep_on_given_plans(cost_mode, dtype):
    """Shapes cover the row-strided sweep (odd widths, the fused cost) and
    the vector-stream sweep (widths divisible by the vector), with support
    masks of up to 512 words per row read ahead and wider ones (n = 20000)
    taking the slow path; about 5% of each row is in the support."""
    _need_gpu()
    rng = np.random.default_rng(3)
    shapes = [(1, 1, 1.0), (1, 9, 2.0), (17, 1, 0.5), (130, 257, 1.0), (64, 5003, 10.0),
              (3, 4, 1.0), (5, 8, 2.0), (130, 256, 1.0), (64, 5004, 10.0), (6, 20000, 1.0),
              (41, 8192, 1.0), (23, 12000, 0.5)]
    for (m, n, w) in shapes:
        d = I.problem_mixture(7, m, n, cost_dtype=dtype)
        T = rng.random((m, n)) * (rng.random((m, n)) < 0.05)
        T[np.arange(m), rng.integers(0, n, m)] += 0.3
        T = T / T.sum(axis=1, keepdims=True) * d["a"][:, None]
        P = _oracle_problem(d, cost_mode, w)
        ref = O.gap(P, T)
        sol = _gpu_problem(d, cost_mode, w)
        sol.set_state(torch.from_numpy(T).to(DEV), 0)
        (g, f, D), rg, rj = sol.gap(per_row=True)
        _close_fg((g, f, D), ref)
        np.testing.assert_array_equal(rj.cpu().numpy(), ref["jstar"])
        np.testing.assert_allclose(rg.cpu().numpy(), ref["grow"], rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("n", [4096, 8192, 12000])
def test_gap_sweep_exact_ties_take_the_lowest_column(n):
    """Rows whose minimum of c_ij + w r_j is attained exactly at three
    columns far apart (r equal there: no plan mass, uniform b): the sweep
    reports the lowest of them, also where rows start their column sweep at
    a rotated offset (8192 columns and more)."""
    _need_gpu()
    m = 9
    rng = np.random.default_rng(11)
    C = (1.0 + rng.random((m, n))).astype(np.float32)
    ties = np.stack([np.arange(m) + 100, np.arange(m) + n // 2 + 7, np.arange(m) + n - 40], axis=1)
    for i in range(m):
        C[i, ties[i]] = 0.25
    a = np.full(m, 1.0 / m)
    b = np.full(n, 1.0 / n)
    T = np.zeros((m, n))
    T[np.arange(m), (np.arange(m) * 37 + 1000) % n] = a  # away from the tied columns
    d = {"a": a, "b": b, "C": C}
    P = _oracle_problem(d, "stored", 1.0)
    ref = O.gap(P, T)
    np.testing.assert_array_equal(ref["jstar"], ties[:, 0])
    sol = _gpu_problem(d, "stored", 1.0)
    sol.set_state(torch.from_numpy(T).to(DEV), 0)
    (g, f, D), rg, rj = sol.gap(per_row=True)
    np.testing.assert_array_equal(rj.cpu().numpy(), ties[:, 0])
    _close_fg((g, f, D), ref)
    sol.close()


@pytest.mark.parametrize("n", [3000, 6000, 20000])
def test_fused_gap_sweep_exact_ties_take_the_lowest_column(n):
    """Fused cost: each row's own point copied into three target columns
    far apart (cost exactly 0 there, r equal: no plan mass, uniform b), so
    the row minimum is attained exactly three times; the sweep reports the
    lowest of them, also through the FP32 screen of rows wider than 4096
    columns."""
    _need_gpu()
    m = 7
    rng = np.random.default_rng(12)
    X = rng.random((m, 3)).astype(np.float32)
    Y = rng.random((n, 3)).astype(np.float32)
    ties = np.stack([np.arange(m) + 100, np.arange(m) + n // 2 + 5, n - 30 - np.arange(m)], axis=1)
    for i in range(m):
        Y[ties[i]] = X[i]
    a = np.full(m, 1.0 / m)
    b = np.full(n, 1.0 / n)
    T = np.zeros((m, n))
    T[np.arange(m), (np.arange(m) * 37 + 1000) % n] = a  # away from the tied columns
    d = {"a": a, "b": b, "X": X, "Y": Y}
    P = _oracle_problem(d, "sqeuclid", 1.0)
    ref = O.gap(P, T)
    np.testing.assert_array_equal(ref["jstar"], ties[:, 0])
    sol = _gpu_problem(d, "sqeuclid", 1.0)
    sol.set_state(torch.from_numpy(T).to(DEV), 0)
    (g, f, D), rg, rj = sol.gap(per_row=True)
    np.testing.assert_array_equal(rj.cpu().numpy(), ties[:, 0])
    np.testing.assert_allclose(rg.cpu().numpy(), ref["grow"], rtol=1e-9, atol=1e-15)
    _close_fg((g, f, D), ref)
    sol.close()


def test_gap_async_into_device_and_pinned_memory():
    """srot_gap_async: the final-sum kernel writes a device destination
    itself, a pinned host one gets a copy; both equal srot_gap bitwise."""
    _need_gpu()
    S = _S()
    for (m, n) in [(130, 256), (40, 8192), (33, 501)]:
        d = I.problem_mixture(4, m, n)
        sol = _gpu_problem(d, "stored", 1.0)
        sol.step(3 * m)
        ref = np.array(sol.gap())
        dev5 = torch.full((5,), float("nan"), dtype=torch.float64, device=DEV)
        host5 = torch.full((5,), float("nan"), dtype=torch.float64).pin_memory()
        S.srot_gap_async(sol.h, dev5)
        S.srot_gap_async(sol.h, host5)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(dev5.cpu().numpy()[:3], ref)
        np.testing.assert_array_equal(host5.numpy()[:3], ref)
        np.testing.assert_array_equal(dev5.cpu().numpy(), host5.numpy())
        sol.close()


def test_decay_rule_and_permutation_sampler():
    _need_gpu()
    m, n = 150, 210
    d = I.problem_mixture(9, m, n, cost_dtype=np.float64)
    P = O.Problem(d["a"], d["b"], 1.0, C=d["C"])
    st = O.State(P)
    idx = I.philox_permutation_indices(13, 0, 7, m)
    otr = O.bcfw_steps(P, st, idx, rule=O.DEC)
    sol = _gpu_problem(d, "stored", 1.0, seed=13, step_rule=_S().SROT_DEC, sampling=_S().SROT_PERMUTE)
    # 7 passes in uneven calls: sampler state must carry across calls
    parts = [1, 149, 300, 500, 0, 7 * m - 950]
    gjs, ggs = [], []
    for c in parts:
        if c == 0:
            continue
        gj, gg = sol.step(c, trace=True)
        gjs.append(gj); ggs.append(gg)
    gj = torch.cat(gjs); gg = torch.cat(ggs)
    _compare_traces(otr, gj, gg)
    # decay steps are bit-identical
    np.testing.assert_array_equal(gg.cpu().numpy(), otr[1])
    _close_fg(sol.gap(), O.gap(P, st.T))


def test_zero_penalty_closed_form_on_gpu():
    _need_gpu()
    m, n = 300, 260
    d = I.problem_mixture(11, m, n, cost_dtype=np.float64)
    sol = _gpu_problem(d, "stored", 0.0)
    perm = np.random.default_rng(0).permutation(m).astype(np.int32)
    sol.step(m, idx=torch.from_numpy(perm).to(DEV))
    T, _ = sol.plan()
    Texp = np.zeros((m, n))
    Texp[np.arange(m), np.argmin(d["C"], axis=1)] = d["a"]
    np.testing.assert_array_equal(T.cpu().numpy(), Texp)
    g, f, D = sol.gap()
    assert g == 0.0
    assert abs(f - float(np.sum(d["a"] * d["C"].min(axis=1)))) < 1e-15


def test_exact_ties_pick_lowest_column():
    _need_gpu()
    # identical target points -> identical cost columns and equal b: while
    # neither twin has been touched, r is exactly -b_j on both sides and the
    # tie is exact, so the lowest column must win.  Once rounding separates the
    # twins, either may win a later rounding-level tie with a nonzero step and
    # the two runs continue on twin-swapped (equivalent) plans, so the traces
    # are compared up to the first such divergence only.
    X = I.mixture_points(1, 40)
    Y = I.mixture_points(2, 30)
    Y[10:20] = Y[0:10]
    d = dict(X=X, Y=Y, a=I.uniform_weights(40), b=I.uniform_weights(30))
    d["C"] = I.sqeuclid_cost(X, Y, np.float64)
    d["b"][10:20] = d["b"][0:10]
    idx = I.philox_uniform_indices(8, 0, 40 * 20, 40)
    for mode in ("stored", "sqeuclid"):
        P = _oracle_problem(d, mode, 1.0)
        st = O.State(P)
        otr = O.bcfw_steps(P, st, idx)
        sol = _gpu_problem(d, mode, 1.0)
        gj, gg = sol.step(len(idx), idx=torch.from_numpy(idx).to(DEV), trace=True)
        gjn = gj.cpu().numpy()
        diff = np.nonzero(gjn != otr[0])[0]
        first = int(diff[0]) if len(diff) else len(idx)
        if first < len(idx):
            assert otr[2][first] <= 1e-12          # diverged only at a tie
        np.testing.assert_allclose(gg.cpu().numpy()[:first], otr[1][:first], rtol=0, atol=1e-9)
        touched = {0}
        checked = 0
        for k in range(first):
            tied = [c for c in otr.near[k] if c >= 0]
            if otr[2][k] == 0.0 and not any(c in touched for c in tied):
                assert gjn[k] == otr[0][k] == min(tied)
                checked += 1
            touched.add(int(otr[0][k]))
        assert checked > 0


@pytest.mark.parametrize("n", [9000, 20000])
def test_wide_rows_with_repeated_points_in_one_thread(n):
    """Wide fused rows where one thread owns several columns with the same
    target point (columns j and j + 512 k): equal cost entries, so its FP32
    screen has several candidates and the exact FP64 pass over all its
    columns decides; the lowest index must win while the twins are untouched."""
    _need_gpu()
    m = 24
    X = I.mixture_points(3, m)
    Y = I.mixture_points(4, n)
    for k in range(1, 4):
        Y[512 * k: 512 * k + 64] = Y[0:64]
    b = I.uniform_weights(n)
    d = dict(X=X, Y=Y, a=I.uniform_weights(m), b=b)
    idx = I.philox_uniform_indices(9, 0, m * 8, m)
    P = _oracle_problem(d, "sqeuclid", 1.0)
    st = O.State(P)
    otr = O.bcfw_steps(P, st, idx)
    sol = _gpu_problem(d, "sqeuclid", 1.0)
    gj, gg = sol.step(len(idx), idx=torch.from_numpy(idx).to(DEV), trace=True)
    gjn = gj.cpu().numpy()
    diff = np.nonzero(gjn != otr[0])[0]
    first = int(diff[0]) if len(diff) else len(idx)
    if first < len(idx):
        assert otr[2][first] <= 1e-12          # diverged only at a tie
    np.testing.assert_allclose(gg.cpu().numpy()[:first], otr[1][:first], rtol=0, atol=1e-9)


def test_rows_with_more_atoms_per_thread_than_prefetched():
    """Rows whose support holds three or four columns of one thread (adjacent
    columns of one 16-byte group) exceed the support entries the prefetching
    chain reads ahead; the chain then stops and the tail kernel finishes the
    launch.  The first such row is visited after 50 ordinary steps.  (The
    handle is created with SROT_LMO_SCREEN=0: at 1024 columns the default is
    the screened chain, whose own test covers such rows.)"""
    _need_gpu()
    m, n, w = 64, 1024, 1.0
    d = I.problem_mixture(19, m, n)
    a = d["a"]
    T = np.zeros((m, n))
    T[:, 0] = a
    for i in range(8):                      # four adjacent columns: one thread
        T[i, 0] = 0.0
        T[i, 4:8] = a[i] / 4
    for i in range(8, 16):                  # three adjacent columns
        T[i, 0] = 0.0
        T[i, 8:11] = a[i] / 3
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.integers(16, m, 50), np.tile(np.arange(16), 3),
                          rng.integers(0, m, 200)]).astype(np.int32)
    P = _oracle_problem(d, "stored", w)
    st = O.State(P, T)
    otr = O.bcfw_steps(P, st, idx, rule=O.ELS)
    os.environ["SROT_LMO_SCREEN"] = "0"
    try:
        sol = _gpu_problem(d, "stored", w)
    finally:
        del os.environ["SROT_LMO_SCREEN"]
    sol.set_state(torch.from_numpy(T).to(DEV), 0)
    gj, gg = sol.step(len(idx), idx=torch.from_numpy(idx).to(DEV), trace=True)
    _compare_traces(otr, gj, gg)
    Tg, r = sol.plan()
    Tg = Tg.cpu().numpy()
    np.testing.assert_allclose(Tg, st.T, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r.cpu().numpy(), Tg.sum(axis=0) - d["b"], rtol=0, atol=1e-13)


def test_resume_from_checkpoint_repeats_the_run():
    _need_gpu()
    m, n = 128, 300
    d = I.problem_mixture(12, m, n)
    full = _gpu_problem(d, "stored", 1.0, seed=5)
    full.step(10 * m)
    T_full, r_full = full.plan()

    part = _gpu_problem(d, "stored", 1.0, seed=5)
    part.step(4 * m + 17)
    T_mid, _ = part.plan()
    k_mid = part.k
    _, r_mid = part.plan()
    resumed = _gpu_problem(d, "stored", 1.0, seed=5)
    resumed.set_state(T_mid, k_mid, r_mid)
    resumed.step(10 * m - k_mid)
    T_res, r_res = resumed.plan()
    assert torch.equal(T_res, T_full)
    torch.testing.assert_close(r_res, r_full, rtol=0, atol=1e-15)


def test_runs_are_deterministic():
    _need_gpu()
    d = I.problem_mixture(13, 400, 900)
    outs = []
    for _ in range(2):
        sol = _gpu_problem(d, "stored", 1.0, seed=3)
        sol.step(5 * 400)
        outs.append(sol.plan()[0])
    assert torch.equal(outs[0], outs[1])


def test_error_paths():
    _need_gpu()
    S = _S()
    d = I.problem_mixture(14, 16, 16)
    sol = _gpu_problem(d, "stored", 1.0)
    bad = torch.tensor([0, 3, 16], dtype=torch.int32, device=DEV)
    with pytest.raises(S.SrotError) as e:
        sol.step(3, idx=bad)
    assert e.value.status == S.SROT_EINVAL
    assert sol.k == 0
    C = torch.from_numpy(d["C"]).to(DEV)
    C[3, 5] = float("nan")
    with pytest.raises(S.SrotError) as e:
        S.Solver(torch.from_numpy(d["a"]).to(DEV), torch.from_numpy(d["b"]).to(DEV), C=C)
    assert e.value.status == S.SROT_ENONFINITE
    a = torch.from_numpy(d["a"]).to(DEV)
    a[0] = -0.1
    with pytest.raises(S.SrotError) as e:
        S.Solver(a, torch.from_numpy(d["b"]).to(DEV), C=torch.from_numpy(d["C"]).to(DEV))
    assert e.value.status == S.SROT_ENONFINITE


def test_full_size_4096_first_passes_and_solve_properties():
    """m = n = 4096 mixture, FP32 C (64 MiB), in the benchmark's launch
    configuration: the first two passes match the oracle step by step; the
    solve to gap 1e-6 ends with a certified plan (invariants, f - D = g) whose
    value agrees with the oracle's own solve within the two gaps."""
    _need_gpu()
    m = n = 4096
    w = 1.0
    d = I.problem_mixture(0, m, n)
    P = O.Problem(d["a"], d["b"], w, C=d["C"].astype(np.float64))
    st = O.State(P)
    idx = I.philox_uniform_indices(0, 0, 2 * m, m)
    otr = O.bcfw_steps(P, st, idx)
    sol = _gpu_problem(d, "stored", w, seed=0, eps=1e-6, max_passes=200)
    gj, gg = sol.step(2 * m, trace=True)
    _compare_traces(otr, gj, gg)
    status, (g, f, D), passes = sol.solve()
    assert status == _S().SROT_OK and g <= 1e-6
    assert abs((f - D) - g) <= 1e-12
    T, r = sol.plan()
    T = T.cpu().numpy()
    assert T.min() >= 0
    np.testing.assert_allclose(T.sum(axis=1), d["a"], rtol=1e-12)
    np.testing.assert_allclose(r.cpu().numpy(), T.sum(axis=0) - d["b"], rtol=0, atol=1e-12)
    # oracle's own solve (same stream): both certified within their gaps
    src = lambda p: I.philox_uniform_indices(0, p * m, m, m)
    st2 = O.State(P)
    st2.T = st.T.copy(); st2.r = st.r.copy(); st2.k = st.k
    _, hist = O.solve(P, lambda p: src(p + 2), eps=1e-6, max_passes=200, state=st2)
    assert abs(f - hist[-1]["f"]) <= g + hist[-1]["g"] + 1e-12


def test_full_size_fused_32768_sampled_rows_and_invariants():
    """m = n = 32768 mixture points, fused cost, b ~ Dirichlet(1), w = 1, in
    the benchmark's launch configuration (one srot_step of m block steps per
    pass).  The dense FP64 oracle does not fit at this size, so after one
    pass the sweep's per-row outputs are checked on sampled rows against an
    FP64 evaluation of those rows (gradient minimum, vertex up to ties, row
    gap), and the plan against invariants that hold at any size: T >= 0,
    row sums a, r = T^T 1 - b, g = sum_i g_i."""
    _need_gpu()
    n = m = 32768
    w = 1.0
    d = I.problem_mixture(0, m, n, dirichlet_b=True, with_cost=False)
    sol = _gpu_problem(d, "sqeuclid", w, seed=0)
    sol.step(m)
    (g, f, D), rg, rj = sol.gap(per_row=True)
    T, r = sol.plan()
    b = torch.from_numpy(d["b"]).to(DEV)
    a = torch.from_numpy(d["a"]).to(DEV)
    assert T.min().item() >= 0.0
    torch.testing.assert_close(T.sum(dim=1), a, rtol=1e-12, atol=0.0)
    torch.testing.assert_close(r, T.sum(dim=0) - b, rtol=0.0, atol=1e-12)
    rg = rg.cpu().numpy()
    assert abs(g - rg.sum()) <= 1e-9 * abs(g)
    assert abs((f - D) - g) <= 1e-9 * max(abs(f), 1e-12)
    rows = np.random.default_rng(4).choice(m, 64, replace=False)
    rn = r.cpu().numpy()
    X = d["X"].astype(np.float64)
    Y = d["Y"].astype(np.float64)
    rjn = rj.cpu().numpy()
    Tr = T[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    for q, i in enumerate(rows):
        v = ((X[i][None, :] - Y) ** 2).sum(axis=1) + w * rn
        G = v.min()
        assert v[rjn[i]] - G <= 1e-12 * max(1.0, abs(G))
        gi = float(np.sum(Tr[q] * (v - G)))
        assert abs(rg[i] - gi) <= 1e-9 * max(gi, 1e-12) + 1e-15
    sol.close()
