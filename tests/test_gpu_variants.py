"""Away-step (Alg. A.2) and pairwise (Alg. A.3) block steps on the GPU
against the FP64 oracle.

Bar: identical FW vertex, away vertex / direction and step size (1e-9
absolute) at every step up to the first step where the oracle reports a
rounding-level tie (margin <= 1e-12) of either vertex, or of the two slopes
of the BCAFW direction choice, and the GPU took the other tied option -- the
line search equalises the gradient on the two atoms it moves between, so
such ties recur by construction and either choice is correct.  At such a
divergence both sides continue in lockstep from the GPU's state after the
tied step, so every step of the run is compared; the final plan, f and g
match the oracle's as in the block-coordinate parity tests.  A second test takes every oracle step from
the GPU's own state, so that each GPU step is checked on its own; after many
passes both sides reach the optimum (g <= 1e-9) and agree on f.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2103_05857_amd import inputs as I

pytestmark = pytest.mark.gpu

DEV = "cuda"
TAU = 1e-12


def _S():
    from paper_2103_05857_amd import srot as S
    return S


def _pair(d, cost_mode, w, **opts):
    S = _S()
    a = torch.from_numpy(d["a"]).to(DEV)
    b = torch.from_numpy(d["b"]).to(DEV)
    if cost_mode == "sqeuclid":
        sol = S.Solver(a, b, X=torch.from_numpy(d["X"]).to(DEV), Y=torch.from_numpy(d["Y"]).to(DEV), w=w, **opts)
        P = O.Problem(d["a"], d["b"], w, X=d["X"], Y=d["Y"])
    else:
        sol = S.Solver(a, b, C=torch.from_numpy(d["C"]).to(DEV), w=w, **opts)
        P = O.Problem(d["a"], d["b"], w, C=d["C"].astype(np.float64))
    return sol, P


def _run_gpu(sol, variant, idx):
    S = _S()
    ns = len(idx)
    tj = torch.empty(ns, dtype=torch.int32, device=DEV)
    ta = torch.empty(ns, dtype=torch.int32, device=DEV)
    tg = torch.empty(ns, dtype=torch.float64, device=DEV)
    S.srot_step_variant(sol.h, variant, ns, torch.from_numpy(idx).to(DEV), tj, ta, tg)
    torch.cuda.synchronize()
    return tj.cpu().numpy(), ta.cpu().numpy(), tg.cpu().numpy()


def _screened(cost_mode, dtype, n):
    """Stored FP32 rows of 513-4096 columns (a multiple of 4): the steps run
    on the screened chain's stepper."""
    return cost_mode == "stored" and dtype == np.float32 and 513 <= n <= 4096 and n % 4 == 0


def _first_divergence(otr, gj, ga, gg, sizes_may_differ=False):
    """Index of the first step where the GPU and the oracle differ (len(gj)
    if none), after checking that the difference is allowed.  With
    sizes_may_differ, a step with the same vertices and direction but
    another step size is returned unchecked: the caller compares the plans
    after it (a direction that is zero up to rounding leaves the plan as it
    is for any step size)."""
    oa = otr["away"]
    same = (gj == otr["j"]) & (ga == oa) & (np.abs(gg - otr["gamma"]) <= 1e-9)
    bad = np.nonzero(~same)[0]
    if len(bad) == 0:
        return len(gj)
    k = int(bad[0])
    if sizes_may_differ and gj[k] == otr["j"][k] and ga[k] == oa[k]:
        return k
    # a divergence is only allowed where the oracle's choice was a rounding-level tie
    gja = -1 - ga[k] if ga[k] < 0 else ga[k]
    tie_j = otr["margin"][k] <= TAU and gj[k] in otr["near"][k]
    tie_a = otr["amargin"][k] <= TAU and gja in otr["anear"][k]
    # the FW / away direction choice may differ only where the oracle's two
    # slopes are equal to rounding
    tie_dir = (gj[k] == otr["j"][k] and gja == (-1 - oa[k] if oa[k] < 0 else oa[k])
               and (ga[k] < 0) != (oa[k] < 0) and abs(otr["dslope"][k]) <= TAU)
    assert tie_j or tie_a or tie_dir, (k, gj[k], otr["j"][k], ga[k], oa[k], gg[k], otr["gamma"][k],
                                       otr["margin"][k], otr["amargin"][k])
    return k


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("cost_mode,dtype,m,n,w", [
    ("stored", np.float64, 64, 96, 1.0),
    ("stored", np.float32, 300, 700, 0.5),
    ("sqeuclid", None, 200, 333, 2.0),
    ("stored", np.float32, 97, 4096, 1.0),
    ("stored", np.float32, 50, 1500, 1.0),         # the screened chain with 8 columns per owner thread
    ("stored", np.float32, 40, 6000, 1.0),         # wide rows: 512 threads x 12 columns
    ("sqeuclid", None, 30, 8192, 1.0),
])
def test_variant_traces_match_oracle(variant, cost_mode, dtype, m, n, w):
    """Every step of six passes in lockstep: both sides run from a common
    state until the first difference, which must be a rounding-level tie of
    the oracle; then the GPU is rolled back to the common state, takes the
    steps up to and including the tied one, and both continue from the GPU's
    state after it.  Ties must stay rare."""
    d = I.problem_mixture(14, m, n, cost_dtype=dtype or np.float32)
    sol, P = _pair(d, cost_mode, w)
    idx = I.philox_uniform_indices(5, 0, 6 * m, m)
    ovar = O.PAIRWISE if variant == 2 else O.AWAY
    pos, ties, slow = 0, 0, 0
    while True:
        T0, r0 = sol.plan()
        st = O.State(P, T0.cpu().numpy())
        st.r = r0.cpu().numpy().copy()
        otr = O.active_steps(P, st, idx[pos:], ovar)
        gj, ga, gg = _run_gpu(sol, variant, idx[pos:])
        slow += _S().srot_chain_stats(sol.h)[1]
        k = _first_divergence(otr, gj, ga, gg, sizes_may_differ=True)
        if k == len(idx) - pos:
            break
        sol.set_state(T0, pos, r0)
        _run_gpu(sol, variant, idx[pos:pos + k + 1])
        if gj[k] == otr["j"][k] and ga[k] == otr["away"][k]:
            # same vertices and direction, another step size: allowed only
            # where the plans after the step agree (a direction that is zero
            # up to rounding)
            st1 = O.State(P, T0.cpu().numpy())
            st1.r = r0.cpu().numpy().copy()
            O.active_steps(P, st1, idx[pos:pos + k + 1], ovar, trace=False)
            T1, _ = sol.plan()
            np.testing.assert_allclose(T1.cpu().numpy(), st1.T, rtol=0, atol=1e-12)
        pos += k + 1
        ties += 1
    assert ties <= 0.05 * len(idx), ties
    if _screened(cost_mode, dtype, n):
        assert _S().srot_chain_stats(sol.h)[2] == _S().SROT_CHAIN_SCREENED
        # rows revisited within the stepper's history were re-read from the
        # plan (about 3% of the steps here)
        assert slow > 0
    T, r = sol.plan()
    T = T.cpu().numpy()
    np.testing.assert_allclose(T, st.T, rtol=0, atol=1e-9)
    ref = O.gap(P, st.T)
    g, f, D = sol.gap()
    assert abs(f - ref["f"]) <= 1e-6 * abs(ref["f"]) + 1e-15
    assert abs(g - ref["g"]) <= 1e-6 * max(ref["g"], 1e-9) + 1e-15
    assert T.min() >= 0.0
    np.testing.assert_allclose(T.sum(axis=1), d["a"], rtol=1e-12)
    np.testing.assert_allclose(r.cpu().numpy(), T.sum(axis=0) - d["b"], rtol=0, atol=1e-13)
    sol.close()


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("cost_mode,dtype,m,n,w", [
    ("stored", np.float64, 48, 96, 1.0),
    ("stored", np.float32, 60, 300, 0.5),
    ("sqeuclid", None, 40, 77, 2.0),
    ("stored", np.float64, 24, 5000, 1.0),
    ("stored", np.float32, 40, 1000, 1.0),       # the screened chain's stepper (513-4096 columns)
    ("stored", np.float32, 24, 700, 10.0),       # wider supports at a large penalty
])
def test_every_step_from_the_gpu_state(variant, cost_mode, dtype, m, n, w):
    """The oracle takes each step from the GPU's own state (plan and
    residual), so every GPU step is checked: same FW and away vertices and
    direction unless the oracle reports a rounding-level tie of the one that
    differs, and then the same step size and plan."""
    S = _S()
    d = I.problem_mixture(17, m, n, cost_dtype=dtype or np.float32)
    sol, P = _pair(d, cost_mode, w)
    idx = I.philox_uniform_indices(6, 0, 4 * m, m)
    ovar = O.PAIRWISE if variant == 2 else O.AWAY
    checked = 0
    for k in range(len(idx)):
        T, r = sol.plan()
        st = O.State(P, T.cpu().numpy())
        st.r = r.cpu().numpy().copy()
        otr = O.active_steps(P, st, idx[k:k + 1], ovar)
        gj, ga, gg = _run_gpu(sol, variant, idx[k:k + 1])
        oa = otr["away"][0]
        gja = -1 - ga[0] if ga[0] < 0 else ga[0]
        oja = -1 - oa if oa < 0 else oa
        if gj[0] != otr["j"][0]:
            assert otr["margin"][0] <= TAU and gj[0] in otr["near"][0]
            continue
        if gja != oja:
            assert otr["amargin"][0] <= TAU and gja in otr["anear"][0]
            continue
        if (ga[0] < 0) != (oa < 0):
            # FW and away slopes equal to rounding: either direction is the
            # algorithm's choice
            assert abs(otr["dslope"][0]) <= TAU, (k, otr["dslope"][0])
            continue
        T2, _ = sol.plan()
        np.testing.assert_allclose(T2.cpu().numpy(), st.T, rtol=0, atol=1e-12)
        i = int(idx[k])
        if np.abs(st.T[i] - T.cpu().numpy()[i]).max() > 1e-14:
            # a direction that is zero up to rounding (one atom at the FW
            # vertex) leaves the plan as it is for any step size; only then
            # may the sizes differ
            assert abs(gg[0] - otr["gamma"][0]) <= 1e-9, (k, gg[0], otr["gamma"][0])
        checked += 1
    assert checked >= 0.8 * len(idx)
    if _screened(cost_mode, dtype, n):
        assert S.srot_chain_stats(sol.h)[2] == S.SROT_CHAIN_SCREENED   # the screened kernel took the steps
    sol.close()


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("dtype,n", [(np.float64, 50), (np.float32, 600)])   # FP32 600: the screened chain
def test_variants_converge_to_the_optimum(variant, dtype, n):
    S = _S()
    m, w = 40, 1.0
    d = I.problem_mixture(15, m, n, cost_dtype=dtype)
    sol, P = _pair(d, "stored", w, eps=1e-9, max_passes=20000, seed=1)
    st, (g, f, D), passes = S.srot_solve_variant(sol.h, variant)
    sol.close()
    assert st == S.SROT_OK and g <= 1e-9
    ost = O.State(P)
    O.active_steps(P, ost, I.philox_uniform_indices(1, 0, passes * m, m),
                   O.PAIRWISE if variant == 2 else O.AWAY, trace=False)
    ref = O.gap(P, ost.T)
    assert ref["g"] <= 1e-7
    assert abs(f - ref["f"]) <= g + ref["g"] + 1e-15       # both within their gaps of f*


@pytest.mark.parametrize("variant,gap_every,max_passes,n,dtype", [
    (1, 1, 400, 90, np.float64), (2, 2, 400, 90, np.float64), (1, 1, 11, 90, np.float64),
    (2, 1, 400, 700, np.float32)])                                   # FP32 700: the screened chain
def test_solve_variant_leaves_the_state_of_its_stopping_pass(variant, gap_every, max_passes, n, dtype):
    """The stop test runs on the device with passes queued ahead: the plan
    and residual left are those of the stopping pass (as stepping that many
    passes by hand) and (g, f, D) is the sweep of that state."""
    S = _S()
    m = 60
    d = I.problem_mixture(16, m, n, cost_dtype=dtype)
    opts = dict(eps=1e-7, max_passes=max_passes, gap_every=gap_every, seed=3)
    sol, _ = _pair(d, "stored", 1.0, **opts)
    ref, _ = _pair(d, "stored", 1.0, **opts)
    st, (g, f, D), passes = S.srot_solve_variant(sol.h, variant)
    for _ in range(passes):
        S.srot_step_variant(ref.h, variant, m)  # one launch per pass, as the solve
    T1, r1 = sol.plan()
    T2, r2 = ref.plan()
    assert torch.equal(T1, T2) and torch.equal(r1, r2)
    assert (g, f, D) == tuple(ref.gap())
    if st == S.SROT_OK:
        assert g <= 1e-7 and passes % gap_every == 0
    else:
        assert passes == max_passes
    sol.close()
    ref.close()


def test_variant_argument_checks():
    S = _S()
    d = I.problem_mixture(16, 10, 12, cost_dtype=np.float64)
    sol, _ = _pair(d, "stored", 1.0, step_rule=S.SROT_DEC)
    with pytest.raises(S.SrotError):
        S.srot_step_variant(sol.h, S.SROT_STEP_PAIRWISE, 5)      # decay rule
    sol.close()
    sol, _ = _pair(d, "stored", 1.0)
    with pytest.raises(S.SrotError):
        S.srot_step_variant(sol.h, 7, 5)
    bad = torch.tensor([0, 10], dtype=torch.int32, device=DEV)
    with pytest.raises(S.SrotError):
        S.srot_step_variant(sol.h, S.SROT_STEP_AWAY, 2, bad)
    sol.close()
