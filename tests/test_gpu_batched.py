"""Batched solver (srot_init_batched / srot_solve_batched) on the GPU.

* With the default tile shapes every problem follows exactly the trajectory
  of the single-problem solver run with the same (prefetching) chain code
  (same tile shape, same Philox block-index stream; the single-problem
  handles are created with SROT_LMO_SCREEN=0, since the screened-LMO chain
  takes the same steps but sums the line-search partials in another order):
  plans and residuals must be bit-identical and the stop pass the same; the
  gap certificates (g, f, D) agree to FP64 rounding (the batched sweep sums
  rows in another order).
* Against the FP64 oracle directly: per-problem f and g after the passes the
  batched solver ran, under the parity bar of the single-problem tests.
* With autotuned tile shapes every problem still converges to the same
  optimum: f within 1e-6 relative of the single-problem solver's, g <= eps.
"""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2103_05857_amd import inputs as I

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _S():
    from paper_2103_05857_amd import srot as S
    return S


def _problems(seed, sizes):
    out = []
    for k, (m, n) in enumerate(sizes):
        d = I.problem_mixture(seed + k, m, n, cost_dtype=np.float32)
        out.append(d)
    return out


def _batch(probs, tune=False, **opts):
    S = _S()
    Cs = [torch.from_numpy(d["C"]).to(DEV) for d in probs]
    As = [torch.from_numpy(d["a"]).to(DEV) for d in probs]
    Bs = [torch.from_numpy(d["b"]).to(DEV) for d in probs]
    return S.BatchSolver(Cs, As, Bs, tune=tune, **opts)


SIZES = [(1, 1), (3, 1), (1, 7), (17, 5), (64, 64), (65, 130), (200, 257), (300, 700),
         (123, 1024), (50, 1500), (40, 2048), (33, 4096), (97, 4093), (256, 256)]


def test_batched_equals_single_problem_solver_bitwise():
    S = _S()
    probs = _problems(10, SIZES)
    opts = dict(w=1.0, eps=1e-6, max_passes=150, seed=3)
    bs = _batch(probs, **opts)
    st, out3, passes, status = bs.solve()
    tiles, _ = bs.tiles()
    for p, d in enumerate(probs):
        os.environ["SROT_LMO_SCREEN"] = "0"
        try:
            sol = S.Solver(torch.from_numpy(d["a"]).to(DEV), torch.from_numpy(d["b"]).to(DEV),
                           C=torch.from_numpy(d["C"]).to(DEV), **opts)
        finally:
            del os.environ["SROT_LMO_SCREEN"]
        s1, (g, f, D), np1 = sol.solve()
        T1, r1 = sol.plan()
        T2, r2 = bs.plan(p)
        torch.cuda.synchronize()
        assert passes[p] == np1, (p, passes[p], np1)
        assert status[p] == s1
        assert torch.equal(T1, T2), p
        assert torch.equal(r1, r2), p
        assert abs(out3[p, 1] - f) <= 1e-12 * abs(f) + 1e-18
        assert abs(out3[p, 0] - g) <= 1e-12 * max(abs(f), g) + 1e-18
        assert abs(out3[p, 2] - D) <= 1e-12 * abs(f) + 1e-18
        m, n = d["C"].shape
        assert tiles[p, 0] * tiles[p, 1] >= n
        sol.close()
    # replaying the graph repeats the solve exactly
    st2, out3b, passes2, status2 = bs.solve()
    assert np.array_equal(out3, out3b) and np.array_equal(passes, passes2)
    bs.close()


def test_batched_against_oracle():
    probs = _problems(30, [(40, 33), (64, 96), (9, 150)])
    w, eps, seed = 0.5, 1e-7, 1
    bs = _batch(probs, w=w, eps=eps, max_passes=400, seed=seed)
    st, out3, passes, status = bs.solve()
    bs.close()
    for p, d in enumerate(probs):
        m = d["C"].shape[0]
        P = O.Problem(d["a"], d["b"], w, C=d["C"].astype(np.float64))
        st_o, hist = O.solve(P, lambda q: I.philox_uniform_indices(seed, q * m, m, m),
                             eps=eps, max_passes=int(passes[p]), gap_every=1)
        ref = hist[-1]
        assert ref["passes"] == passes[p]
        assert abs(out3[p, 1] - ref["f"]) <= 1e-6 * abs(ref["f"]) + 1e-15
        assert abs(out3[p, 0] - ref["g"]) <= 1e-6 * max(ref["g"], 1e-9) + 1e-15


def test_batched_autotuned_tiles_converge_to_the_same_optimum():
    S = _S()
    probs = _problems(50, [(300, 700), (128, 1000), (200, 200), (64, 4096), (90, 60)])
    opts = dict(w=1.0, eps=1e-6, max_passes=4000, seed=0)
    bs = _batch(probs, tune=True, **opts)
    st, out3, passes, status = bs.solve()
    tiles, ms = bs.tiles()
    for p, d in enumerate(probs):
        m, n = d["C"].shape
        assert tiles[p, 0] * tiles[p, 1] >= n and ms[p] > 0
        sol = S.Solver(torch.from_numpy(d["a"]).to(DEV), torch.from_numpy(d["b"]).to(DEV),
                       C=torch.from_numpy(d["C"]).to(DEV), **opts)
        s1, (g, f, D), np1 = sol.solve()
        sol.close()
        info = (p, m, n, tuple(tiles[p]), status[p], passes[p], out3[p], s1, np1, g)
        assert status[p] == S.SROT_OK and out3[p, 0] <= 1e-6, info
        # both within the gap of the optimum: |f1 - f2| <= g1 + g2
        assert abs(out3[p, 1] - f) <= out3[p, 0] + g + 1e-15
        T, r = bs.plan(p)
        Th = T.cpu().numpy()
        np.testing.assert_allclose(Th.sum(axis=1), d["a"], rtol=0, atol=1e-15)
        assert Th.min() >= 0.0
        np.testing.assert_allclose(r.cpu().numpy(), Th.sum(axis=0) - d["b"], rtol=0, atol=1e-13)
    bs.close()


def test_batched_error_paths():
    S = _S()
    probs = _problems(70, [(8, 9), (5, 6)])
    with pytest.raises(S.SrotError) as e:
        _batch(probs, sampling=S.SROT_PERMUTE)
    assert e.value.status == S.SROT_EINVAL
    bad = [dict(d) for d in probs]
    bad[1]["C"] = bad[1]["C"].copy()
    bad[1]["C"][2, 3] = np.nan
    with pytest.raises(S.SrotError) as e:
        _batch(bad)
    assert e.value.status == S.SROT_ENONFINITE
    opt = S.srot_default_options()
    assert S.srot_workspace_size_batched([4, 4], [4, 5000], opt) == 0
    assert S.srot_workspace_size_batched([4, 0], [4, 4], opt) == 0
    C = torch.zeros(64, dtype=torch.float32, device=DEV)
    a = torch.full((8,), 0.125, dtype=torch.float64, device=DEV)
    ws = torch.empty(256, dtype=torch.uint8, device=DEV)
    with pytest.raises(S.SrotError) as e:
        S.srot_init_batched([4, 4], [4, 4], None, C, a, a, ws, opt)
    assert e.value.status == S.SROT_ENOMEM


def test_full_size_512_problems_autotuned():
    """The 512-problem workload (m, n log-uniform in [64, 4096], mixture
    palettes, FP32 costs, w = 1, gap 1e-6) in the benchmark's launch
    configuration (one graph launch, autotuned tiles): every problem reaches
    its gap, and sampled problems agree with the single-problem solver
    within the two gaps and satisfy the plan invariants."""
    S = _S()
    count = 512
    ms, ns = I.batched_sizes(0, count)
    probs = [I.batched_problem(0, p, int(ms[p]), int(ns[p])) for p in range(count)]
    opts = dict(w=1.0, eps=1e-6, max_passes=20000, seed=0)
    Cs = []
    for d in probs:   # squared Euclidean in FP64 on the device, stored in FP32
        X = torch.from_numpy(d["X"]).to(DEV).double()
        Y = torch.from_numpy(d["Y"]).to(DEV).double()
        Cs.append(((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1).float().contiguous())
    As = [torch.from_numpy(d["a"]).to(DEV) for d in probs]
    Bs = [torch.from_numpy(d["b"]).to(DEV) for d in probs]
    bs = S.BatchSolver(Cs, As, Bs, tune=True, **opts)
    st, out3, passes, status = bs.solve()
    assert np.all(status == S.SROT_OK) and np.all(out3[:, 0] <= 1e-6)
    assert np.allclose(out3[:, 1] - out3[:, 2], out3[:, 0], rtol=1e-9, atol=1e-15)
    small = [p for p in range(count) if ms[p] * ns[p] <= 300_000]
    for p in np.random.default_rng(1).choice(small, 6, replace=False):
        sol = S.Solver(As[p], Bs[p], C=Cs[p], **opts)
        s1, (g, f, D), _ = sol.solve()
        sol.close()
        assert s1 == S.SROT_OK
        assert abs(out3[p, 1] - f) <= out3[p, 0] + g + 1e-15
        T, r = bs.plan(int(p))
        Th = T.cpu().numpy()
        assert Th.min() >= 0.0
        np.testing.assert_allclose(Th.sum(axis=1), probs[p]["a"], rtol=1e-12)
        np.testing.assert_allclose(r.cpu().numpy(), Th.sum(axis=0) - probs[p]["b"], rtol=0, atol=1e-13)
    bs.close()
