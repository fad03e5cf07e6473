"""srot_backward_noalloc (the allocation-free srot_backward: its scratch in
the library's static device array) against srot_backward on the same
handles, through the C ABI: bit-identical outputs on two calls in a row,
the second with a smaller problem, so that the static scratch holds the
first call's contents when the second runs; and the size limit is refused
with an error before any kernel runs."""
import numpy as np
import pytest
import torch

from paper_2103_05857_amd import inputs as I

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _S():
    from paper_2103_05857_amd import srot as S
    return S


def _solver(d, fused, w, passes):
    S = _S()
    a = torch.from_numpy(d["a"]).to(DEV)
    b = torch.from_numpy(d["b"]).to(DEV)
    if fused:
        sol = S.Solver(a, b, X=torch.from_numpy(d["X"]).to(DEV), Y=torch.from_numpy(d["Y"]).to(DEV), w=w, seed=3)
    else:
        sol = S.Solver(a, b, C=torch.from_numpy(d["C"]).to(DEV), w=w, seed=3)
    sol.step(passes * sol.m)
    return sol


def _outputs(sol, fused, fn, g):
    m, n = sol.m, sol.n
    out = dict(da=torch.full((m,), np.nan, dtype=torch.float64, device=DEV),
               db=torch.full((n,), np.nan, dtype=torch.float64, device=DEV))
    if fused:
        out["dX"] = torch.full((m, 3), np.nan, dtype=torch.float32, device=DEV)
        out["dY"] = torch.full((n, 3), np.nan, dtype=torch.float32, device=DEV)
    else:
        out["dC"] = torch.full((m, n), np.nan, dtype=torch.float32, device=DEV)
    fn(sol.h, g, out.get("dC"), out.get("dX"), out.get("dY"), out["da"], out["db"])
    torch.cuda.synchronize()
    return {k: v.cpu() for k, v in out.items()}


def _same(sol, fused, g):
    S = _S()
    ref = _outputs(sol, fused, S.srot_backward, g)
    got = _outputs(sol, fused, S.srot_backward_noalloc, g)
    for k in ref:
        assert torch.isfinite(ref[k]).all(), k
        assert torch.equal(got[k], ref[k]), k


def test_noalloc_backward_matches_backward_two_calls():
    print("noalloc: fused 3000 x 4096, then stored 200 x 700, then fused 40 x 96", flush=True)
    big = _solver(I.problem_mixture(7, 3000, 4096, with_cost=False), True, 1.0, 2)
    _same(big, True, 1.5)
    small = _solver(I.problem_mixture(8, 200, 700, cost_dtype=np.float32), False, 0.5, 3)
    _same(small, False, -2.0)
    tiny = _solver(I.problem_mixture(9, 40, 96, with_cost=False), True, 3.0, 5)
    _same(tiny, True, 0.25)
    # the big handle again, after the small calls left their scratch behind
    _same(big, True, 1.0)
    for s in (big, small, tiny):
        s.close()


def test_noalloc_backward_refuses_sizes_beyond_its_scratch():
    S = _S()
    m, n = 64, 12000                      # 24 n x 32 slices > 8 MiB for dY
    sol = _solver(I.problem_mixture(10, m, n, with_cost=False), True, 1.0, 1)
    dY = torch.zeros(n, 3, dtype=torch.float32, device=DEV)
    with pytest.raises(S.SrotError) as e:
        S.srot_backward_noalloc(sol.h, 1.0, dY=dY)
    assert e.value.status == S.SROT_EINVAL
    assert torch.count_nonzero(dY).item() == 0          # refused before any kernel
    # without dY the same handle fits
    _same_parts = {}
    for fn in (S.srot_backward, S.srot_backward_noalloc):
        dX = torch.empty(m, 3, dtype=torch.float32, device=DEV)
        da = torch.empty(m, dtype=torch.float64, device=DEV)
        db = torch.empty(n, dtype=torch.float64, device=DEV)
        fn(sol.h, 1.0, None, dX, None, da, db)
        torch.cuda.synchronize()
        _same_parts[fn.__name__] = (dX.cpu(), da.cpu(), db.cpu())
    for x, y in zip(_same_parts["srot_backward"], _same_parts["srot_backward_noalloc"]):
        assert torch.equal(x, y)
    sol.close()
