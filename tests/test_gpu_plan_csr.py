"""The plan in compressed sparse rows (srot_get_plan_csr) against the dense
plan: row i's entries are exactly its support (the active set of Sec. 4.1,
eq. ActiveSet: the columns with t_ij > 0) in ascending column order, with
the plan's values bit for bit; a buffer one entry short gets SROT_ECAPACITY
and the count."""
import numpy as np
import pytest
import torch

from paper_2103_05857_amd import inputs as I

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _S():
    from paper_2103_05857_amd import srot as S
    return S


def _solver(d, cost_mode, w):
    S = _S()
    a = torch.from_numpy(d["a"]).to(DEV)
    b = torch.from_numpy(d["b"]).to(DEV)
    if cost_mode == "sqeuclid":
        return S.Solver(a, b, X=torch.from_numpy(d["X"]).to(DEV), Y=torch.from_numpy(d["Y"]).to(DEV), w=w)
    return S.Solver(a, b, C=torch.from_numpy(d["C"]).to(DEV), w=w)


@pytest.mark.parametrize("cost_mode,dtype,m,n,w,passes", [
    ("stored", np.float64, 64, 96, 1.0, 20),         # one-word layouts
    ("stored", np.float32, 200, 1000, 10.0, 6),      # the screened chain's layout, wide supports
    ("stored", np.float32, 40, 5000, 1.0, 5),        # rows of several mask words per thread
    ("sqeuclid", None, 30, 20000, 0.5, 3),           # the team chain's layout
    ("stored", np.float32, 1, 7, 1.0, 0),            # one row, the initial plan
    ("stored", np.float64, 20000, 16, 1.0, 1),       # rows beyond one launch's waves, 20 per scan thread
])
def test_csr_plan_matches_the_dense_plan(cost_mode, dtype, m, n, w, passes):
    S = _S()
    d = I.problem_mixture(21, m, n, cost_dtype=dtype or np.float32)
    sol = _solver(d, cost_mode, w)
    if passes:
        S.srot_step(sol.h, passes * m)
    row_ptr, col, val = sol.plan_csr()
    T, _ = sol.plan()
    torch.cuda.synchronize()
    T = T.cpu().numpy()
    rp, cj, tv = row_ptr.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
    nz = np.nonzero(T > 0)
    assert rp[0] == 0 and rp[-1] == len(nz[0]) == len(cj)
    assert np.array_equal(np.diff(rp), (T > 0).sum(axis=1))
    # rows in order, columns ascending within a row: the same order as np.nonzero
    assert np.array_equal(cj, nz[1])
    assert np.array_equal(tv, T[nz])                  # bit for bit
    # one entry short: the count comes back with SROT_ECAPACITY, col / val untouched
    nnz = len(cj)
    short_c = torch.full((nnz - 1,), -7, dtype=torch.int32, device=DEV)
    short_v = torch.full((nnz - 1,), -7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(S.SrotError) as e:
        S.srot_get_plan_csr(sol.h, row_ptr, short_c, short_v)
    assert e.value.status == S.SROT_ECAPACITY
    assert S.srot_get_plan_csr(sol.h, row_ptr) == nnz
    assert bool((short_c == -7).all()) and bool((short_v == -7.0).all())
    sol.close()
