"""Differentiable semi-relaxed OT value through libsrot (argument marshalling).

semi_relaxed_ot(a, b, C=None, X=None, Y=None, w=1.0, ...) solves
    V = min { <T, C> + (w/2) ||T^T 1 - b||^2 : T >= 0, T 1 = a }
with the BCFW solver (srot_solve) and returns V as a 0-d float64 tensor.
The cost is either a stored matrix C (float32 or float64, m x n) or, when C
is None, the squared Euclidean distance of the float32 point sets X (m x 3)
and Y (n x 3), evaluated on the fly.  Backward calls srot_backward at the
converged plan: gradients flow to C (stored cost) or to X and Y (fused
cost), and to a and b.  They are the envelope-theorem derivatives, exact
at an optimal plan; at the plan where the solver stopped (duality gap <= eps)
their accuracy follows from that gap.
"""
import warnings

import torch

from . import srot as S


class SemiRelaxedOT(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b, C, X, Y, w, eps, max_passes, seed):
        fused = C is None
        sol = S.Solver(a.detach().contiguous(), b.detach().contiguous(),
                       C=None if fused else C.detach().contiguous(),
                       X=X.detach().contiguous() if fused else None,
                       Y=Y.detach().contiguous() if fused else None,
                       w=float(w), eps=float(eps), max_passes=int(max_passes), seed=int(seed))
        status, (g, f, D), passes = sol.solve()
        if status != S.SROT_OK:
            # an unconverged plan: V is an upper bound within g of the
            # optimum, and the envelope gradients are only approximate
            warnings.warn(f"semi_relaxed_ot: no convergence to gap {eps:g} in {passes} passes "
                          f"(gap {g:.3e}); the value and its gradients are those of the last plan",
                          RuntimeWarning, stacklevel=3)
        ctx.sol = sol
        ctx.fused = fused
        ctx.info = dict(status=status, gap=g, f=f, dual=D, passes=passes)
        return torch.tensor(f, dtype=torch.float64, device=a.device)

    @staticmethod
    def backward(ctx, grad_V):
        need_a, need_b, need_C, need_X, need_Y = ctx.needs_input_grad[:5]
        sol = ctx.sol
        out = sol.backward(float(grad_V), dC=need_C and not ctx.fused,
                           dX=need_X and ctx.fused, dY=need_Y and ctx.fused,
                           da=need_a, db=need_b)
        return (out.get("da"), out.get("db"), out.get("dC"), out.get("dX"), out.get("dY"),
                None, None, None, None)


def semi_relaxed_ot(a, b, C=None, X=None, Y=None, w=1.0, eps=1e-6, max_passes=1000, seed=0):
    """Optimal value of the semi-relaxed problem (see the module docstring)."""
    if C is None and (X is None or Y is None):
        raise ValueError("give a stored cost C or both point sets X and Y")
    return SemiRelaxedOT.apply(a, b, C, X, Y, w, eps, max_passes, seed)
