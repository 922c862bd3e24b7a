"""torch.autograd binding of the solve: gradients with respect to the
coefficient fields, the source and the boundary data.

The backward pass reuses the factors stored by the forward build: one
transposed solve (hps_solve_adjoint) gives lam = G^T grad_u, and
hps_coeff_grad forms dJ/dc_t = -lam * d_t u at interior leaf points.  Both
run in the library's kernels; this module only marshals tensors.  With
subtree_depth > 0 the forward build keeps only the top levels
(hps_build_subtrees) and the backward pass rebuilds the subtrees' factors
from the coefficients instead of storing them (checkpointing, Section 4.1).
"""
from __future__ import annotations

import torch

from . import Operator, Tree


class HPSSolve(torch.autograd.Function):
    """u = solve(L(coeffs), bdry, src) with u [nrhs, n_leaves, p^dim]."""

    @staticmethod
    def forward(ctx, coeffs, bdry, src, t: Tree, p: int, subtree_depth: int = 0):
        op = Operator(t, p, coeffs.detach().contiguous(), subtree_depth=subtree_depth)
        u = op.solve(bdry.detach().contiguous(), None if src is None else src.detach().contiguous())
        ctx.op = op
        ctx.has_src = src is not None
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        (u,) = ctx.saved_tensors
        op = ctx.op
        need_c, need_b, need_s = ctx.needs_input_grad[:3]
        w = grad_u.contiguous()
        lam_bdry = None
        if need_b:
            lam_bdry = torch.empty((w.shape[0], op.sizes.n_root_bdry), dtype=torch.float64, device=w.device)
        lam_src, lam_bdry = op.solve_adjoint(w, lam_bdry=lam_bdry)
        grad_c = op.coeff_grad(u, lam_src) if need_c else None
        grad_s = lam_src if (need_s and ctx.has_src) else None
        return grad_c, lam_bdry, grad_s, None, None, None


def solve(t: Tree, p: int, coeffs, bdry, src=None, subtree_depth: int = 0):
    """Differentiable build + solve (see HPSSolve); subtree_depth > 0 builds
    with subtree recomputation."""
    return HPSSolve.apply(coeffs, bdry, src, t, p, subtree_depth)
