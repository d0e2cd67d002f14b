"""V-FPI step as a differentiable PyTorch operation, and a checkpointed rollout.

``vfpi_solve`` runs ``vfpi_step`` (FP64, to tolerance) in the forward pass and
``vfpi_step_backward`` (the hand-written adjoint of the converged step, with
the active branch of every contact's projection) in the backward pass;
gradients flow to A's values, b, phi, mu and (anisotropic friction) mu2.  The warm start carries no
gradient (the converged solution does not depend on it).

``rollout`` advances x_{k+1} = x_k + h v_{k+1} with a caller-supplied
differentiable ``assemble(x, v, *params)`` and keeps only every
``checkpoint_every``-th state: in the backward pass each segment is
recomputed (forward again, new tapes) and then differentiated.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from .solver import Bsr, Contacts, Solver


class VfpiStepFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A_val, b, phi, mu, v_warm, solver: Solver, row_ptr, col_idx, n_nodes, c_node, R, fwd_opts,
                bwd_opts, mu2=None):
        nc = int(c_node.numel())
        dev = b.device
        A = Bsr(n_nodes, row_ptr, col_idx, A_val.detach().contiguous())
        crp = torch.arange(nc + 1, dtype=torch.int32, device=dev)
        Jc = Contacts(nc, crp, c_node.contiguous(), R.detach().contiguous(), phi.detach().contiguous(),
                      mu.detach().contiguous(), None if mu2 is None else mu2.detach().contiguous())
        v = v_warm.detach().clone().contiguous()
        tape = solver.tape(n_nodes, nc)
        lam, stats = solver.step(A, b.detach().contiguous(), Jc, v, tape=tape, **fwd_opts)
        ctx.solver = solver
        ctx.A = A
        ctx.Jc = Jc
        ctx.bwd_opts = bwd_opts
        ctx.need_A = A_val.requires_grad
        ctx.save_for_backward(tape, stats)
        ctx.mark_non_differentiable(stats)
        return v, lam, stats

    @staticmethod
    def backward(ctx, gv, glam, _gstats):
        tape, _ = ctx.saved_tensors
        n = 3 * ctx.A.n_nodes
        gv = torch.zeros(n, dtype=torch.float64, device=tape.device) if gv is None else gv.contiguous()
        gl = None if glam is None else glam.contiguous()
        g = ctx.solver.step_backward(ctx.A, ctx.Jc, tape, gv, gl, want_A=ctx.need_A, **ctx.bwd_opts)
        gA = g["A"].view(-1, 3, 3) if ctx.need_A else None
        return gA, g["b"], g["phi"], g["mu"], None, None, None, None, None, None, None, None, None, g.get("mu2")


DEFAULT_FWD = dict(max_iters=100000, tol=1e-13)
DEFAULT_BWD = dict(max_iters=100000, tol=1e-13)


def vfpi_solve(solver, A_val, b, phi, mu, v_warm, row_ptr, col_idx, n_nodes, c_node, R, fwd_opts=None,
               bwd_opts=None, mu2=None):
    """Differentiable V-FPI step; returns (v, lambda, stats tensor).  The
    backward pass uses the forward's contact regularization (omega) and
    projection operator.  ``mu2`` (optional) is the second friction
    coefficient of anisotropic friction; it receives a gradient too."""
    fwd = dict(fwd_opts or DEFAULT_FWD)
    bwd = dict(bwd_opts or DEFAULT_BWD)
    bwd["omega"] = fwd.get("omega", 0.0)
    bwd["projection"] = fwd.get("projection", "strict")
    return VfpiStepFn.apply(A_val, b, phi, mu, v_warm, solver, row_ptr, col_idx, n_nodes, c_node, R, fwd, bwd, mu2)


def rollout(scene, solver, x0, v0, params, steps, checkpoint_every=10, fwd_opts=None, bwd_opts=None,
            record=None):
    """Differentiable rollout of ``steps`` time steps.  ``scene`` provides
    ``assemble(x, v, *params) -> (A_val, b, c_node, R, phi, mu)``, ``row_ptr``,
    ``col_idx``, ``n_nodes`` and ``h``.  Returns the final positions; with
    ``checkpoint_every`` > 0 only segment boundaries are kept for backward."""

    def one_step(x, v):
        A_val, b, c_node, R, phi, mu = scene.assemble(x, v, *params)
        vn, lam, st = vfpi_solve(solver, A_val, b, phi, mu, v.reshape(-1), scene.row_ptr, scene.col_idx,
                                 scene.n_nodes, c_node, R, fwd_opts, bwd_opts)
        if record is not None:
            record.append(st)
        vn = vn.view(-1, 3)
        return x + scene.h * vn, vn

    def segment(x, v, n):
        for _ in range(n):
            x, v = one_step(x, v)
        return x, v

    x, v = x0, v0
    k = 0
    while k < steps:
        n = min(checkpoint_every if checkpoint_every > 0 else steps, steps - k)
        if checkpoint_every > 0 and torch.is_grad_enabled():
            x, v = checkpoint(segment, x, v, n, use_reentrant=False)
        else:
            x, v = segment(x, v, n)
        k += n
    return x, v
