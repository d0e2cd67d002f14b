"""V-FPI step as a differentiable PyTorch operation, and a checkpointed rollout.

``vfpi_solve`` runs ``vfpi_step`` (FP64, to tolerance) in the forward pass and
``vfpi_step_backward`` (the hand-written adjoint of the converged step, with
the active branch of every contact's projection) in the backward pass;
gradients flow to A's values, b, phi, mu and (anisotropic friction) mu2.  The warm start carries no
gradient (the converged solution does not depend on it).  Contacts are
S-contacts (one block R at node i) or, where ``c_node_j`` >= 0, D-contacts
between nodes i and j (blocks R and -R, eq. jcnode).

Implicit differentiation is valid only at the fixed point (the consistency
remark of Sec. III-B with the adjoint of Sec. IV): a forward or backward solve
that stopped at max_iters, or that the library skipped because of a data
error (its stats.status bits), raises ``VfpiError`` instead of producing a
gradient.  In a rollout the forward status bits are accumulated on the device
and checked once after the loop; every backward call checks its own status
and that of the forward it differentiates.

``rollout`` advances x_{k+1} = x_k + h v_{k+1} with a caller-supplied
differentiable ``assemble(x, v, *params)`` and keeps only every
``checkpoint_every``-th state: in the backward pass each segment is
recomputed (forward again, new tapes) and then differentiated.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from . import _abi
from .solver import Bsr, Contacts, Solver


class ConvergenceError(_abi.VfpiError):
    """A differentiated solve did not reach its fixed point (or was skipped)."""

    def __init__(self, status: int, where: str):
        RuntimeError.__init__(self, f"{where}: {describe_status(status)} (status {status:#x}); the implicit "
                                    f"gradient is defined only at a converged step")
        self.code = status


_STATUS_NAMES = ((_abi.VFPI_S_MAXITER, "stopped at max_iters before theta < tol"),
                 (_abi.VFPI_S_NONFINITE, "non-finite input"), (_abi.VFPI_S_NOT_NODAL, "J_c row not nodal"),
                 (_abi.VFPI_S_NOT_ORTHONORMAL, "R not orthonormal"),
                 (_abi.VFPI_S_SHARED_NODE, "two contacts on one node"),
                 (_abi.VFPI_S_NONPOS_DIAG, "non-positive diagonal of A"),
                 (_abi.VFPI_S_BAD_PATTERN, "column index out of range"), (_abi.VFPI_S_BAD_W, "invalid user W"),
                 (_abi.VFPI_S_BAD_MU, "negative friction coefficient"))


def describe_status(status: int) -> str:
    names = [s for bit, s in _STATUS_NAMES if status & bit]
    return "; ".join(names) if names else "ok"


def _status_word(stats: torch.Tensor) -> torch.Tensor:
    """The status field (int32 at byte offset 4) of a device vfpi_stats record."""
    return stats[4:8].view(torch.int32)


class StatusGuard:
    """Device-side OR of the status bits of many solves, read back once."""

    def __init__(self, device):
        self.bits = torch.zeros(1, dtype=torch.int32, device=device)

    def add(self, stats: torch.Tensor):
        self.bits.bitwise_or_(_status_word(stats))

    def check(self, where: str):
        s = int(self.bits.item())
        if s:
            raise ConvergenceError(s, where)


def _jc_rows(c_node, c_node_j, R):
    """Block rows of J_c: [R] at node i for an S-contact, [R, -R] at nodes i, j
    for a D-contact (c_node_j >= 0), in contact order."""
    nc = int(c_node.numel())
    dev = c_node.device
    if c_node_j is None:
        return torch.arange(nc + 1, dtype=torch.int32, device=dev), c_node.contiguous(), R.contiguous()
    d = (c_node_j >= 0)
    cnt = 1 + d.to(torch.int32)
    row_ptr = torch.zeros(nc + 1, dtype=torch.int32, device=dev)
    row_ptr[1:] = torch.cumsum(cnt, 0)
    nnzb = int(row_ptr[-1].item())
    first = row_ptr[:-1].long()
    col = torch.empty(nnzb, dtype=torch.int32, device=dev)
    val = torch.empty(nnzb, 3, 3, dtype=R.dtype, device=dev)
    col[first] = c_node.to(torch.int32)
    val[first] = R
    dj = torch.nonzero(d).squeeze(1)
    col[first[dj] + 1] = c_node_j[dj].to(torch.int32)
    val[first[dj] + 1] = -R[dj]
    return row_ptr, col, val


class VfpiStepFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A_val, b, phi, mu, v_warm, solver: Solver, row_ptr, col_idx, n_nodes, c_node, R, fwd_opts,
                bwd_opts, mu2=None, c_node_j=None, guard=None, record=None):
        nc = int(c_node.numel())
        A = Bsr(n_nodes, row_ptr, col_idx, A_val.detach().contiguous())
        crp, ccol, cval = _jc_rows(c_node, c_node_j, R.detach())
        Jc = Contacts(nc, crp, ccol, cval.contiguous(), phi.detach().contiguous(), mu.detach().contiguous(),
                      None if mu2 is None else mu2.detach().contiguous())
        v = v_warm.detach().clone().contiguous()
        tape = solver.tape(n_nodes, nc)
        lam, stats = solver.step(A, b.detach().contiguous(), Jc, v, tape=tape, **fwd_opts)
        if guard is None:
            s = int(_status_word(stats).item())
            if s:
                raise ConvergenceError(s, "vfpi_solve forward")
        else:
            guard.add(stats)
        if record is not None:
            off = 48 * n_nodes + 24 * nc  # tape layout: w, v (3N doubles each), lambda* (3 n_c), branch (n_c)
            record.append((stats, tape[off:off + 4 * nc].view(torch.int32).clone()))
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
        tape, fstats = ctx.saved_tensors
        n = 3 * ctx.A.n_nodes
        gv = torch.zeros(n, dtype=torch.float64, device=tape.device) if gv is None else gv.contiguous()
        gl = None if glam is None else glam.contiguous()
        g = ctx.solver.step_backward(ctx.A, ctx.Jc, tape, gv, gl, want_A=ctx.need_A, **ctx.bwd_opts)
        # one read-back per backward call: the forward this gradient belongs to
        # and the adjoint solve itself must both have converged
        fs, bs = torch.cat([_status_word(fstats), _status_word(g["stats"])]).tolist()
        if fs:
            raise ConvergenceError(fs, "vfpi_solve forward (differentiated)")
        if bs:
            raise ConvergenceError(bs, "vfpi_step_backward")
        gA = g["A"].view(-1, 3, 3) if ctx.need_A else None
        return (gA, g["b"], g["phi"], g["mu"], None, None, None, None, None, None, None, None, None, g.get("mu2"),
                None, None, None)


DEFAULT_FWD = dict(max_iters=100000, tol=1e-13)
DEFAULT_BWD = dict(max_iters=100000, tol=1e-13)


def vfpi_solve(solver, A_val, b, phi, mu, v_warm, row_ptr, col_idx, n_nodes, c_node, R, fwd_opts=None,
               bwd_opts=None, mu2=None, c_node_j=None, guard=None, record=None):
    """Differentiable V-FPI step; returns (v, lambda, stats tensor).  The
    backward pass uses the forward's contact regularization (omega) and
    projection operator.  ``mu2`` (optional) is the second friction
    coefficient of anisotropic friction; it receives a gradient too.
    ``c_node_j`` (optional, -1 for S-contacts) makes contact m a D-contact
    between nodes c_node[m] and c_node_j[m].  Without ``guard`` the forward's
    status is checked at once (one device read); with a ``StatusGuard`` it is
    accumulated there for the caller to check.  ``record`` (a list) receives
    (stats, per-contact branch) of the forward."""
    fwd = dict(fwd_opts or DEFAULT_FWD)
    if fwd.get("w_mode") in ("bb1", "bb2"):
        raise ValueError("vfpi_solve: Barzilai-Borwein steps are not differentiated (their last alpha need not "
                         "make the adjoint iteration contract); use a Frobenius, diagonal or scalar W")
    if fwd.get("fixed_iters"):
        raise ValueError("vfpi_solve: fixed_iters stops before the fixed point; give max_iters and tol")
    bwd = dict(bwd_opts or DEFAULT_BWD)
    bwd["omega"] = fwd.get("omega", 0.0)
    bwd["projection"] = fwd.get("projection", "strict")
    return VfpiStepFn.apply(A_val, b, phi, mu, v_warm, solver, row_ptr, col_idx, n_nodes, c_node, R, fwd, bwd, mu2,
                            c_node_j, guard, record)


def rollout(scene, solver, x0, v0, params, steps, checkpoint_every=10, fwd_opts=None, bwd_opts=None,
            record=None):
    """Differentiable rollout of ``steps`` time steps.  ``scene`` provides
    ``assemble(x, v, *params) -> (A_val, b, c_node, R, phi, mu)``, ``row_ptr``,
    ``col_idx``, ``n_nodes`` and ``h``.  Returns the final positions; with
    ``checkpoint_every`` > 0 only segment boundaries are kept for backward.
    Raises ``ConvergenceError`` after the loop if any step's solve did not
    converge.  ``record`` (a list) receives (stats, branch) per step."""
    guard = StatusGuard(x0.device)

    def one_step(x, v):
        A_val, b, c_node, R, phi, mu = scene.assemble(x, v, *params)
        vn, lam, st = vfpi_solve(solver, A_val, b, phi, mu, v.reshape(-1), scene.row_ptr, scene.col_idx,
                                 scene.n_nodes, c_node, R, fwd_opts, bwd_opts, guard=guard, record=record)
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
    guard.check("rollout forward")
    return x, v
