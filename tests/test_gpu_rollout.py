"""Differentiable rollouts through the HIP adjoint (torch.autograd.Function +
segment checkpointing): gradients w.r.t. the spring stiffness k, per-node
friction mu and initial velocities vs central finite differences of the HIP
forward (bar 1e-4 relative), vs the FP64 oracle's own gradient of the same
rollout (small cloth and the full 64x64 cloth), the sliding particle's closed
form, and the refusal to differentiate a solve that did not converge.

A finite-difference direction is discarded (and counted) when the +eps and
-eps rollouts take a different branch at any contact of any step: the loss is
only piecewise smooth, and its derivative across a branch change is not the
adjoint's."""
import numpy as np
import pytest
import torch

import oracle
import paper_2201_09212_amd as vf
import scenes
from oracle.adjoint import adjoint as oracle_adjoint
from paper_2201_09212_amd.autograd import rollout
from scenes.cloth_torch import TorchCloth
from tests.gpu_util import gate, say

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _setup(side, steps, seed=0, drop=0.01):
    sc, x0, v0 = scenes.cloth_cfg5_scene(seed, side=side)
    x0[:, 2] = drop
    tc = TorchCloth(sc, DEV)
    s = vf.Solver(sc.n_nodes, tc.nnzb, sc.n_nodes)
    g = np.random.default_rng(seed + 100)
    target = torch.as_tensor(x0 + g.normal(0, 0.01, size=x0.shape), device=DEV)
    return sc, tc, s, torch.as_tensor(x0, device=DEV), torch.as_tensor(v0, device=DEV), target


def _loss(tc, s, x0, v0, k, mu, target, steps, every=10, record=None):
    xN, _ = rollout(tc, s, x0, v0, (k, mu), steps, checkpoint_every=every, record=record)
    return ((xN - target) ** 2).sum()


def _counts(record):
    return [tuple(vf.read_stats(st)[0][f] for f in ("n_open", "n_stick", "n_slip")) for st, _ in record]


def _same_branches(ra, rb):
    """True when two rollouts took the same branch at every contact of every step."""
    if len(ra) != len(rb):
        return False
    return all(a.shape == b.shape and torch.equal(a, b) for (_, a), (_, b) in zip(ra, rb))


def test_rollout_gradients_vs_central_differences():
    side, steps = 10, 30
    sc, tc, s, x0, v0, target = _setup(side, steps)
    k = torch.tensor(1e3, device=DEV, dtype=torch.float64, requires_grad=True)
    mu = torch.full((sc.n_nodes,), 0.5, device=DEV, dtype=torch.float64, requires_grad=True)
    v0r = v0.clone().requires_grad_(True)
    L = _loss(tc, s, x0, v0r, k, mu, target, steps)
    L.backward()
    grads = {"k": k.grad.item(), "mu": mu.grad.cpu().numpy(), "v0": v0r.grad.cpu().numpy()}
    eps = 1e-6
    checked = discarded = 0

    def fd(perturb):
        rp, rm = [], []
        with torch.no_grad():
            lp = _loss(tc, s, x0, *perturb(+eps), target, steps, record=rp).item()
            lm = _loss(tc, s, x0, *perturb(-eps), target, steps, record=rm).item()
        return (lp - lm) / (2 * eps), _same_branches(rp, rm)

    def check(name, val, exact):
        nonlocal checked, discarded
        num, same = val
        if not same:
            discarded += 1
            return
        assert abs(num - exact) <= 1e-4 * max(abs(num), 1e-3), (name, num, exact)
        checked += 1

    kd = k.detach()
    check("k", fd(lambda e: (v0, kd * (1 + e), mu.detach())), grads["k"] * kd.item())
    mu_nodes = np.argsort(-np.abs(grads["mu"]))[:4]
    for n in mu_nodes:
        def pm(e, n=n):
            m = mu.detach().clone()
            m[n] += e
            return v0, kd, m
        check(f"mu[{n}]", fd(pm), grads["mu"][n])
    for n in (3, 57):
        for c in (0, 2):
            def pv(e, n=n, c=c):
                vv = v0.clone()
                vv[n, c] += e
                return vv, kd, mu.detach()
            check(f"v0[{n},{c}]", fd(pv), grads["v0"][n, c])
    say(f"  rollout FD: {checked} directions checked, {discarded} discarded (active set changed)")
    assert checked >= 5


def test_checkpointing_does_not_change_gradients():
    side, steps = 8, 25
    sc, tc, s, x0, v0, target = _setup(side, steps, seed=1)
    out = []
    for every in (0, 10, 7):
        k = torch.tensor(1e3, device=DEV, dtype=torch.float64, requires_grad=True)
        mu = torch.full((sc.n_nodes,), 0.5, device=DEV, dtype=torch.float64, requires_grad=True)
        _loss(tc, s, x0, v0, k, mu, target, steps, every=every).backward()
        out.append((k.grad.item(), mu.grad.cpu().numpy()))
    for kg, mg in out[1:]:
        assert kg == out[0][0] and np.array_equal(mg, out[0][1])


class _OracleStepFn(torch.autograd.Function):
    """The same step solved and differentiated by the CPU FP64 oracle."""

    @staticmethod
    def forward(ctx, A_val, b, phi, mu, v_warm, row_ptr, col_idx, n_nodes, c_node, R):
        p = scenes.Problem(n_nodes=n_nodes, row_ptr=row_ptr, col_idx=col_idx, val=A_val.detach().numpy(),
                           b=b.detach().numpy(), v0=v_warm.detach().numpy(), c_node=c_node,
                           c_node_j=np.full(len(c_node), -1), R=R.detach().numpy(), phi=phi.detach().numpy(),
                           mu=mu.detach().numpy())
        f = oracle.vfpi(p, max_iters=200000, tol=1e-13)
        ctx.p, ctx.f = p, f
        return torch.as_tensor(f["v"]), torch.as_tensor(f["lam"].ravel())

    @staticmethod
    def backward(ctx, gv, glam):
        a = oracle_adjoint(ctx.p, ctx.f, gv.numpy(), None if glam is None else glam.numpy(), tol=1e-14)
        return (torch.as_tensor(a["A"]), torch.as_tensor(a["b"]), torch.as_tensor(a["phi"]),
                torch.as_tensor(a["mu"]), None, None, None, None, None, None)


def _rollout_grads(backend, sc, x0, v0, target, steps, mu0, every):
    """dL/dk, dL/dmu, dL/dv0 of the rollout loss, with the GPU step (through
    the checkpointed rollout) or the oracle step; also the contacts per step."""
    dev = DEV if backend == "gpu" else torch.device("cpu")
    tc = TorchCloth(sc, dev)
    k = torch.tensor(1e3, device=dev, dtype=torch.float64, requires_grad=True)
    mu = torch.full((sc.n_nodes,), mu0, device=dev, dtype=torch.float64, requires_grad=True)
    x = torch.as_tensor(x0, device=dev)
    v = torch.as_tensor(v0, device=dev).requires_grad_(True)
    v_init = v
    ncs = []
    if backend == "gpu":
        s = vf.Solver(sc.n_nodes, tc.nnzb, sc.n_nodes)
        rec = []
        xN, _ = rollout(tc, s, x, v, (k, mu), steps, checkpoint_every=every, record=rec)
        ncs = [int(b.numel()) for _, b in rec[:steps]]
    else:
        rp, ci = sc.row_ptr, sc.col_idx
        for _ in range(steps):
            A_val, b, cn, R, phi, mm = tc.assemble(x, v, k, mu)
            ncs.append(int(cn.numel()))
            vn, _ = _OracleStepFn.apply(A_val, b, phi, mm, v.reshape(-1), rp, ci, sc.n_nodes, cn.numpy(), R)
            v = vn.view(-1, 3)
            x = x + sc.h * v
        xN = x
    L = ((xN - torch.as_tensor(target, device=dev)) ** 2).sum()
    L.backward()
    return k.grad.item(), mu.grad.cpu().numpy(), v_init.grad.cpu().numpy(), ncs


def test_rollout_gradient_matches_oracle_rollout_gradient():
    side, steps = 8, 20
    sc, x0, v0 = scenes.cloth_cfg5_scene(2, side=side)
    x0[:, 2] = 0.006
    target = x0 + np.random.default_rng(5).normal(0, 0.01, size=x0.shape)
    (kg, mg, vg, _), (ko, mo, vo, _) = (_rollout_grads(b, sc, x0, v0, target, steps, 0.4, 5)
                                        for b in ("gpu", "oracle"))
    say(f"  rollout gradient gpu vs oracle: k {kg:.6e} / {ko:.6e}")
    gate([kg], [ko], 1e-6, "dL/dk")
    gate(mg, mo, 1e-6, "dL/dmu")
    gate(vg, vo, 1e-6, "dL/dv0")


class _Particle:
    """One particle on an inclined plane (normal (sin a, 0, cos a))."""

    def __init__(self, alpha, mass, h, g):
        self.a, self.m, self.h, self.g = alpha, mass, h, g
        self.row_ptr = torch.tensor([0, 1], dtype=torch.int32, device=DEV)
        self.col_idx = torch.tensor([0], dtype=torch.int32, device=DEV)
        self.n_nodes = 1
        nrm = np.array([[np.sin(alpha), 0.0, np.cos(alpha)]])
        self.n = torch.as_tensor(nrm[0], device=DEV)
        self.R = torch.as_tensor(scenes.onb_duff(nrm), device=DEV)

    def assemble(self, x, v, mu):
        A = (self.m * torch.eye(3, device=DEV, dtype=torch.float64))[None]
        b = (self.m * (v + self.h * torch.tensor([0.0, 0.0, -self.g], device=DEV, dtype=torch.float64))).reshape(-1)
        phi = (x[0] @ self.n / self.h).reshape(1)
        return A, b, torch.tensor([0], dtype=torch.int32, device=DEV), self.R, phi, mu.reshape(1)


def test_sliding_particle_closed_form_through_autograd():
    a, mu0, m, h, g, N = 0.5, 0.2, 1.3, 0.01, 9.81, 20
    sc = _Particle(a, m, h, g)
    s = vf.Solver(1, 1, 1)
    mu = torch.tensor(mu0, device=DEV, dtype=torch.float64, requires_grad=True)
    x0 = torch.zeros(1, 3, device=DEV, dtype=torch.float64)
    v0 = torch.zeros(1, 3, device=DEV, dtype=torch.float64)
    xN, _ = rollout(sc, s, x0, v0, (mu,), N, checkpoint_every=6)
    t_dir = torch.tensor([np.cos(a), 0.0, -np.sin(a)], device=DEV, dtype=torch.float64)
    L = xN[0] @ t_dir
    L.backward()
    np.testing.assert_allclose(L.item(), h * h * g * (np.sin(a) - mu0 * np.cos(a)) * N * (N + 1) / 2, rtol=1e-12)
    np.testing.assert_allclose(mu.grad.item(), -h * h * g * np.cos(a) * N * (N + 1) / 2, rtol=1e-10)


def _fd_check(name, fd_fn, exact, eps_list, log):
    """Central difference along one direction, retried with smaller steps
    while the +/- rollouts change a branch.  Returns True when checked."""
    for eps in eps_list:
        num, same = fd_fn(eps)
        if same:
            ok = abs(num - exact) <= 1e-4 * abs(num) + 1e-9
            log.append(f"{name}: fd {num:.8e} adjoint {exact:.8e} (eps {eps:g})")
            assert ok, (name, num, exact, eps)
            return True
    log.append(f"{name}: discarded (branch change at every eps)")
    return False


def test_cloth64_100_steps_full_size():
    """The full adjoint workload: 64x64 cloth dropped 2 cm onto the plane,
    100 steps, checkpoints every 10, loss = squared distance of the final
    positions to a seeded target.  dL/dk, 16 candidate dL/dmu entries and 16
    candidate dL/dv0 entries (the largest of each) against central
    differences of the HIP forward; k must be checked, and at least 8 mu and
    8 v0 entries."""
    steps = 100
    sc, tc, s, x0, v0, target = _setup(64, steps, seed=0, drop=0.02)
    k = torch.tensor(1e3, device=DEV, dtype=torch.float64, requires_grad=True)
    mu = torch.full((sc.n_nodes,), 0.5, device=DEV, dtype=torch.float64, requires_grad=True)
    v0r = v0.clone().requires_grad_(True)
    rec = []
    L = _loss(tc, s, x0, v0r, k, mu, target, steps, record=rec)
    L.backward()
    nc = [sum(c) for c in _counts(rec[:steps])]
    gk, gmu, gv0 = k.grad.item(), mu.grad.cpu().numpy(), v0r.grad.cpu().numpy()
    say(f"  cloth64: loss {L.item():.6e}, contacts at steps 0/50/99: {nc[0]}/{nc[50]}/{nc[99]}, "
        f"dL/dk {gk:.4e}, |dL/dmu| {np.linalg.norm(gmu):.4e}, |dL/dv0| {np.linalg.norm(gv0):.4e}")
    kd, mud = k.detach(), mu.detach()

    def run(kk, mm, vv):
        r = []
        with torch.no_grad():
            val = _loss(tc, s, x0, vv, kk, mm, target, steps, record=r).item()
        return val, r

    def fd_k(eps):
        (lp, rp), (lm, rm) = run(kd * (1 + eps), mud, v0), run(kd * (1 - eps), mud, v0)
        return (lp - lm) / (2 * eps), _same_branches(rp, rm)

    def fd_mu(n):
        def f(eps):
            mp, mm = mud.clone(), mud.clone()
            mp[n] += eps
            mm[n] -= eps
            (lp, rp), (lm, rm) = run(kd, mp, v0), run(kd, mm, v0)
            return (lp - lm) / (2 * eps), _same_branches(rp, rm)
        return f

    def fd_v0(n, c):
        def f(eps):
            vp, vm = v0.clone(), v0.clone()
            vp[n, c] += eps
            vm[n, c] -= eps
            (lp, rp), (lm, rm) = run(kd, mud, vp), run(kd, mud, vm)
            return (lp - lm) / (2 * eps), _same_branches(rp, rm)
        return f

    log = []
    eps_list = (1e-6, 3e-7, 1e-7)
    k_ok = _fd_check("k", fd_k, gk * kd.item(), eps_list, log)
    mu_ok = sum(_fd_check(f"mu[{n}]", fd_mu(int(n)), gmu[n], eps_list, log)
                for n in np.argsort(-np.abs(gmu))[:16])
    flat = np.argsort(-np.abs(gv0.ravel()))[:16]
    v_ok = sum(_fd_check(f"v0[{q // 3},{q % 3}]", fd_v0(int(q // 3), int(q % 3)), gv0.ravel()[q], eps_list, log)
               for q in flat)
    for line in log:
        say("   " + line)
    say(f"  cloth64 FD: k {'checked' if k_ok else 'discarded'}, mu {mu_ok}/16 checked, v0 {v_ok}/16 checked "
        f"({16 - mu_ok + 16 - v_ok + (not k_ok)} discarded)")
    assert k_ok and mu_ok >= 8 and v_ok >= 8


def test_cloth64_rollout_gradient_matches_oracle_rollout_gradient():
    """The same 64x64 drop as the full adjoint workload over its first 20
    steps (contacts appear): the GPU rollout gradient (k, every mu, every
    v0) equals the FP64 oracle's own rollout gradient element by element."""
    steps = 20
    sc, x0, v0 = scenes.cloth_cfg5_scene(0, side=64)
    x0[:, 2] = 0.02
    target = x0 + np.random.default_rng(100).normal(0, 0.01, size=x0.shape)
    grads = []
    for backend in ("gpu", "oracle"):
        grads.append(_rollout_grads(backend, sc, x0, v0, target, steps, mu0=0.5, every=10))
    (kg, mg, vg, ncg), (ko, mo, vo, nco) = grads
    say(f"  cloth64 x {steps} steps, contacts per step gpu {ncg} oracle {nco}; dL/dk gpu {kg:.8e} oracle {ko:.8e}")
    assert ncg == nco and max(ncg) > 100
    gate([kg], [ko], 1e-6, "dL/dk")
    gate(mg, mo, 1e-6, "dL/dmu")
    gate(vg, vo, 1e-6, "dL/dv0")


def test_unconverged_forward_is_not_differentiated():
    """A forward that stops at max_iters (tol out of reach) raises instead of
    handing an adjoint of a non-fixed point to autograd, in a rollout and in
    a single vfpi_solve; so does a backward that stops at max_iters."""
    from paper_2201_09212_amd.autograd import ConvergenceError, vfpi_solve
    sc, tc, s, x0, v0, target = _setup(8, 3, seed=3, drop=0.003)
    k = torch.tensor(1e3, device=DEV, dtype=torch.float64, requires_grad=True)
    mu = torch.full((sc.n_nodes,), 0.5, device=DEV, dtype=torch.float64, requires_grad=True)
    with pytest.raises(ConvergenceError, match="max_iters"):
        rollout(tc, s, x0, v0, (k, mu), 3, fwd_opts=dict(max_iters=5, tol=1e-13))
    A_val, b, c_node, R, phi, mm = tc.assemble(x0, v0, k, mu)
    assert c_node.numel() > 0
    with pytest.raises(ConvergenceError, match="max_iters"):
        vfpi_solve(s, A_val, b, phi, mm, v0.reshape(-1), tc.row_ptr, tc.col_idx, tc.n_nodes, c_node, R,
                   fwd_opts=dict(max_iters=5, tol=1e-13))
    v, lam, st = vfpi_solve(s, A_val, b, phi, mm, v0.reshape(-1), tc.row_ptr, tc.col_idx, tc.n_nodes, c_node, R,
                            bwd_opts=dict(max_iters=3, tol=1e-13))
    with pytest.raises(ConvergenceError, match="vfpi_step_backward"):
        ((v - 1.0) ** 2).sum().backward()
    with pytest.raises(ValueError, match="Barzilai"):
        vfpi_solve(s, A_val, b, phi, mm, v0.reshape(-1), tc.row_ptr, tc.col_idx, tc.n_nodes, c_node, R,
                   fwd_opts=dict(max_iters=1000, tol=1e-10, w_mode="bb1"))
