"""Batched FP32 HIP path (FP64 residual) vs the FP64 oracle per environment:
bar 1e-4 relative, element by element, on v and lambda at a fixed sweep count, for every kernel
variant, work-queue order and a sample of the full 2048-environment batch."""
import numpy as np
import pytest
import torch

import oracle
import paper_2201_09212_amd as vf
import scenes
from paper_2201_09212_amd import _abi
from tests.gpu_util import gate, say

pytestmark = pytest.mark.gpu
TOL = 1e-4

VARIANTS = {"node1": 1 | (1 << 8), "node2": 1 | (2 << 8), "node4": 1 | (4 << 8), "node8": 1 | (8 << 8),
            "row1": 2 | (1 << 8), "row2": 2 | (2 << 8), "node4_3wg": 1 | (4 << 8) | (3 << 16),
            "node4_occ4": 3 | (4 << 8), "node8_occ4": 3 | (8 << 8),
            "lds16": 4 | (16 << 8), "lds8_regs": 4 | (8 << 8), "lds8_regs_u4": 4 | (8 << 8) | (1 << 26)}
LDS_VARIANTS = [4 | (16 << 8), 4 | (8 << 8)]


def _envs_small():
    envs = [sc.assemble(x, v) for sc, x, v in scenes.cloth_cfg4_envs(7, n_env=14, smin=3, smax=20)]
    envs += [scenes.random_problem(n, nc, 100 + n, degree=4.0, phi_scale=0.3)
             for n, nc in [(1, 1), (2, 0), (65, 40), (130, 130)]]
    return envs


def _upload_batch(batch, dev):
    p = batch.problem
    A = vf.bsr_from_arrays(p.n_nodes, p.row_ptr, p.col_idx, p.val, dtype=torch.float32, device=dev)
    crp, ccol, cval = p.jc_bsr()
    Jc = vf.contacts_from_arrays(crp, ccol, cval, p.phi, p.mu, dtype=torch.float32, device=dev, mu2=p.mu2)
    b = torch.as_tensor(p.b, device=dev).float()
    v = torch.as_tensor(p.v0, device=dev).float()
    no = torch.as_tensor(batch.env_node_off, device=dev)
    co = torch.as_tensor(batch.env_con_off, device=dev)
    return A, Jc, b, v, no, co


def run_batched(batch, order=None, **opt):
    dev = torch.device("cuda", 0)
    p = batch.problem
    s = vf.Solver(p.n_nodes, p.nnzb, max(p.n_contacts, 1), batch.n_env)
    A, Jc, b, v, no, co = _upload_batch(batch, dev)
    eo = None if order is None else torch.as_tensor(np.asarray(order, np.int32), device=dev)
    lam, st = s.step_batched(batch.n_env, no, co, A, b, Jc, v, env_order=eo, **opt)
    torch.cuda.synchronize()
    return v.cpu().numpy().astype(np.float64), lam.cpu().numpy().astype(np.float64), vf.read_stats(st)


def _check_envs(batch, v, lam, stats, L, envs_idx=None, **okw):
    worst = 0.0
    idx = range(batch.n_env) if envs_idx is None else envs_idx
    for e in idx:
        pe = batch.envs[e]
        ref = oracle.vfpi(pe, max_iters=L, fixed_iters=True, **okw)
        n0, n1 = batch.env_node_off[e], batch.env_node_off[e + 1]
        m0, m1 = batch.env_con_off[e], batch.env_con_off[e + 1]
        assert stats[e]["iters"] == L and stats[e]["status"] == _abi.VFPI_S_MAXITER, (e, stats[e])
        ev = gate(v[3 * n0:3 * n1], ref["v"], TOL, f"env {e} (N={pe.n_nodes}) v")
        el = gate(lam[3 * m0:3 * m1], ref["lam"], TOL, f"env {e} (nc={pe.n_contacts}) lambda")
        worst = max(worst, ev, el)
    return worst


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_batched_parity_variants(variant):
    envs = _envs_small()
    batch = scenes.concat_problems(envs)
    L = 30
    v, lam, st = run_batched(batch, max_iters=L, fixed_iters=True, variant=VARIANTS[variant])
    worst = _check_envs(batch, v, lam, st, L)
    say(f"  batched {variant}: {batch.n_env} envs, worst rel err {worst:.2e}")


def test_batched_order_and_scalar_w():
    envs = _envs_small()
    batch = scenes.concat_problems(envs)
    order = np.argsort([-e.nnzb for e in envs]).astype(np.int32)
    v, lam, st = run_batched(batch, order=order, max_iters=20, fixed_iters=True, variant=1 | (4 << 8))
    _check_envs(batch, v, lam, st, 20)
    alpha = float(np.float32(0.9 * min(oracle.core.gershgorin_alpha(oracle.system_matrix(e)) for e in envs)))
    v, lam, st = run_batched(batch, max_iters=20, fixed_iters=True, w_mode="scalar", alpha=alpha)
    _check_envs(batch, v, lam, st, 20, w_mode="scalar", alpha_user=alpha)


def test_batched_per_env_convergence():
    envs = _envs_small()
    batch = scenes.concat_problems(envs)
    v, lam, st = run_batched(batch, max_iters=5000, tol=3e-5)
    for e, pe in enumerate(envs):
        ref = oracle.vfpi(pe, max_iters=5000, tol=3e-5)
        assert st[e]["status"] == _abi.VFPI_S_CONVERGED and st[e]["theta"] < 3e-5, (e, st[e])
        n0, n1 = batch.env_node_off[e], batch.env_node_off[e + 1]
        gate(v[3 * n0:3 * n1], ref["v"], 1e-3, f"env {e} converged v")
    iters = [s["iters"] for s in st]
    say(f"  per-env sweeps: min {min(iters)} max {max(iters)}")
    assert len(set(iters)) > 1  # environments stop on their own residual


def test_batched_bad_env_isolated():
    envs = _envs_small()
    k = len(envs) - 2  # the random environment with 40 contacts
    bad = envs[k]
    envs[k] = scenes.Problem(**{**bad.__dict__, "c_node": np.array([bad.c_node[0]] * 2 + list(bad.c_node[2:]))})
    batch = scenes.concat_problems(envs)
    v, lam, st = run_batched(batch, max_iters=10, fixed_iters=True)
    assert st[k]["status"] & _abi.VFPI_S_SHARED_NODE and st[k]["iters"] == 0
    assert np.all(lam[3 * batch.env_con_off[k]:3 * batch.env_con_off[k + 1]] == 0)
    good = [e for e in range(len(envs)) if e != k]
    _check_envs(batch, v, lam, st, 10, envs_idx=good)


@pytest.mark.parametrize("variant", [0, 3 | (8 << 8), 4 | (16 << 8)])
def test_full_batch_sampled(variant):
    envs = [sc.assemble(x, v) for sc, x, v in scenes.cloth_cfg4_envs(0)]
    batch = scenes.concat_problems(envs)
    L = 25
    v, lam, st = run_batched(batch, max_iters=L, fixed_iters=True, variant=variant)
    sample = np.random.default_rng(0).choice(batch.n_env, 40, replace=False)
    sizes = [envs[e].n_nodes for e in sample]
    worst = _check_envs(batch, v, lam, st, L, envs_idx=sample)
    say(f"  full batch: {batch.n_env} envs, {batch.problem.n_nodes} nodes, sample sizes {min(sizes)}-{max(sizes)}, "
        f"worst rel {worst:.2e}")


@pytest.mark.parametrize("variant", LDS_VARIANTS)
def test_lds_kernel_environment_beyond_lds(variant):
    """The LDS-resident kernel holds environments of up to 3,072 nodes; a
    60 x 60 cloth (3,600 nodes) in the same batch runs the global-memory loop
    of the same launch.  Both against the oracle, with and without
    convergence by tolerance."""
    envs = [sc.assemble(x, v) for sc, x, v in scenes.cloth_cfg4_envs(3, n_env=6, smin=20, smax=48)]
    sc, x, v = scenes.cloth_cfg4_envs(4, n_env=1, smin=60, smax=60)[0]
    envs.insert(2, sc.assemble(x, v))
    assert max(e.n_nodes for e in envs) > 3072
    batch = scenes.concat_problems(envs)
    L = 40
    v, lam, st = run_batched(batch, max_iters=L, fixed_iters=True, variant=variant)
    worst = _check_envs(batch, v, lam, st, L)
    for e, pe in enumerate(envs):  # every contact counted once, in one branch
        assert st[e]["n_open"] + st[e]["n_stick"] + st[e]["n_slip"] == pe.n_contacts, (e, st[e])
    v2, lam2, st2 = run_batched(batch, max_iters=5000, tol=3e-5, variant=variant)
    for e, pe in enumerate(envs):
        ref = oracle.vfpi(pe, max_iters=5000, tol=3e-5)
        assert st2[e]["status"] == _abi.VFPI_S_CONVERGED, (e, st2[e])
        n0, n1 = batch.env_node_off[e], batch.env_node_off[e + 1]
        gate(v2[3 * n0:3 * n1], ref["v"], 1e-3, f"env {e} converged v")
    say(f"  lds kernel {variant:#x}: sizes {[e.n_nodes for e in envs]}, worst rel {worst:.2e}")


@pytest.mark.parametrize("variant", [0] + LDS_VARIANTS)
def test_graph_capture_replays_match_eager(variant):
    """The batched step captured in a HIP graph (torch.cuda.CUDAGraph) gives
    the eager result on every replay, with eager work and syncs in between."""
    envs = _envs_small()
    batch = scenes.concat_problems(envs)
    dev = torch.device("cuda", 0)
    p = batch.problem
    s = vf.Solver(p.n_nodes, p.nnzb, max(p.n_contacts, 1), batch.n_env)
    A, Jc, b, v, no, co = _upload_batch(batch, dev)
    v0 = v.clone()
    lam = torch.empty(3 * p.n_contacts, dtype=torch.float32, device=dev)
    st = vf.new_stats(batch.n_env, dev)
    opt = dict(max_iters=15, fixed_iters=True, variant=variant)
    s.step_batched(batch.n_env, no, co, A, b, Jc, v, lam, stats=st, **opt)
    torch.cuda.synchronize()
    ref_v, ref_l = v.clone(), lam.clone()
    g = torch.cuda.CUDAGraph()
    v.copy_(v0)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        s.step_batched(batch.n_env, no, co, A, b, Jc, v, lam, stats=st, **opt)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        s.step_batched(batch.n_env, no, co, A, b, Jc, v, lam, stats=st, **opt)
    for rep in range(4):
        v.copy_(v0)          # eager work between replays
        lam.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(v, ref_v) and torch.equal(lam, ref_l), rep
        assert all(x["iters"] == 15 for x in vf.read_stats(st))
