"""Virtual nodes on the GPU: the eq. vnode system built by the library
(vfpi_vnode_pattern + vfpi_vnode_values) against the oracle's, the V-FPI
solve of it against the oracle (1e-9 at a fixed sweep count), and Prop. 2:
the sliding box's error against its closed form falls like 1 / k_v."""
import numpy as np
import pytest
import torch

import oracle
import paper_2201_09212_amd as vf
import scenes
from oracle.vnode import augment, augmented_matrix
from paper_2201_09212_amd import _abi
from tests.gpu_util import gate, say

pytestmark = pytest.mark.gpu


def _gpu_system(vs, k_v):
    dev = torch.device("cuda", 0)
    A_o = vf.bsr_from_arrays(vs.n_o, vs.row_ptr, vs.col_idx, vs.val, device=dev)
    b_o = torch.as_tensor(vs.b, device=dev)
    v_o = torch.as_tensor(vs.v0, device=dev)
    A, b, v = vf.vnode_augment(A_o, b_o, v_o, torch.as_tensor(vs.jv_ptr), torch.as_tensor(vs.jv_col),
                               torch.as_tensor(vs.jv_val), k_v)
    torch.cuda.synchronize()
    return A, b, v


def _contacts(vs, dev="cuda"):
    p = scenes.Problem(n_nodes=vs.n_o + vs.n_v, row_ptr=np.zeros(vs.n_o + vs.n_v + 1), col_idx=np.zeros(0),
                       val=np.zeros((0, 3, 3)), b=np.zeros(3 * (vs.n_o + vs.n_v)), v0=np.zeros(3 * (vs.n_o + vs.n_v)),
                       c_node=vs.c_node, c_node_j=vs.c_node_j, R=vs.R, phi=vs.phi, mu=vs.mu)
    crp, ccol, cval = p.jc_bsr()
    return vf.contacts_from_arrays(crp, ccol, cval, vs.phi, vs.mu, device=dev)


def _dense(A: vf.Bsr):
    n = A.n_nodes
    rp, ci, val = A.row_ptr.cpu().numpy(), A.col_idx.cpu().numpy(), A.val.cpu().numpy().reshape(-1, 3, 3)
    D = np.zeros((n, 3, n, 3))
    for r in range(n):
        for k in range(rp[r], rp[r + 1]):
            D[r, :, ci[k], :] = val[k]
    return D.reshape(3 * n, 3 * n)


@pytest.mark.parametrize("k_v", [0.5, 1e4])
def test_gpu_system_matches_oracle(k_v):
    for vs in (scenes.rigid_box_on_floor(), scenes.particles_on_cloth(0), scenes.particles_on_cloth(2)):
        A, b, v = _gpu_system(vs, k_v)
        ref = augmented_matrix(vs, k_v).toarray()
        p = augment(vs, k_v)
        err = np.abs(_dense(A) - ref).max() / np.abs(ref).max()
        say(f"  {vs.meta['scene']} k_v={k_v}: {A.nnzb} blocks, max rel err {err:.2e}")
        assert err <= 1e-15
        assert np.array_equal(b.cpu().numpy(), p.b)
        np.testing.assert_allclose(v.cpu().numpy(), p.v0, rtol=0, atol=1e-15 * np.abs(p.v0).max())


@pytest.mark.parametrize("k_v", [0.1, 1.0])
def test_vnode_solve_parity(k_v):
    for seed in (0, 1):
        vs = scenes.particles_on_cloth(seed)
        A, b, v = _gpu_system(vs, k_v)
        Jc = _contacts(vs)
        s = vf.Solver(A.n_nodes, A.nnzb, len(vs.c_node))
        L = 200
        lam, st = s.step(A, b, Jc, v, max_iters=L, fixed_iters=True)
        torch.cuda.synchronize()
        ref = oracle.vfpi(augment(vs, k_v), max_iters=L, fixed_iters=True)
        ev = gate(v.cpu().numpy(), ref["v"], 1e-9, "v")
        el = gate(lam.cpu().numpy(), ref["lam"], 1e-9, "lambda")
        say(f"  particles_on_cloth({seed}) k_v={k_v} L={L}: rel_v={ev:.2e} rel_lam={el:.2e}")


def test_prop2_box_trend_on_gpu():
    vs = scenes.rigid_box_on_floor()
    m, h, g, mu, F = (vs.meta[k] for k in ("mass", "h", "g", "mu", "force"))
    exact = np.array([0.0, h * (F[1] / m - mu * g), 0.0, 0.0, 0.0, 0.0])
    Jc = _contacts(vs)
    errs = []
    for k_v in (10.0, 100.0, 1000.0):
        A, b, v = _gpu_system(vs, k_v)
        s = vf.Solver(A.n_nodes, A.nnzb, len(vs.c_node))
        lam, st = s.step(A, b, Jc, v, max_iters=2_000_000, tol=1e-14, cheby_ls=10)
        torch.cuda.synchronize()
        stt = vf.read_stats(st)[0]
        errs.append(np.abs(v.cpu().numpy()[:6] - exact).max())
        say(f"  box k_v={k_v}: {stt['iters']} sweeps, status {stt['status']}, error {errs[-1]:.3e}")
        assert stt["status"] == _abi.VFPI_S_CONVERGED
    r = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(r > 7) and np.all(r < 13), (errs, r)
