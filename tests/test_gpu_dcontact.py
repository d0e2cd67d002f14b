"""Node-node (D) contacts on the GPU (eq. jcnode, D case): every launch
variant against the FP64 oracle at fixed sweep counts (1e-9), the batched
FP32 kernel (1e-4 per environment), the two-body closed form, momentum
conservation of the two-sheet collision, and the adjoint (1e-7 vs the oracle
adjoint)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2201_09212_amd as vf
import scenes
from oracle.adjoint import adjoint as oracle_adjoint
from paper_2201_09212_amd import _abi
from tests.gpu_util import fixed_parity, gate, gpu_step, rel, say, upload
from tests.test_gpu_batched import TOL, run_batched

pytestmark = pytest.mark.gpu

VARIANTS = {"grid_node1": 1 | (1 << 8), "grid_node2": 1 | (2 << 8), "grid_node4_cap8": 1 | (4 << 8) | (8 << 16),
            "grid_row1": 2 | (1 << 8), "grid_row2": 2 | (2 << 8), "wg1_node16": 3 | (16 << 8), "wg1_row5": 4,
            "regs1": 5 | (1 << 8), "regs2": 5 | (2 << 8), "regs4": 5 | (4 << 8), "regs8": 5 | (8 << 8)}


def _problems():
    yield "random700_d", scenes.random_problem(700, 300, 4, degree=5.0, phi_scale=0.5, n_d_contacts=120)
    yield "random90_d", scenes.random_problem(90, 40, 2, degree=4.0, phi_scale=0.5, n_d_contacts=40)
    yield "cloth_pair32", scenes.cloth_pair_collision(0, side=32)


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_d_contacts_fixed_sweeps_parity(variant):
    for name, p in _problems():
        L = 40
        ref = oracle.vfpi(p, max_iters=L, fixed_iters=True)
        ev, el, st, ties = fixed_parity(p, ref, L, 1e-9, f"{name} {variant}", variant=VARIANTS[variant])
        say(f"  {name} {variant}: rel_v={ev:.2e} rel_lam={el:.2e} status={st['status']} ties={ties}")
        assert st["n_open"] + st["n_stick"] + st["n_slip"] == p.n_contacts


@pytest.mark.parametrize("opts", [dict(w_mode="scalar", alpha=0.05), dict(projection="proximal"),
                                  dict(omega=0.05), dict(cheby_ls=5, cheby_u=0.9), dict(w_mode="bb1"),
                                  dict(w_mode="bb2")])
def test_d_contacts_with_other_options(opts):
    p = scenes.random_problem(700, 300, 4, degree=5.0, phi_scale=0.5, n_d_contacts=120)
    L = 30
    o = dict(opts)
    if "alpha" in o:
        o["alpha_user"] = o.pop("alpha")
    if "cheby_ls" in o:
        from oracle.chebyshev import vfpi_chebyshev
        ref = vfpi_chebyshev(p, max_iters=L, fixed_iters=True, l_s=o["cheby_ls"], u=o["cheby_u"])
    else:
        ref = oracle.vfpi(p, max_iters=L, fixed_iters=True, **o)
    for var in (0, 1 | (2 << 8), 3 | (16 << 8)):  # 0: the register-resident kernel (BB: its own kernel)
        o2 = dict(opts)
        proj = o2.pop("projection", "strict")
        ev, el, st, ties = fixed_parity(p, ref, L, 1e-9, f"random700_d {opts} {var:#x}", projection=proj,
                                        variant=var, **o2)
        say(f"  random700_d {opts} variant {var:#x}: rel_v={ev:.2e} rel_lam={el:.2e} ties={ties}")


def test_two_body_closed_form_on_gpu():
    from tests.test_oracle_dcontact import _pair_closed_form
    g = np.random.default_rng(5)
    K = 30
    m1, m2 = g.uniform(0.2, 3.0, K), g.uniform(0.2, 3.0, K)
    nrm = g.normal(size=(K, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    mu = g.uniform(0.1, 1.2, K)
    t = np.cross(nrm, g.normal(size=(K, 3)))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    a = g.uniform(0.5, 2.0, K) * np.where(np.arange(K) % 3 == 0, -1.0, 1.0)
    s = np.where(np.arange(K) % 3 == 1, 0.5, 2.0)
    vj = g.normal(size=(K, 3))
    vi = vj - a[:, None] * nrm + (s * mu * np.abs(a))[:, None] * t
    p = scenes.colliding_particle_pairs(m1, m2, nrm, vi, vj, mu)
    v, lam, st, _ = gpu_step(p, max_iters=100000, tol=1e-15)
    err = 0.0
    for k in range(K):
        ei, ej, P, _ = _pair_closed_form(m1[k], m2[k], nrm[k], vi[k], vj[k], mu[k], 0.01, 9.81)
        err = max(err, np.abs(v[6 * k:6 * k + 3] - ei).max(), np.abs(v[6 * k + 3:6 * k + 6] - ej).max(),
                  np.abs(lam[k] - p.R[k] @ P).max())
    say(f"  {K} particle pairs: {st['iters']} sweeps, max error {err:.2e}")
    assert err <= 1e-12


def test_cloth_pair_momentum_and_converged_oracle():
    p = scenes.cloth_pair_collision(1, side=64)
    v, lam, st, _ = gpu_step(p, max_iters=100000, tol=1e-13)
    res = (oracle.system_matrix(p) @ v.ravel() - p.b).reshape(-1, 3).sum(0)
    ref = oracle.vfpi(p, max_iters=100000, tol=1e-13)
    say(f"  cloth_pair64: {p.n_contacts} contacts, {st['iters']} sweeps (oracle {ref['iters']}), "
        f"momentum residual {np.abs(res).max():.2e}, rel_v {rel(v, ref['v']):.2e}")
    assert st["status"] == _abi.VFPI_S_CONVERGED
    assert np.abs(res).max() <= 1e-10 * np.abs(p.b).max()
    gate(v, ref["v"], 1e-9, "pair collision converged v")


def test_batched_d_contacts():
    envs = [scenes.random_problem(n, nc, s, degree=4.0, phi_scale=0.5, n_d_contacts=nd)
            for s, (n, nc, nd) in enumerate([(90, 40, 40), (300, 100, 60), (64, 0, 0), (500, 200, 10), (12, 6, 6)])]
    envs.append(scenes.cloth_pair_collision(2, side=16))
    batch = scenes.concat_problems(envs)
    L = 30
    for var in (1 | (2 << 8), 1 | (8 << 8), 2 | (1 << 8), 4 | (16 << 8), 4 | (8 << 8)):
        v, lam, st = run_batched(batch, max_iters=L, fixed_iters=True, variant=var)
        worst = 0.0
        for e, pe in enumerate(envs):
            ref = oracle.vfpi(pe, max_iters=L, fixed_iters=True)
            n0, n1 = batch.env_node_off[e], batch.env_node_off[e + 1]
            m0, m1 = batch.env_con_off[e], batch.env_con_off[e + 1]
            ev = gate(v[3 * n0:3 * n1], ref["v"], TOL, f"env {e} v")
            el = gate(lam[3 * m0:3 * m1], ref["lam"], TOL, f"env {e} lambda")
            assert st[e]["iters"] == L, (e, st[e])
            worst = max(worst, ev, el)
        say(f"  batched D variant {var:#x}: worst rel {worst:.2e}")
        assert worst <= TOL


@pytest.mark.parametrize("omega", [0.0, 0.1])
def test_adjoint_with_d_contacts(omega):
    p = scenes.random_problem(200, 90, 2, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), tag="adj",
                              n_d_contacts=40)
    g = np.random.default_rng(3)
    gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)
    A, Jc, b, v = upload(p)
    tape = s.tape(p.n_nodes, p.n_contacts)
    lam, st = s.step(A, b, Jc, v, tape=tape, max_iters=200000, tol=1e-14, omega=omega)
    for glt in (None, gl):
        out = s.step_backward(A, Jc, tape, torch.as_tensor(gv, device="cuda"),
                              None if glt is None else torch.as_tensor(glt, device="cuda"), want_A=True,
                              max_iters=200000, tol=1e-13, omega=omega)
        torch.cuda.synchronize()
        fwd = oracle.vfpi(p, max_iters=200000, tol=1e-14, omega=omega)
        ref = oracle_adjoint(p, fwd, gv, glt, tol=1e-14)
        assert vf.read_stats(st)[0]["status"] == _abi.VFPI_S_CONVERGED
        assert vf.read_stats(out["stats"])[0]["status"] == _abi.VFPI_S_CONVERGED
        errs = {k: gate(out[k].cpu().numpy(), ref[k], 1e-7, f"grad {k}") for k in ("b", "A", "phi", "mu")}
        say(f"  D adjoint omega={omega} glam={glt is not None}: {errs}")
        for k, e in errs.items():
            assert e <= 1e-7, (k, e)


@pytest.mark.parametrize("omega", [0.0, 0.1])
def test_autograd_solve_with_d_contacts(omega):
    """vfpi_solve with c_node_j (two-block D rows built in torch) hands A, b,
    phi and mu gradients to PyTorch that equal the oracle adjoint's."""
    from paper_2201_09212_amd.autograd import vfpi_solve
    p = scenes.random_problem(200, 90, 4, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), tag="adj",
                              n_d_contacts=40)
    dev = torch.device("cuda", 0)
    t = {k: torch.tensor(np.asarray(getattr(p, k), dtype=np.float64), device=dev, requires_grad=True)
         for k in ("b", "phi", "mu")}
    A_val = torch.tensor(p.val, device=dev).view(-1, 3, 3).requires_grad_(True)
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)
    g = np.random.default_rng(13)
    gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
    v, lam, st = vfpi_solve(s, A_val, t["b"], t["phi"], t["mu"], torch.as_tensor(p.v0, device=dev),
                            torch.as_tensor(p.row_ptr, device=dev, dtype=torch.int32),
                            torch.as_tensor(p.col_idx, device=dev, dtype=torch.int32), p.n_nodes,
                            torch.as_tensor(p.c_node, device=dev, dtype=torch.int32),
                            torch.as_tensor(p.R, device=dev),
                            c_node_j=torch.as_tensor(p.c_node_j, device=dev, dtype=torch.int32),
                            fwd_opts=dict(max_iters=200000, tol=1e-14, omega=omega),
                            bwd_opts=dict(max_iters=200000, tol=1e-13))
    L = (torch.as_tensor(gv, device=dev) * v).sum() + (torch.as_tensor(gl, device=dev) * lam).sum()
    L.backward()
    fwd = oracle.vfpi(p, max_iters=200000, tol=1e-14, omega=omega)
    gate(v.detach().cpu().numpy(), fwd["v"], 1e-9, "v")
    ref = oracle_adjoint(p, fwd, gv, gl, tol=1e-14)
    errs = {k: gate(t[k].grad.cpu().numpy(), ref[k], 1e-7, f"autograd D grad {k}") for k in ("b", "phi", "mu")}
    errs["A"] = gate(A_val.grad.cpu().numpy().ravel(), ref["A"].ravel(), 1e-7, "autograd D grad A")
    say(f"  autograd D-contacts omega={omega}: {int((p.c_node_j >= 0).sum())} D rows, {errs}")


def test_d_contact_validation():
    p = scenes.random_problem(60, 20, 3, n_d_contacts=8)
    # a D row whose second block is not -R: NOT_NODAL
    crp, ccol, cval = p.jc_bsr()
    bad = cval.copy()
    d0 = int(np.nonzero(p.c_node_j >= 0)[0][0])
    bad[crp[d0] + 1] *= 0.5
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)
    A, _, b, v = upload(p)
    Jc = vf.contacts_from_arrays(crp, ccol, bad, p.phi, p.mu, dtype=torch.float64, device="cuda")
    _, st = s.step(A, b, Jc, v, max_iters=5)
    assert vf.read_stats(st)[0]["status"] & _abi.VFPI_S_NOT_NODAL
    # a node in an S-contact and a D-contact: SHARED_NODE
    cj = p.c_node_j.copy()
    d = np.nonzero(cj >= 0)[0][0]
    cj[d] = p.c_node[np.nonzero(p.c_node_j < 0)[0][0]]
    q = scenes.Problem(**{**p.__dict__, "c_node_j": cj})
    A, Jc, b, v = upload(q)
    _, st = s.step(A, b, Jc, v, max_iters=5)
    assert vf.read_stats(st)[0]["status"] & _abi.VFPI_S_SHARED_NODE
