"""FP64 HIP adjoint (vfpi_step_backward) vs the FP64 oracle adjoint at a
converged forward step, and vs central finite differences of the HIP
forward itself (bar 1e-4 relative; the oracle comparison is held to 1e-7)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2201_09212_amd as vf
import scenes
from oracle.adjoint import adjoint as oracle_adjoint
from paper_2201_09212_amd import _abi
from tests.gpu_util import gate, say, upload

pytestmark = pytest.mark.gpu


def gpu_fwd_bwd(p, gv, gl=None, tol=1e-14, want_A=True, variant=0, **opt):
    s = vf.Solver(p.n_nodes, p.nnzb, max(p.n_contacts, 1))
    A, Jc, b, v = upload(p)
    tape = s.tape(p.n_nodes, p.n_contacts)
    lam, st = s.step(A, b, Jc, v, tape=tape, max_iters=200000, tol=tol, **opt)
    gvt = torch.as_tensor(gv, device="cuda")
    glt = None if gl is None else torch.as_tensor(gl, device="cuda")
    g = s.step_backward(A, Jc, tape, gvt, glt, want_A=want_A, max_iters=200000, tol=1e-13, variant=variant,
                        **opt)
    torch.cuda.synchronize()
    out = {k: (t.cpu().numpy() if isinstance(t, torch.Tensor) and k != "stats" else t) for k, t in g.items()}
    out["fwd_stats"] = vf.read_stats(st)[0]
    out["bwd_stats"] = vf.read_stats(g["stats"])[0]
    out["v"] = v.cpu().numpy()
    out["lam"] = lam.cpu().numpy()
    return out


def _cases():
    sc, x, v = scenes.cloth_cfg1(0)
    yield "cloth10", sc.assemble(x, v)
    for n, nc, seed in [(14, 7, 0), (70, 40, 1), (200, 90, 2)]:
        yield f"random{n}", scenes.random_problem(n, nc, seed, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), tag="adj")


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("with_glam", [False, True])
@pytest.mark.parametrize("name,p", list(_cases()))
def test_adjoint_matches_oracle(name, p, with_glam, variant):
    g = np.random.default_rng(3)
    gv = g.normal(size=p.n)
    gl = g.normal(size=3 * p.n_contacts) if with_glam else None
    out = gpu_fwd_bwd(p, gv, gl, variant=variant)
    fwd = oracle.vfpi(p, max_iters=200000, tol=1e-14)
    ref = oracle_adjoint(p, fwd, gv, gl, tol=1e-14)
    assert out["fwd_stats"]["status"] == _abi.VFPI_S_CONVERGED
    assert out["bwd_stats"]["status"] == _abi.VFPI_S_CONVERGED, out["bwd_stats"]
    errs = {k: gate(out[k], ref[k], 1e-7, f"{name} grad {k}") for k in ("b", "A", "phi", "mu")}
    say(f"  {name} glam={with_glam}: fwd {out['fwd_stats']['iters']} bwd {out['bwd_stats']['iters']} sweeps, {errs}")


@pytest.mark.parametrize("opt", [{}, {"projection": "proximal"}, {"projection": "proximal", "omega": 0.05}])
@pytest.mark.parametrize("variant", [0, 1, 3])
def test_proximal_adjoint_matches_oracle(variant, opt):
    """The proximal operator's adjoint (cone projection Jacobian) against the
    oracle's, with and without the invertible contact; {} is the strict
    reference of the same problems."""
    for name, p in list(_cases())[1:]:
        g = np.random.default_rng(5)
        gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
        out = gpu_fwd_bwd(p, gv, gl, variant=variant, **opt)
        fwd = oracle.vfpi(p, max_iters=200000, tol=1e-14, **opt)
        ref = oracle_adjoint(p, fwd, gv, gl, tol=1e-14)
        assert out["fwd_stats"]["status"] == _abi.VFPI_S_CONVERGED
        assert out["bwd_stats"]["status"] == _abi.VFPI_S_CONVERGED, out["bwd_stats"]
        errs = {k: gate(out[k], ref[k], 1e-7, f"{name} grad {k}") for k in ("b", "A", "phi", "mu")}
        slip = int((fwd["branch"] == 2).sum())
        say(f"  {name} {opt} variant {variant}: {slip} slipping, bwd {out['bwd_stats']['iters']} sweeps, {errs}")


@pytest.mark.parametrize("opt", [{}, {"projection": "proximal"}])
def test_adjoint_vs_central_differences_of_gpu_forward(opt):
    p = scenes.random_problem(40, 18, 5, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), tag="adj")
    g = np.random.default_rng(4)
    gv = g.normal(size=p.n)
    out = gpu_fwd_bwd(p, gv, **opt)
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)

    def loss(q):
        A, Jc, b, v = upload(q)
        lam, st = s.step(A, b, Jc, v, max_iters=200000, tol=1e-14, **opt)
        torch.cuda.synchronize()
        return float(gv @ v.cpu().numpy())

    eps = 1e-6
    checked = 0
    for k in g.choice(p.n, 8, replace=False):
        e = np.zeros(p.n)
        e[k] = eps
        fd = (loss(scenes.Problem(**{**p.__dict__, "b": p.b + e})) - loss(scenes.Problem(**{**p.__dict__, "b": p.b - e}))) / (2 * eps)
        assert abs(fd - out["b"][k]) <= 1e-4 * max(1.0, abs(fd)), (k, fd, out["b"][k])
        checked += 1
    for m in range(p.n_contacts):
        for name in ("phi", "mu"):
            e = np.zeros(p.n_contacts)
            e[m] = eps
            base = getattr(p, name)
            fd = (loss(scenes.Problem(**{**p.__dict__, name: base + e})) -
                  loss(scenes.Problem(**{**p.__dict__, name: base - e}))) / (2 * eps)
            assert abs(fd - out[name][m]) <= 1e-4 * max(1.0, abs(fd)), (name, m, fd, out[name][m])
            checked += 1
    say(f"  central differences checked: {checked}")


def test_adjoint_grid_and_single_workgroup_agree():
    """The register-resident adjoint (default; kind 5 with 2 or 8 chunk
    slots), the streaming one (kind 1) and one workgroup (kind 3) agree."""
    sc, x, v = scenes.cloth_cfg5_scene(0)
    x[:, 2] = np.random.default_rng(1).uniform(-5e-4, 4e-3, size=x.shape[0])
    p = sc.assemble(x, v)
    gv = np.random.default_rng(2).normal(size=p.n)
    a = gpu_fwd_bwd(p, gv, tol=1e-13)
    for var in (1, 3, 5 | (8 << 8)):
        b = gpu_fwd_bwd(p, gv, tol=1e-13, variant=var)
        say(f"  adjoint variant {var:#x}: {b['bwd_stats']['iters']} sweeps (default {a['bwd_stats']['iters']})")
        assert abs(b["bwd_stats"]["iters"] - a["bwd_stats"]["iters"]) <= 1
        for k in ("b", "A", "phi", "mu"):
            gate(a[k], b[k], 1e-10, f"variant {var:#x} grad {k}")
    fwd = oracle.vfpi(p, max_iters=200000, tol=1e-13)
    ref = oracle_adjoint(p, fwd, gv, tol=1e-14)
    errs = {k: gate(a[k], ref[k], 1e-6, f"cloth64 grad {k}") for k in ("b", "A", "phi", "mu")}
    say(f"  cloth64 adjoint: fwd {a['fwd_stats']['iters']} bwd {a['bwd_stats']['iters']} sweeps, {errs}")


def test_adjoint_solid_mesh_launches_agree():
    """A solid mesh (FEM 16x16x4 cells, rows of up to 19 blocks, so every
    register-resident instance streams levels beyond the ones it keeps): the
    register-resident adjoint with 2 (default), 4, 5 and 8 chunk slots and
    the streaming one agree, and the default matches the oracle's adjoint."""
    sc, x, v = scenes.fem_ctx(0)
    p = sc.assemble(x, v)
    gv = np.random.default_rng(3).normal(size=p.n)
    a = gpu_fwd_bwd(p, gv, tol=1e-13)
    assert a["fwd_stats"]["status"] == _abi.VFPI_S_CONVERGED
    assert a["bwd_stats"]["status"] == _abi.VFPI_S_CONVERGED, a["bwd_stats"]
    for var in (1, 5 | (4 << 8), 5 | (5 << 8), 5 | (8 << 8)):
        b = gpu_fwd_bwd(p, gv, tol=1e-13, variant=var)
        say(f"  FEM adjoint variant {var:#x}: {b['bwd_stats']['iters']} sweeps (default {a['bwd_stats']['iters']})")
        assert abs(b["bwd_stats"]["iters"] - a["bwd_stats"]["iters"]) <= 1
        for k in ("b", "A", "phi", "mu"):
            gate(a[k], b[k], 1e-10, f"FEM variant {var:#x} grad {k}")
    fwd = oracle.vfpi(p, max_iters=200000, tol=1e-13)
    ref = oracle_adjoint(p, fwd, gv, tol=1e-14)
    errs = {k: gate(a[k], ref[k], 1e-6, f"FEM grad {k}") for k in ("b", "A", "phi", "mu")}
    say(f"  FEM 16x16x4 adjoint: fwd {a['fwd_stats']['iters']} bwd {a['bwd_stats']['iters']} sweeps, {errs}")


def test_d_contact_adjoint_launches_agree():
    """D-contacts (two 32x32 cloths meeting, J_m = [R, -R]): the register-
    resident adjoint (default and 8 chunk slots), the streaming one and one
    workgroup agree, and the default matches the oracle's adjoint."""
    p = scenes.cloth_pair_collision(0, side=32)
    assert p.n_contacts > 100 and (np.asarray(p.c_node_j) >= 0).all()
    g = np.random.default_rng(5)
    gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
    a = gpu_fwd_bwd(p, gv, gl, tol=1e-13)
    assert a["fwd_stats"]["status"] == _abi.VFPI_S_CONVERGED
    assert a["bwd_stats"]["status"] == _abi.VFPI_S_CONVERGED, a["bwd_stats"]
    for var in (1, 3, 5 | (8 << 8)):
        b = gpu_fwd_bwd(p, gv, gl, tol=1e-13, variant=var)
        say(f"  D adjoint variant {var:#x}: {b['bwd_stats']['iters']} sweeps (default {a['bwd_stats']['iters']})")
        assert abs(b["bwd_stats"]["iters"] - a["bwd_stats"]["iters"]) <= 1
        for k in ("b", "A", "phi", "mu"):
            gate(a[k], b[k], 1e-10, f"D variant {var:#x} grad {k}")
    fwd = oracle.vfpi(p, max_iters=200000, tol=1e-13)
    ref = oracle_adjoint(p, fwd, gv, gl, tol=1e-14)
    errs = {k: gate(a[k], ref[k], 1e-6, f"cloth pair grad {k}") for k in ("b", "A", "phi", "mu")}
    say(f"  cloth pair D adjoint: {p.n_contacts} contacts, bwd {a['bwd_stats']['iters']} sweeps, {errs}")


def _aniso_cases():
    for name, p in list(_cases())[1:]:
        p.mu2 = np.asarray(p.mu) * np.random.default_rng(p.n_nodes).uniform(0.3, 1.8, size=p.n_contacts)
        yield name, p
    p = scenes.random_problem(120, 50, 6, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), n_d_contacts=15,
                              tag="adj")
    p.mu2 = np.asarray(p.mu) * np.random.default_rng(7).uniform(0.3, 1.8, size=p.n_contacts)
    yield "random120_d", p
    # zero coefficients: the ellipse degenerates to a segment (componentwise clamp)
    p = scenes.random_problem(200, 90, 2, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), tag="adj")
    mu, mu2 = np.array(p.mu, dtype=np.float64), np.array(p.mu, dtype=np.float64) * 0.6
    mu[::5] = 0.0
    mu2[2::5] = 0.0
    p.mu, p.mu2 = mu, mu2
    yield "random200_zero", p


@pytest.mark.parametrize("variant", [0, 1, 3])
def test_aniso_adjoint_matches_oracle(variant):
    """Anisotropic friction (strict operator on the elliptic cone): the
    adjoint's b, A, phi, mu and mu2 gradients against the oracle's, on
    S-contacts, D-contacts and with zero coefficients (segments)."""
    for name, p in _aniso_cases():
        g = np.random.default_rng(8)
        gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
        out = gpu_fwd_bwd(p, gv, gl, variant=variant)
        fwd = oracle.vfpi(p, max_iters=200000, tol=1e-14)
        ref = oracle_adjoint(p, fwd, gv, gl, tol=1e-14)
        assert out["fwd_stats"]["status"] == _abi.VFPI_S_CONVERGED
        assert out["bwd_stats"]["status"] == _abi.VFPI_S_CONVERGED, out["bwd_stats"]
        errs = {k: gate(out[k], ref[k], 1e-7, f"{name} aniso grad {k}") for k in ("b", "A", "phi", "mu", "mu2")}
        slip = int((fwd["branch"] == 2).sum())
        say(f"  {name} aniso variant {variant}: {slip} slipping, bwd {out['bwd_stats']['iters']} sweeps, {errs}")
        assert slip >= 3


def test_aniso_adjoint_vs_central_differences_of_gpu_forward():
    """b, phi, mu and mu2 gradients with anisotropic friction against central
    differences of the HIP forward."""
    p = scenes.random_problem(40, 18, 5, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), tag="adj")
    p.mu2 = np.asarray(p.mu) * np.random.default_rng(9).uniform(0.3, 1.8, size=p.n_contacts)
    g = np.random.default_rng(4)
    gv = g.normal(size=p.n)
    out = gpu_fwd_bwd(p, gv)
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)

    def loss(q):
        A, Jc, b, v = upload(q)
        lam, st = s.step(A, b, Jc, v, max_iters=200000, tol=1e-14)
        torch.cuda.synchronize()
        return float(gv @ v.cpu().numpy())

    eps = 1e-6
    checked = 0
    for k in g.choice(p.n, 6, replace=False):
        e = np.zeros(p.n)
        e[k] = eps
        fd = (loss(scenes.Problem(**{**p.__dict__, "b": p.b + e})) - loss(scenes.Problem(**{**p.__dict__, "b": p.b - e}))) / (2 * eps)
        assert abs(fd - out["b"][k]) <= 1e-4 * max(1.0, abs(fd)), (k, fd, out["b"][k])
        checked += 1
    for m in range(p.n_contacts):
        for name in ("phi", "mu", "mu2"):
            e = np.zeros(p.n_contacts)
            e[m] = eps
            base = np.asarray(getattr(p, name))
            fd = (loss(scenes.Problem(**{**p.__dict__, name: base + e})) -
                  loss(scenes.Problem(**{**p.__dict__, name: base - e}))) / (2 * eps)
            assert abs(fd - out[name][m]) <= 1e-4 * max(1.0, abs(fd)), (name, m, fd, out[name][m])
            checked += 1
    say(f"  central differences checked (aniso): {checked}")


def test_autograd_solve_with_aniso_friction():
    """vfpi_solve (torch.autograd.Function over the HIP forward and adjoint)
    hands b, phi, mu and mu2 gradients to PyTorch: they equal the oracle's."""
    from paper_2201_09212_amd.autograd import vfpi_solve
    p = scenes.random_problem(70, 40, 1, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), tag="adj")
    p.mu2 = np.asarray(p.mu) * np.random.default_rng(11).uniform(0.3, 1.8, size=p.n_contacts)
    crp, ccol, cval = p.jc_bsr()
    assert np.array_equal(np.diff(crp), np.ones(p.n_contacts))  # S-contacts: one block per row
    dev = torch.device("cuda", 0)
    t = {k: torch.tensor(np.asarray(getattr(p, k), dtype=np.float64), device=dev, requires_grad=True)
         for k in ("b", "phi", "mu", "mu2")}
    A_val = torch.tensor(p.val, device=dev).view(-1, 3, 3).requires_grad_(True)
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)
    g = np.random.default_rng(12)
    gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
    v, lam, st = vfpi_solve(s, A_val, t["b"], t["phi"], t["mu"], torch.as_tensor(p.v0, device=dev),
                            torch.as_tensor(p.row_ptr, device=dev, dtype=torch.int32),
                            torch.as_tensor(p.col_idx, device=dev, dtype=torch.int32), p.n_nodes,
                            torch.as_tensor(ccol, device=dev, dtype=torch.int32),
                            torch.as_tensor(cval, device=dev).view(-1, 3, 3), mu2=t["mu2"],
                            fwd_opts=dict(max_iters=200000, tol=1e-14), bwd_opts=dict(max_iters=200000, tol=1e-13))
    L = (torch.as_tensor(gv, device=dev) * v).sum() + (torch.as_tensor(gl, device=dev) * lam).sum()
    L.backward()
    fwd = oracle.vfpi(p, max_iters=200000, tol=1e-14)
    ref = oracle_adjoint(p, fwd, gv, gl, tol=1e-14)
    errs = {k: gate(t[k].grad.cpu().numpy(), ref[k], 1e-7, f"autograd grad {k}") for k in ("b", "phi", "mu", "mu2")}
    errs["A"] = gate(A_val.grad.cpu().numpy().ravel(), ref["A"].ravel(), 1e-7, "autograd grad A")
    say(f"  autograd aniso: {errs}")
