"""Invertible contact (Sec. III-E, eq. invt, Omega = omega I) on the GPU: the
forward kernels, the batched FP32 kernel and the adjoint against the FP64
oracle run with the same omega."""
import numpy as np
import pytest
import torch

import oracle
import paper_2201_09212_amd as vf
import scenes
from oracle.adjoint import adjoint as oracle_adjoint
from paper_2201_09212_amd import _abi
from tests.gpu_util import fixed_parity, gate, gpu_step, rel, say, upload
from tests.test_gpu_batched import _check_envs, _envs_small, run_batched

pytestmark = pytest.mark.gpu

VARIANTS = {"grid_node2": 1 | (2 << 8), "grid_row1": 2, "regs2": 5 | (2 << 8), "regs8": 5 | (8 << 8),
            "wg1_node16": 3}


def _problems():
    sc, x, v = scenes.cloth_cfg1(0)
    yield "cloth10", sc.assemble(x, v)
    yield "random700", scenes.random_problem(700, 300, 4, degree=5.0, phi_scale=0.5)


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("omega", [1e-3, 0.5])
def test_invertible_fixed_sweeps_parity(variant, omega):
    for name, p in _problems():
        L = 40
        ref = oracle.vfpi(p, max_iters=L, fixed_iters=True, omega=omega)
        ev, el, st, ties = fixed_parity(p, ref, L, 1e-9, f"{name} {variant} omega={omega}",
                                        variant=VARIANTS[variant], omega=omega)
        say(f"  {name} {variant} omega={omega}: rel_v={ev:.2e} rel_lam={el:.2e} branch ties={ties}")


def test_invertible_converged_impulse_from_velocity():
    p = scenes.random_problem(700, 300, 4, degree=5.0, phi_scale=0.5)
    omega = 0.05
    v, lam, st, _ = gpu_step(p, max_iters=100000, tol=1e-13, omega=omega)
    assert st["status"] == _abi.VFPI_S_CONVERGED
    u = (oracle.contact_jacobian(p) @ v).reshape(-1, 3)
    u[:, 0] += p.phi
    lam_v, _ = oracle.project_strict(-u / omega, p.mu)
    say(f"  random700 omega={omega}: {st['iters']} sweeps, rel(lambda, P(-u/omega)) = {rel(lam, lam_v):.2e}")
    gate(lam, lam_v, 1e-9, "lambda vs P(-u/omega)")


def test_batched_invertible_parity():
    envs = _envs_small()
    batch = scenes.concat_problems(envs)
    L = 30
    v, lam, st = run_batched(batch, max_iters=L, fixed_iters=True, omega=0.01)
    worst = _check_envs(batch, v, lam, st, L, omega=0.01)
    say(f"  batched omega=0.01: worst rel {worst:.2e}")


@pytest.mark.parametrize("omega", [0.02, 0.3])
def test_invertible_adjoint_matches_oracle(omega):
    p = scenes.random_problem(200, 90, 2, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), tag="adj")
    g = np.random.default_rng(3)
    gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)
    A, Jc, b, v = upload(p)
    tape = s.tape(p.n_nodes, p.n_contacts)
    lam, st = s.step(A, b, Jc, v, tape=tape, max_iters=200000, tol=1e-14, omega=omega)
    out = s.step_backward(A, Jc, tape, torch.as_tensor(gv, device="cuda"), torch.as_tensor(gl, device="cuda"),
                          want_A=True, max_iters=200000, tol=1e-13, omega=omega)
    torch.cuda.synchronize()
    fwd = oracle.vfpi(p, max_iters=200000, tol=1e-14, omega=omega)
    ref = oracle_adjoint(p, fwd, gv, gl, tol=1e-14)
    assert vf.read_stats(st)[0]["status"] == _abi.VFPI_S_CONVERGED
    assert vf.read_stats(out["stats"])[0]["status"] == _abi.VFPI_S_CONVERGED
    errs = {k: gate(out[k].cpu().numpy(), ref[k], 1e-7, f"grad {k}") for k in ("b", "A", "phi", "mu")}
    say(f"  adjoint omega={omega}: {errs}")
