"""Pins of the V-FPI oracle (Alg. 1 + Alg. 2) against what the paper and the
mathematics fix: a Cholesky solve without contacts, the analytic inclined-plane
particle, Prop. 4 after every sweep, the consistency remark, the Delassus
form solved by PGS and by mode enumeration, and invariances."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import scenes
from oracle import BRANCH_OPEN, BRANCH_SLIP, BRANCH_STICK, contact_jacobian, system_matrix
from oracle.core import InvalidProblem
from oracle.delassus import delassus, pgs
from oracle.enumerate import lcp_enumerate, mode_enumerate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _inclined_analytic(alpha, mu, m, h, g, v_k):
    """Closed-form one-step solution of a particle on an inclined plane:
    free velocity v_f = v_k + h g; if v_f points into the plane the normal
    impulse cancels it; the particle sticks iff m |v_f,t| <= mu lambda_n, else
    slides with friction mu lambda_n opposite to v_f,t."""
    nrm = np.array([np.sin(alpha), 0.0, np.cos(alpha)])
    vf = v_k + h * np.array([0.0, 0.0, -g])
    vn = vf @ nrm
    if vn >= 0:
        return vf, np.zeros(3), "open"
    ln = -m * vn
    vt = vf - vn * nrm
    st = np.linalg.norm(vt)
    if m * st <= mu * ln:
        return np.zeros(3), -m * vf, "stick"
    F = ln * nrm - mu * ln * vt / st
    return vt - (mu * ln / m) * vt / st, F, "slip"


def test_no_contact_converges_to_cholesky_solve():
    p = scenes.random_problem(40, 0, 3, degree=5.0)
    r = oracle.vfpi(p, max_iters=20000, tol=1e-15)
    A = system_matrix(p).toarray()
    x = sla.cho_solve(sla.cho_factor(A), p.b)
    np.testing.assert_allclose(r["v"], x, rtol=0, atol=1e-11 * np.abs(x).max())


@pytest.mark.parametrize("v_t0", [0.0, 0.3])
def test_inclined_plane_threshold_analytic(v_t0):
    """Stick iff mu >= tan(alpha) (from rest), probed at mu = tan(alpha) -+ 1e-6."""
    alpha = np.array([0.2, 0.2, 0.45, 0.45, 0.7, 0.7, 1.0, 0.3])
    mu = np.tan(alpha) + np.array([-1e-6, 1e-6, -1e-6, 1e-6, -1e-6, 1e-6, 0.5, 0.0])
    mu[-1] = 0.0
    m, h, g = 2.0, 0.01, 9.81
    nrm = np.stack([np.sin(alpha), 0 * alpha, np.cos(alpha)], 1)
    t_dir = np.stack([np.cos(alpha), 0 * alpha, -np.sin(alpha)], 1)  # downhill
    v_k = v_t0 * np.cross(nrm, t_dir)  # sideways initial slide, in the plane
    p = scenes.inclined_plane_particles(alpha, mu, mass=m, h=h, g=g, v_k=v_k)
    r = oracle.vfpi(p, max_iters=2, fixed_iters=True, history=True)
    for k in range(alpha.shape[0]):
        v_exp, F_exp, mode = _inclined_analytic(alpha[k], mu[k], m, h, g, v_k[k])
        np.testing.assert_allclose(r["v"][3 * k:3 * k + 3], v_exp, atol=1e-15)
        np.testing.assert_allclose(p.R[k] @ F_exp, r["lam"][k], atol=1e-14)
        exp_branch = {"open": BRANCH_OPEN, "stick": BRANCH_STICK, "slip": BRANCH_SLIP}[mode]
        assert r["branch"][k] == exp_branch
    if v_t0 == 0.0:
        assert r["branch"][:6].tolist() == [BRANCH_SLIP, BRANCH_STICK] * 3
    # W = A^{-1} reaches the exact solution in one sweep: sweep 2 does not move
    assert r["history"][1] <= 1e-15


def test_inclined_plane_golden_fixture():
    """Values in tests/golden/inclined_plane.json are closed-form (written by
    tests/golden/make_inclined_plane.py, which does not call the oracle)."""
    with open(os.path.join(GOLDEN, "inclined_plane.json")) as f:
        cases = json.load(f)["cases"]
    alpha = np.array([c["alpha"] for c in cases])
    mu = np.array([c["mu"] for c in cases])
    p = scenes.inclined_plane_particles(alpha, mu, mass=cases[0]["mass"], h=cases[0]["h"], g=cases[0]["g"])
    # a smaller scalar step converges to the same point
    r = oracle.vfpi(p, max_iters=500, tol=1e-15, w_mode="scalar", alpha_user=0.5 / cases[0]["mass"])
    for k, c in enumerate(cases):
        np.testing.assert_allclose(r["v"][3 * k:3 * k + 3], c["v_next"], atol=1e-13)
        assert r["branch"][k] == {"open": BRANCH_OPEN, "stick": BRANCH_STICK, "slip": BRANCH_SLIP}[c["mode"]]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_prop4_surrogate_scc_exact_every_sweep(seed):
    """After every sweep, (lambda, J v^{l+1} + phi e1) satisfies the SCC of the
    surrogate problem to rounding (Prop. 4) -- checked from v^{l+1} and J alone."""
    p = scenes.random_problem(30, 12, seed, degree=4.0, phi_scale=0.5)
    J = contact_jacobian(p)
    for L in range(1, 8):
        r = oracle.vfpi(p, max_iters=L, fixed_iters=True)
        u = (J @ r["v"]).reshape(-1, 3)
        u[:, 0] += p.phi
        lam = r["lam"]
        sc = 1e-12 * (1 + np.abs(u).max() + np.abs(lam).max())
        assert np.all(lam[:, 0] >= 0) and np.all(u[:, 0] >= -sc)
        assert np.all(np.abs(lam[:, 0] * u[:, 0]) <= sc * (1 + np.abs(lam[:, 0])))
        for m in range(p.n_contacts):
            lt, ut = lam[m, 1:], u[m, 1:]
            assert np.hypot(*lt) <= p.mu[m] * lam[m, 0] + sc
            if r["branch"][m] == BRANCH_STICK:
                assert np.abs(ut).max() <= sc
            elif r["branch"][m] == BRANCH_SLIP:
                assert abs(np.hypot(*lt) - p.mu[m] * lam[m, 0]) <= sc
                assert lt @ ut <= -(1 - 1e-9) * np.hypot(*lt) * np.hypot(*ut) + sc


def test_consistency_at_convergence():
    """Fixed point => A v = b + J^T lambda (consistency remark, Sec. III-B)."""
    sc_, x, v = scenes.cloth_cfg1(0)
    p = sc_.assemble(x, v)
    r = oracle.vfpi(p, max_iters=5000, tol=1e-14)
    A, J = system_matrix(p), contact_jacobian(p)
    res = A @ r["v"] - p.b - J.T @ r["lam"].ravel()
    assert np.linalg.norm(res) <= 1e-9 * np.linalg.norm(p.b)


@pytest.mark.parametrize("seed", range(4))
def test_frictionless_matches_lcp_enumeration(seed):
    p = scenes.random_problem(12, 6, seed, degree=4.0, mu_range=(0.0, 0.0), phi_scale=1.0)
    D, c, Y, vf = delassus(p)
    sols = lcp_enumerate(D[0::3, 0::3], c[0::3])
    assert len(sols) == 1  # D_nn is positive definite: the LCP solution is unique
    r = oracle.vfpi(p, max_iters=100000, tol=1e-15)
    np.testing.assert_allclose(r["lam"][:, 0], sols[0], atol=1e-9 * max(1, np.abs(sols[0]).max()))
    np.testing.assert_allclose(r["lam"][:, 1:], 0, atol=1e-14)
    np.testing.assert_allclose(r["v"], vf + Y[:, 0::3] @ sols[0], atol=1e-9)


@pytest.mark.parametrize("nc,seed", [(1, 0), (1, 1), (2, 2), (2, 3), (3, 4), (3, 5)])
def test_one_to_three_contacts_match_mode_enumeration(nc, seed):
    p = scenes.random_problem(5, nc, seed, degree=3.0, phi_scale=0.6, mu_range=(0.1, 0.9), tag="enum")
    D, c, Y, vf = delassus(p)
    sols = mode_enumerate(D, c, p.mu, seed=seed)
    assert len(sols) >= 1
    r = oracle.vfpi(p, max_iters=200000, tol=1e-15)
    q = pgs(p, tol=1e-15, max_sweeps=200000)
    for lam in (r["lam"].ravel(), q["lam"].ravel()):
        err = min(np.abs(lam - s).max() for s, _ in sols)
        assert err <= 1e-8 * max(1.0, np.abs(lam).max())
    # V-FPI's velocity is the one of its impulse through the Delassus map
    np.testing.assert_allclose(r["v"], vf + Y @ r["lam"].ravel(), atol=1e-8)


def test_cloth10_matches_pgs():
    sc_, x, v = scenes.cloth_cfg1(0)
    p = sc_.assemble(x, v)
    r = oracle.vfpi(p, max_iters=5000, tol=1e-14)
    q = pgs(p, tol=1e-14, max_sweeps=20000)
    np.testing.assert_allclose(r["v"], q["v"], atol=1e-11)
    np.testing.assert_allclose(r["lam"], q["lam"], atol=1e-11 * np.abs(q["lam"]).max())


def test_tangent_basis_invariance():
    """Rotating a contact's tangent pair leaves v unchanged and rotates lambda_t."""
    p = scenes.random_problem(25, 10, 7, degree=4.0, phi_scale=0.5)
    g = np.random.default_rng(0)
    psi = g.uniform(0, 2 * np.pi, size=p.n_contacts)
    c, s = np.cos(psi), np.sin(psi)
    Q = np.zeros((p.n_contacts, 3, 3))
    Q[:, 0, 0] = 1
    Q[:, 1, 1], Q[:, 1, 2], Q[:, 2, 1], Q[:, 2, 2] = c, s, -s, c
    p2 = scenes.Problem(**{**p.__dict__, "R": Q @ p.R})
    r1 = oracle.vfpi(p, max_iters=30, fixed_iters=True)
    r2 = oracle.vfpi(p2, max_iters=30, fixed_iters=True)
    np.testing.assert_allclose(r2["v"], r1["v"], atol=1e-12)
    np.testing.assert_allclose(r2["lam"], np.einsum("mij,mj->mi", Q, r1["lam"]), atol=1e-12)


@pytest.mark.parametrize("mode", ["scalar", "bb1", "bb2"])
def test_converged_solution_independent_of_w(mode):
    sc_, x, v = scenes.cloth_cfg1(0)
    p = sc_.assemble(x, v)
    ref = oracle.vfpi(p, max_iters=5000, tol=1e-14)
    alpha = oracle.core.gershgorin_alpha(system_matrix(p)) if mode == "scalar" else None
    r = oracle.vfpi(p, max_iters=50000, tol=1e-14, w_mode=mode, alpha_user=alpha)
    np.testing.assert_allclose(r["v"], ref["v"], atol=1e-10)


def test_validation_rejects_broken_preconditions():
    p = scenes.random_problem(10, 3, 0)
    bad = scenes.Problem(**{**p.__dict__, "c_node": np.array([1, 1, 2])})
    with pytest.raises(InvalidProblem, match="SHARED_NODE"):
        oracle.vfpi(bad)
    R = p.R.copy()
    R[0, 0] *= 1.01
    with pytest.raises(InvalidProblem, match="NOT_ORTHONORMAL"):
        oracle.vfpi(scenes.Problem(**{**p.__dict__, "R": R}))
    val = p.val.copy()
    d0 = p.row_ptr[0] + np.nonzero(p.col_idx[p.row_ptr[0]:p.row_ptr[1]] == 0)[0][0]
    val[d0, 0, 0] = -1.0
    with pytest.raises(InvalidProblem, match="NONPOS_DIAG"):
        oracle.vfpi(scenes.Problem(**{**p.__dict__, "val": val}))
    b = p.b.copy()
    b[3] = np.nan
    with pytest.raises(InvalidProblem, match="NONFINITE"):
        oracle.vfpi(scenes.Problem(**{**p.__dict__, "b": b}))


def test_zero_iterations_and_empty_contacts():
    p = scenes.random_problem(10, 0, 1)
    r = oracle.vfpi(p, max_iters=0)
    np.testing.assert_array_equal(r["v"], p.v0)
    assert r["iters"] == 0 and r["lam"].shape == (0, 3)


@pytest.mark.parametrize("omega", [1e-3, 0.05])
def test_invertible_contact_recovers_impulse_from_velocity(omega):
    """Invertible contact (eq. invt, Omega = omega I): at convergence the
    impulse is a function of the velocity alone, lambda_m =
    ProjectFC(-(J_m v + phi_m e1) / omega)."""
    p = scenes.random_problem(40, 16, 9, degree=4.0, phi_scale=0.5, mu_range=(0.1, 0.9))
    r = oracle.vfpi(p, max_iters=200000, tol=1e-15, omega=omega)
    u = (contact_jacobian(p) @ r["v"]).reshape(-1, 3)
    u[:, 0] += p.phi
    lam_from_v, _ = oracle.project_strict(-u / omega, p.mu)
    np.testing.assert_allclose(r["lam"], lam_from_v, atol=1e-9 * max(1.0, np.abs(r["lam"]).max()))
    # and it differs from the exact (omega = 0) model
    r0 = oracle.vfpi(p, max_iters=200000, tol=1e-15)
    assert np.abs(r0["v"] - r["v"]).max() > 1e-6 * omega


@pytest.mark.parametrize("mode", ["bb1", "bb2"])
def test_bb_step_is_exact_on_one_eigenspace(mode):
    """A = diag(1, 4) (Gershgorin alpha^1 = 1/4), error in the eigenvalue-1 space:
    sweep 1 shrinks it by 3/4, so s and z = A s lie in that space and both BB
    quotients give alpha^2 = 1 exactly; sweep 2 then lands on A^-1 b and sweep 3
    does not move (Sec. IV-C.2)."""
    p, x = scenes.two_level_diagonal(20, 0)
    r1 = oracle.vfpi(p, max_iters=1, fixed_iters=True, w_mode=mode)
    np.testing.assert_allclose(r1["v"] - x, 0.75 * (p.v0 - x), atol=1e-15)
    r = oracle.vfpi(p, max_iters=3, fixed_iters=True, w_mode=mode, history=True)
    assert r["alpha"] == 1.0
    np.testing.assert_allclose(r["v"], x, atol=1e-14)
    assert r["history"][2] <= 1e-14 and r["history"][1] > 0.1


@pytest.mark.parametrize("mode", ["bb1", "bb2"])
def test_bb_converges_on_two_eigenvalues(mode):
    p, x = scenes.two_level_diagonal(20, 1, in_low_space=False)
    r = oracle.vfpi(p, max_iters=200, tol=1e-13, w_mode=mode)
    assert r["iters"] < 200
    np.testing.assert_allclose(r["v"], x, atol=1e-12)
