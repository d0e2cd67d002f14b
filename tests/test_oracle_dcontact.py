"""Pins of the oracle on node-node (D) contacts (eq. jcnode, D case; Prop. 3
with gamma = w_i + w_j): the two-body collision in closed form, conservation
of momentum, Prop. 4 after every sweep, mode enumeration and PGS."""
import numpy as np
import pytest

import oracle
import scenes
from oracle import BRANCH_OPEN, BRANCH_SLIP, BRANCH_STICK, contact_jacobian, system_matrix
from oracle.delassus import delassus, pgs
from oracle.enumerate import mode_enumerate


def _pair_closed_form(m1, m2, n, vi, vj, mu, h, g):
    """Relative motion of two particles is the one-particle problem with the
    reduced mass m1 m2 / (m1 + m2): impulse P on i (-P on j)."""
    grav = np.array([0.0, 0.0, -g * h])
    uf = (vi + grav) - (vj + grav)
    mr = m1 * m2 / (m1 + m2)
    un = uf @ n
    if un >= 0:
        P, mode = np.zeros(3), "open"
    else:
        ln = -mr * un
        ut = uf - un * n
        st = np.linalg.norm(ut)
        if mr * st <= mu * ln:
            P, mode = -mr * uf, "stick"
        else:
            P, mode = ln * n - mu * ln * ut / st, "slip"
    return vi + grav + P / m1, vj + grav - P / m2, P, mode


def test_two_body_collision_closed_form():
    g = np.random.default_rng(11)
    K = 12
    m1, m2 = g.uniform(0.2, 3.0, K), g.uniform(0.2, 3.0, K)
    nrm = g.normal(size=(K, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    mu = g.uniform(0.1, 1.2, K)
    # relative velocity: approach speed a along -n plus a tangential part of
    # size s * mu * a (s < 1: stick, s > 1: slip) or separation (open)
    t = np.cross(nrm, g.normal(size=(K, 3)))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    a = g.uniform(0.5, 2.0, K) * np.where(np.arange(K) % 3 == 0, -1.0, 1.0)
    s = np.where(np.arange(K) % 3 == 1, 0.5, 2.0)
    vj = g.normal(size=(K, 3))
    vi = vj - a[:, None] * nrm + (s * mu * np.abs(a))[:, None] * t
    p = scenes.colliding_particle_pairs(m1, m2, nrm, vi, vj, mu, h=0.01, g=9.81)
    r = oracle.vfpi(p, max_iters=100000, tol=1e-15)
    modes = set()
    for k in range(K):
        ei, ej, P, mode = _pair_closed_form(m1[k], m2[k], nrm[k], vi[k], vj[k], mu[k], 0.01, 9.81)
        modes.add(mode)
        np.testing.assert_allclose(r["v"][6 * k:6 * k + 3], ei, atol=1e-12)
        np.testing.assert_allclose(r["v"][6 * k + 3:6 * k + 6], ej, atol=1e-12)
        np.testing.assert_allclose(p.R[k] @ P, r["lam"][k], atol=1e-12)
        assert r["branch"][k] == {"open": BRANCH_OPEN, "stick": BRANCH_STICK, "slip": BRANCH_SLIP}[mode]
    assert modes == {"open", "stick", "slip"}
    # the pair's two nodes share one w (6 DOFs) and gamma = 2 w (Prop. 3)
    np.testing.assert_allclose(r["gamma"], 2 * r["w"][6 * np.arange(K)], rtol=0)
    assert np.all(r["w"][6 * np.arange(K)] == r["w"][6 * np.arange(K) + 3])


@pytest.mark.parametrize("seed", [0, 1])
def test_momentum_conserved_with_d_contacts_only(seed):
    """J^T lambda of a D-contact applies R^T lambda to one node and the
    opposite to the other, so at the fixed point (A v - b) sums to zero over
    the nodes, per axis."""
    p = scenes.random_problem(60, 20, seed, degree=4.0, phi_scale=0.5, n_d_contacts=20, mu_range=(0.2, 0.9))
    r = oracle.vfpi(p, max_iters=200000, tol=1e-14)
    res = (system_matrix(p) @ r["v"] - p.b).reshape(-1, 3).sum(0)
    assert np.abs(res).max() <= 1e-10 * np.abs(p.b).max()
    assert np.abs(r["lam"]).max() > 1e-3  # the contacts are active


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_prop4_with_d_contacts(seed):
    p = scenes.random_problem(40, 14, seed, degree=4.0, phi_scale=0.5, n_d_contacts=8)
    J = contact_jacobian(p)
    for L in range(1, 7):
        r = oracle.vfpi(p, max_iters=L, fixed_iters=True)
        u = (J @ r["v"]).reshape(-1, 3)
        u[:, 0] += p.phi
        lam = r["lam"]
        sc = 1e-12 * (1 + np.abs(u).max() + np.abs(lam).max())
        assert np.all(lam[:, 0] >= 0) and np.all(u[:, 0] >= -sc)
        assert np.all(np.abs(lam[:, 0] * u[:, 0]) <= sc * (1 + np.abs(lam[:, 0])))
        for m in range(p.n_contacts):
            if r["branch"][m] == BRANCH_STICK:
                assert np.abs(u[m, 1:]).max() <= sc
            elif r["branch"][m] == BRANCH_SLIP:
                lt, ut = lam[m, 1:], u[m, 1:]
                assert abs(np.hypot(*lt) - p.mu[m] * lam[m, 0]) <= sc
                assert lt @ ut <= -(1 - 1e-9) * np.hypot(*lt) * np.hypot(*ut) + sc


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_d_contacts_match_mode_enumeration_and_pgs(seed):
    p = scenes.random_problem(7, 2, seed, degree=3.0, phi_scale=0.6, mu_range=(0.1, 0.9), n_d_contacts=1,
                              tag="enum_d")
    D, c, Y, vf = delassus(p)
    sols = mode_enumerate(D, c, p.mu, seed=seed)
    assert sols
    r = oracle.vfpi(p, max_iters=200000, tol=1e-15)
    q = pgs(p, tol=1e-15, max_sweeps=200000)
    for lam in (r["lam"].ravel(), q["lam"].ravel()):
        err = min(np.abs(lam - s).max() for s, _ in sols)
        assert err <= 1e-8 * max(1.0, np.abs(lam).max())
    np.testing.assert_allclose(r["v"], vf + Y @ r["lam"].ravel(), atol=1e-8)


def test_cloth_pair_collision_conserves_momentum():
    """Two sheets meeting in free fall: springs and D-contacts are internal,
    so at the fixed point sum_i (A v - b)_i = 0 (per axis)."""
    p = scenes.cloth_pair_collision(0, side=16)
    r = oracle.vfpi(p, max_iters=20000, tol=1e-13)
    assert r["iters"] < 20000 and np.count_nonzero(r["branch"]) > 10
    res = (system_matrix(p) @ r["v"] - p.b).reshape(-1, 3).sum(0)
    assert np.abs(res).max() <= 1e-10 * np.abs(p.b).max()
