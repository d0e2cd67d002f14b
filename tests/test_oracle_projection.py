"""Pins of the two ProjectFC operators (eq. operator) against closed forms,
brute force and Moreau's decomposition -- independent of how the oracle
writes them."""
import numpy as np
import pytest

from oracle import BRANCH_OPEN, BRANCH_SLIP, BRANCH_STICK, project_proximal, project_strict


def test_strict_closed_form_cases():
    mu = np.array([0.5, 0.5, 0.5, 0.5, 0.0, 0.5])
    ls = np.array([
        [-1.0, 3.0, 4.0],    # separating: open, all zero
        [2.0, 0.3, 0.4],     # |t| = 0.5 <= mu n = 1: stick, unchanged
        [2.0, 3.0, 4.0],     # |t| = 5 > 1: slip, t scaled to length 1
        [2.0, 0.0, 0.0],     # no tangential part: stick
        [2.0, 3.0, 4.0],     # mu = 0: frictionless slip, t -> 0
        [0.0, 1.0, 0.0],     # lambda*_n = 0: open (tie goes to open)
    ])
    lam, br = project_strict(ls, mu)
    exp = np.array([[0, 0, 0], [2, 0.3, 0.4], [2, 0.6, 0.8], [2, 0, 0], [2, 0, 0], [0, 0, 0]], dtype=float)
    np.testing.assert_allclose(lam, exp, rtol=0, atol=1e-15)
    assert br.tolist() == [BRANCH_OPEN, BRANCH_STICK, BRANCH_SLIP, BRANCH_STICK, BRANCH_SLIP, BRANCH_OPEN]


def test_strict_is_normal_clamp_plus_disk_projection_bruteforce():
    g = np.random.default_rng(1)
    ls = g.normal(size=(200, 3))
    mu = g.uniform(0, 1.5, size=200)
    lam, _ = project_strict(ls, mu)
    np.testing.assert_array_equal(lam[:, 0], np.maximum(ls[:, 0], 0))
    # brute force: the closest point of a fine polar grid of the disk
    rr = np.linspace(0, 1, 401)[:, None]
    aa = np.linspace(0, 2 * np.pi, 721)[None, :]
    for k in range(0, 200, 7):
        rad = mu[k] * max(ls[k, 0], 0)
        pts = np.stack([(rad * rr * np.cos(aa)).ravel(), (rad * rr * np.sin(aa)).ravel()], 1)
        best = pts[np.argmin(((pts - ls[k, 1:]) ** 2).sum(1))]
        assert np.linalg.norm(lam[k, 1:] - best) <= rad * 0.01 + 1e-14


def _in_cone(lam, mu, tol=1e-12):
    return (lam[:, 0] >= -tol) & (np.hypot(lam[:, 1], lam[:, 2]) <= mu * lam[:, 0] + tol)


def test_proximal_moreau_decomposition():
    """x = P_K(x) + P_K°(x): the residual x - P_K(x) lies in the polar cone
    K° = {mu |t| <= -n} and is orthogonal to P_K(x)."""
    g = np.random.default_rng(2)
    x = g.normal(size=(500, 3)) * 3
    mu = g.uniform(0, 2, size=500)
    lam, _ = project_proximal(x, mu)
    assert np.all(_in_cone(lam, mu))
    res = x - lam
    assert np.all(mu * np.hypot(res[:, 1], res[:, 2]) <= -res[:, 0] + 1e-12)
    np.testing.assert_allclose(np.einsum("ij,ij->i", res, lam), 0, atol=1e-12)


def test_proximal_bruteforce_small():
    g = np.random.default_rng(3)
    x = g.normal(size=(30, 3))
    mu = g.uniform(0.1, 1.2, size=30)
    lam, _ = project_proximal(x, mu)
    for k in range(30):
        # sample the cone surface and interior densely; no sample beats the projection
        n = np.linspace(0, 4, 161)
        r = np.linspace(0, 1, 41)
        a = np.linspace(0, 2 * np.pi, 91)
        N, Rr, Aa = np.meshgrid(n, r, a, indexing="ij")
        pts = np.stack([N.ravel(), (mu[k] * N * Rr * np.cos(Aa)).ravel(), (mu[k] * N * Rr * np.sin(Aa)).ravel()], 1)
        dbest = np.sqrt(((pts - x[k]) ** 2).sum(1).min())
        assert np.linalg.norm(lam[k] - x[k]) <= dbest + 1e-12


@pytest.mark.parametrize("proj", [project_strict, project_proximal])
def test_projection_idempotent_and_fixed_inside(proj):
    g = np.random.default_rng(4)
    x = g.normal(size=(300, 3))
    mu = g.uniform(0, 1, size=300)
    lam, _ = proj(x, mu)
    lam2, _ = proj(lam, mu)
    np.testing.assert_allclose(lam2, lam, atol=1e-15)
