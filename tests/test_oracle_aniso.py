"""Pins of the anisotropic strict operator (Sec. III-E, elliptic cone; Prop.
6): the closest point in the ellipse by brute force over its boundary, the
Lagrange (normal-direction) condition, the isotropic special case, the MDP
objective, and one converged particle sliding on a plane."""
import numpy as np
import pytest

import oracle
import scenes
from oracle import BRANCH_OPEN, BRANCH_SLIP, BRANCH_STICK
from oracle.core import project_strict, project_strict_aniso


def _cases(k, seed):
    g = np.random.default_rng(seed)
    ls = g.normal(size=(k, 3)) * np.array([1.0, 0.7, 0.7]) + np.array([0.4, 0.0, 0.0])
    mu1 = g.uniform(0.05, 1.5, k)
    mu2 = g.uniform(0.05, 1.5, k)
    return ls, mu1, mu2


def test_projection_is_closest_point_by_brute_force():
    ls, mu1, mu2 = _cases(300, 0)
    lam, br = project_strict_aniso(ls, mu1, mu2)
    th = np.linspace(0, 2 * np.pi, 400001)
    counts = np.bincount(br, minlength=3)
    assert np.all(counts > 20), counts
    for m in range(ls.shape[0]):
        if ls[m, 0] <= 0:
            assert br[m] == BRANCH_OPEN and np.all(lam[m] == 0)
            continue
        a, b = mu1[m] * ls[m, 0], mu2[m] * ls[m, 0]
        y = ls[m, 1:]
        x = lam[m, 1:]
        assert lam[m, 0] == ls[m, 0]
        assert (x[0] / a) ** 2 + (x[1] / b) ** 2 <= 1 + 1e-12
        if br[m] == BRANCH_STICK:
            assert np.array_equal(x, y)
            continue
        pts = np.stack([a * np.cos(th), b * np.sin(th)], 1)
        dmin = np.sqrt(((pts - y) ** 2).sum(1)).min()
        d = np.linalg.norm(x - y)
        assert d <= dmin + 1e-9 * (1 + dmin) and d >= dmin - 1e-6 * (1 + dmin)
        # Lagrange condition: y - x along the outward normal (x1/a^2, x2/b^2)
        nrm = np.array([x[0] / a ** 2, x[1] / b ** 2])
        cross = (y - x)[0] * nrm[1] - (y - x)[1] * nrm[0]
        assert abs(cross) <= 1e-9 * np.linalg.norm(y - x) * np.linalg.norm(nrm)
        assert (y - x) @ nrm > 0


def test_isotropic_special_case_is_the_disk_projection():
    ls, mu1, _ = _cases(200, 1)
    a, ba = project_strict_aniso(ls, mu1, mu1)
    d, bd = project_strict(ls, mu1)
    np.testing.assert_allclose(a, d, rtol=0, atol=1e-14 * np.abs(ls).max())
    assert np.array_equal(ba, bd)


def test_degenerate_axis_is_a_segment():
    ls = np.array([[1.0, 0.7, 0.3], [1.0, 0.2, -2.0], [2.0, 0.0, 0.1]])
    lam, br = project_strict_aniso(ls, np.array([0.0, 0.5, 0.0]), np.array([0.4, 0.0, 0.2]))
    np.testing.assert_array_equal(lam, [[1.0, 0.0, 0.3], [1.0, 0.2, 0.0], [2.0, 0.0, 0.1]])
    assert br.tolist() == [BRANCH_SLIP, BRANCH_SLIP, BRANCH_STICK]


def test_mdp_objective_minimal_at_projection():
    """Prop. 6: with lambda_n fixed by the Signorini part, the MDP cost
    gamma/2 |lambda_t|^2 + lambda_t . eta_t over the ellipse is smallest at the
    strict projection of lambda*_t = -eta_t / gamma."""
    g = np.random.default_rng(4)
    th = np.linspace(0, 2 * np.pi, 200001)
    for _ in range(100):
        gamma = g.uniform(0.1, 3.0)
        eta = g.normal(size=3)
        ls = -eta / gamma
        ls[0] = abs(ls[0]) + 0.1
        mu1, mu2 = g.uniform(0.05, 1.5, 2)
        lam, br = project_strict_aniso(ls[None], np.array([mu1]), np.array([mu2]))
        a, b = mu1 * ls[0], mu2 * ls[0]
        r = np.sqrt(g.uniform(0, 1, 20000))
        ph = g.uniform(0, 2 * np.pi, 20000)
        cand = np.concatenate([np.stack([a * np.cos(th), b * np.sin(th)], 1),
                               np.stack([a * r * np.cos(ph), b * r * np.sin(ph)], 1)])
        cost = 0.5 * gamma * (cand ** 2).sum(1) + cand @ (-gamma * ls[1:])
        x = lam[0, 1:]
        c0 = 0.5 * gamma * x @ x + x @ (-gamma * ls[1:])
        assert c0 <= cost.min() + 1e-10 * (1 + abs(cost.min()))


def test_particle_slides_along_the_projection_not_against_the_slip():
    """One particle on a horizontal plane, W = 1/m: one sweep is exact, the
    impulse is the ellipse projection of -m v_t; with mu1 != mu2 it is not
    opposite to the slip direction (the figure of Sec. III-E)."""
    m, h, g = 1.5, 0.01, 9.81
    vk = np.array([[1.0, 1.0, 0.0]])
    p = scenes.inclined_plane_particles([0.0], [0.2], mass=m, h=h, g=g, v_k=vk, mu2=np.array([0.8]))
    r = oracle.vfpi(p, max_iters=3, fixed_iters=True, w_mode="scalar", alpha_user=1 / m, history=True)
    R = p.R[0]
    vf = vk[0] + h * np.array([0.0, 0.0, -g])
    ls = -m * (R @ vf)
    lam_exp, br = project_strict_aniso(ls[None], np.array([0.2]), np.array([0.8]))
    np.testing.assert_allclose(r["lam"][0], lam_exp[0], atol=1e-14)
    assert br[0] == BRANCH_SLIP and r["history"][1] <= 1e-15
    v = r["v"]
    slip_t = (R @ v)[1:]
    fric = r["lam"][0, 1:]
    cosang = fric @ slip_t / (np.linalg.norm(fric) * np.linalg.norm(slip_t))
    assert cosang > -0.99  # not antiparallel
    # isotropic control: antiparallel
    p_iso = scenes.inclined_plane_particles([0.0], [0.5], mass=m, h=h, g=g, v_k=vk)
    ri = oracle.vfpi(p_iso, max_iters=3, fixed_iters=True, w_mode="scalar", alpha_user=1 / m)
    st, fr = (p_iso.R[0] @ ri["v"])[1:], ri["lam"][0, 1:]
    assert fr @ st / (np.linalg.norm(fr) * np.linalg.norm(st)) < -1 + 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_aniso_prop4_surrogate_scc_each_sweep(seed):
    """Prop. 4 with the elliptic cone: after each sweep lambda is in the cone
    and u_n lambda_n = 0, and in slip the friction is the closest point to
    lambda* (so u_t = gamma (lambda_t - lambda*_t) is along the ellipse normal)."""
    p = scenes.random_problem(30, 12, seed, degree=4.0, phi_scale=0.5)
    g = np.random.default_rng(seed)
    p.mu2 = g.uniform(0.05, 1.2, p.n_contacts)
    J = oracle.contact_jacobian(p)
    for L in range(1, 6):
        r = oracle.vfpi(p, max_iters=L, fixed_iters=True)
        u = (J @ r["v"]).reshape(-1, 3)
        u[:, 0] += p.phi
        lam = r["lam"]
        sc = 1e-12 * (1 + np.abs(u).max() + np.abs(lam).max())
        assert np.all(np.abs(lam[:, 0] * u[:, 0]) <= sc * (1 + np.abs(lam[:, 0])))
        for m in range(p.n_contacts):
            if r["branch"][m] == BRANCH_OPEN:
                continue
            a, b = p.mu[m] * lam[m, 0], p.mu2[m] * lam[m, 0]
            assert (lam[m, 1] / a) ** 2 + (lam[m, 2] / b) ** 2 <= 1 + 1e-10
            if r["branch"][m] == BRANCH_SLIP:
                nrm = np.array([lam[m, 1] / a ** 2, lam[m, 2] / b ** 2])
                ut = u[m, 1:]
                assert abs(ut[0] * nrm[1] - ut[1] * nrm[0]) <= 1e-8 * (np.linalg.norm(ut) * np.linalg.norm(nrm) + sc)
                assert ut @ nrm <= sc
