"""Pins of the oracle adjoint of a converged V-FPI step: the transposed
fixed-point solve against a dense LU, central finite differences of the
converged forward, W-independence, and the sliding particle's closed form."""
import numpy as np
import pytest

import oracle
import scenes
from oracle.adjoint import adjoint, adjoint_dense


def _fwd(p, **kw):
    kw.setdefault("max_iters", 200000)
    kw.setdefault("tol", 1e-15)
    return oracle.vfpi(p, **kw)


def _problem(seed):
    return scenes.random_problem(14, 7, seed, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), tag="adj")


@pytest.mark.parametrize("seed,projection", [(0, "strict"), (1, "strict"), (2, "strict"), (0, "proximal"),
                                             (2, "proximal")])
def test_iterative_adjoint_matches_dense(seed, projection):
    p = _problem(seed)
    f = _fwd(p, projection=projection)
    g = np.random.default_rng(seed)
    gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
    a = adjoint(p, f, gv, gl)
    d = adjoint_dense(p, f, gv, gl)
    for k in ("b", "A", "phi", "mu"):
        np.testing.assert_allclose(a[k], d[k], rtol=0, atol=1e-10 * (1 + np.abs(d[k]).max()))


def _loss(p, gv, gl, omega=0.0, projection="strict"):
    f = _fwd(p, omega=omega, projection=projection)
    return gv @ f["v"] + gl @ f["lam"].ravel(), f["branch"]


@pytest.mark.parametrize("seed,omega,projection", [(0, 0.0, "strict"), (1, 0.0, "strict"), (2, 0.0, "strict"),
                                                   (0, 0.02, "strict"), (1, 0.3, "strict"),
                                                   (0, 0.0, "proximal"), (1, 0.02, "proximal"),
                                                   (2, 0.3, "proximal")])
def test_adjoint_matches_central_differences(seed, omega, projection):
    """With omega > 0 (invertible contact, eq. invt) the same adjoint applies
    with gamma + omega in the contact step; with the proximal operator D_P is
    the cone projection's Jacobian."""
    p = _problem(seed)
    f = _fwd(p, omega=omega, projection=projection)
    g = np.random.default_rng(100 + seed)
    gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
    grad = adjoint(p, f, gv, gl)
    eps = 1e-6
    checked = 0

    def fd(make):
        lp, bp = _loss(make(+eps), gv, gl, omega, projection)
        lm, bm = _loss(make(-eps), gv, gl, omega, projection)
        if not (np.array_equal(bp, f["branch"]) and np.array_equal(bm, f["branch"])):
            return None  # the active set changed inside +-eps: not differentiable there
        return (lp - lm) / (2 * eps)

    def with_(name, arr):
        return scenes.Problem(**{**p.__dict__, name: arr})

    for k in g.choice(p.n, 6, replace=False):
        e = np.zeros(p.n)
        e[k] = 1
        val = fd(lambda s: with_("b", p.b + s * e))
        if val is not None:
            assert abs(val - grad["b"][k]) <= 1e-6 * (1 + abs(val))
            checked += 1
    for m in range(p.n_contacts):
        e = np.zeros(p.n_contacts)
        e[m] = 1
        for name in ("phi", "mu"):
            val = fd(lambda s: with_(name, getattr(p, name) + s * e))
            if val is not None:
                assert abs(val - grad[name][m]) <= 1e-6 * (1 + abs(val)), (name, m)
                checked += 1
    # symmetric perturbation of one off-diagonal block pair of A
    rows = np.repeat(np.arange(p.n_nodes), np.diff(p.row_ptr))
    offd = np.nonzero(rows != p.col_idx)[0]
    for blk in g.choice(offd, 3, replace=False):
        i, c = rows[blk], p.col_idx[blk]
        tr = p.row_ptr[c] + np.nonzero(p.col_idx[p.row_ptr[c]:p.row_ptr[c + 1]] == i)[0][0]
        E = np.zeros_like(p.val)
        E[blk, 0, 1] = 1
        E[tr, 1, 0] = 1
        val = fd(lambda s: with_("val", p.val + s * E))
        if val is not None:
            exp = grad["A"][blk, 0, 1] + grad["A"][tr, 1, 0]
            assert abs(val - exp) <= 1e-6 * (1 + abs(val))
            checked += 1
    assert checked >= 10


@pytest.mark.parametrize("projection", ["strict", "proximal"])
def test_gradient_independent_of_w(projection):
    p = _problem(3)
    g = np.random.default_rng(7)
    gv = g.normal(size=p.n)
    f1 = _fwd(p, projection=projection)
    alpha = oracle.core.gershgorin_alpha(oracle.system_matrix(p))
    f2 = _fwd(p, w_mode="scalar", alpha_user=alpha, projection=projection)
    a1, a2 = adjoint(p, f1, gv), adjoint(p, f2, gv)
    for k in ("b", "phi", "mu"):
        np.testing.assert_allclose(a1[k], a2[k], atol=1e-8 * (1 + np.abs(a1[k]).max()))


def test_sliding_particle_closed_form():
    """x_N . t = h^2 g (sin a - mu cos a) N (N+1) / 2 for a particle sliding from
    rest, so dL/dmu = -h^2 g cos(a) N (N+1) / 2 with L = t . x_N."""
    a, mu, m, h, g, N = 0.5, 0.2, 1.3, 0.01, 9.81, 20
    t_dir = np.array([np.cos(a), 0.0, -np.sin(a)])
    v = np.zeros(3)
    steps = []
    for _ in range(N):
        p = scenes.inclined_plane_particles([a], [mu], mass=m, h=h, g=g, v_k=v[None])
        f = _fwd(p)
        steps.append((p, f))
        v = f["v"]
    # reverse sweep: L = t . x_N, x_k = x_{k-1} + h v_k, b_{k+1} = m (v_k + h g)
    mu_bar = 0.0
    v_bar_next_b = np.zeros(3)
    for p, f in reversed(steps):
        gv = h * t_dir + m * v_bar_next_b
        ad = adjoint(p, f, gv)
        mu_bar += ad["mu"][0]
        v_bar_next_b = ad["b"]
    np.testing.assert_allclose(mu_bar, -h * h * g * np.cos(a) * N * (N + 1) / 2, rtol=1e-10)


def test_proximal_projection_jacobian_vs_differences():
    """D_P and dP/dmu of the cone projection (proximal operator) against
    central differences of oracle.core.project_proximal, on points well
    inside each branch."""
    from oracle.adjoint import projection_jacobians
    from oracle.core import project_proximal
    g = np.random.default_rng(11)
    pts, mus = [], []
    while len(pts) < 60:
        mu = g.uniform(0.1, 1.5)
        ls = g.normal(size=3)
        s = np.hypot(ls[1], ls[2])
        # stay away from the branch boundaries s = mu n and mu s = -n
        if abs(s - mu * ls[0]) < 0.05 or abs(mu * s + ls[0]) < 0.05 or s < 0.05:
            continue
        pts.append(ls)
        mus.append(mu)
    lam_star, mu = np.array(pts), np.array(mus)
    _, branch = project_proximal(lam_star, mu)
    assert set(branch.tolist()) == {0, 1, 2}
    DP, dmu, _ = projection_jacobians(lam_star, branch, mu, "proximal")
    eps = 1e-7
    for k in range(3):
        e = np.zeros(3)
        e[k] = eps
        num = (project_proximal(lam_star + e, mu)[0] - project_proximal(lam_star - e, mu)[0]) / (2 * eps)
        np.testing.assert_allclose(DP[:, :, k], num, atol=1e-7)
    num = (project_proximal(lam_star, mu + eps)[0] - project_proximal(lam_star, mu - eps)[0]) / (2 * eps)
    np.testing.assert_allclose(dmu, num, atol=1e-7)


def test_ellipse_projection_jacobian_vs_differences():
    """D_P, dP/dmu1 and dP/dmu2 of the strict operator on the elliptic cone
    (anisotropic friction) against central differences of
    oracle.core.project_strict_aniso, on points well inside each branch; and
    at mu1 = mu2 the ellipse Jacobian equals the disk's."""
    from oracle.adjoint import ellipse_jacobian, projection_jacobians
    from oracle.core import project_strict_aniso
    g = np.random.default_rng(12)
    pts, m1, m2 = [], [], []
    while len(pts) < 40:
        a1, a2 = g.uniform(0.2, 1.2, size=2)
        ls = g.normal(size=3)
        if ls[0] < 0.1 and ls[0] > -0.1:
            continue
        q = (ls[1] / (a1 * ls[0])) ** 2 + (ls[2] / (a2 * ls[0])) ** 2 if ls[0] > 0 else 9.0
        if abs(q - 1.0) < 0.1:   # near the ellipse boundary: branch may flip under +-eps
            continue
        pts.append(ls)
        m1.append(a1)
        m2.append(a2)
    lam_star, mu1, mu2 = np.array(pts), np.array(m1), np.array(m2)
    _, branch = project_strict_aniso(lam_star, mu1, mu2)
    assert set(branch.tolist()) == {0, 1, 2}
    DP, dmu1, dmu2 = projection_jacobians(lam_star, branch, mu1, "strict", mu2)
    eps = 1e-7
    for k in range(3):
        e = np.zeros(3)
        e[k] = eps
        num = (project_strict_aniso(lam_star + e, mu1, mu2)[0] - project_strict_aniso(lam_star - e, mu1, mu2)[0]) / (2 * eps)
        np.testing.assert_allclose(DP[:, :, k], num, atol=2e-7)
    num = (project_strict_aniso(lam_star, mu1 + eps, mu2)[0] - project_strict_aniso(lam_star, mu1 - eps, mu2)[0]) / (2 * eps)
    np.testing.assert_allclose(dmu1, num, atol=2e-7)
    num = (project_strict_aniso(lam_star, mu1, mu2 + eps)[0] - project_strict_aniso(lam_star, mu1, mu2 - eps)[0]) / (2 * eps)
    np.testing.assert_allclose(dmu2, num, atol=2e-7)
    # a zero coefficient (segment): the clamp's Jacobian, on both tangents
    for za, zb in ((0.0, 0.8), (0.6, 0.0)):
        pts = np.array([[0.9, 0.3, 1.5], [0.9, 1.2, -0.2], [0.5, -2.0, 0.1], [1.1, 0.2, -0.05]])
        m1, m2 = np.full(4, za), np.full(4, zb)
        _, br = project_strict_aniso(pts, m1, m2)
        assert (br == 2).all()
        DP, d1, d2 = projection_jacobians(pts, br, m1, "strict", m2)
        for k in range(3):
            e = np.zeros(3)
            e[k] = eps
            num = (project_strict_aniso(pts + e, m1, m2)[0] - project_strict_aniso(pts - e, m1, m2)[0]) / (2 * eps)
            np.testing.assert_allclose(DP[:, :, k], num, atol=2e-7)
        # derivatives in mu: central for the nonzero coefficient, one-sided
        # (mu >= 0) for the zero one
        h = 1e-9

        def dproj(d1, d2):
            return (project_strict_aniso(pts, m1 + d1, m2 + d2)[0] - project_strict_aniso(pts, m1 - d1 * (za > 0),
                                                                                      m2 - d2 * (zb > 0))[0])
        num1 = dproj(h, 0.0) / (h * (1 + (za > 0)))
        num2 = dproj(0.0, h) / (h * (1 + (zb > 0)))
        np.testing.assert_allclose(d1, num1, atol=1e-6)
        np.testing.assert_allclose(d2, num2, atol=1e-6)
    # circle: the disk operator's Jacobian, and dP/dmu1 + dP/dmu2 = dP/dmu of the disk
    ls = np.array([[0.7, 1.1, -0.4]])
    DPd, dmud, _ = projection_jacobians(ls, np.array([2]), np.array([0.5]))
    DPe, d1, d2 = ellipse_jacobian(0.7, ls[0, 1:], 0.5, 0.5)
    np.testing.assert_allclose(DPe, DPd[0], atol=1e-12)
    np.testing.assert_allclose(d1 + d2, dmud[0], atol=1e-12)


@pytest.mark.parametrize("seed", [0, 2, 7])
def test_anisotropic_adjoint_matches_central_differences(seed):
    """The adjoint with the elliptic cone: b, phi, mu1 and mu2 gradients of a
    converged step against central differences; the dense solve agrees."""
    p = _problem(seed)
    p.mu2 = np.asarray(p.mu) * np.random.default_rng(seed).uniform(0.3, 1.8, size=p.n_contacts)
    f = _fwd(p)
    assert (f["branch"] == 2).sum() >= 2
    g = np.random.default_rng(200 + seed)
    gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
    grad = adjoint(p, f, gv, gl)
    dense = adjoint_dense(p, f, gv, gl)
    for k in ("b", "phi", "mu", "mu2"):
        np.testing.assert_allclose(grad[k], dense[k], rtol=0, atol=1e-9 * (1 + np.abs(dense[k]).max()))
    eps = 1e-6
    checked = 0

    def fd(name, arr_p, arr_m):
        out = []
        for arr in (arr_p, arr_m):
            q = scenes.Problem(**{**p.__dict__, name: arr})
            fq = _fwd(q)
            if not np.array_equal(fq["branch"], f["branch"]):
                return None
            out.append(gv @ fq["v"] + gl @ fq["lam"].ravel())
        return (out[0] - out[1]) / (2 * eps)

    for k in g.choice(p.n, 5, replace=False):
        e = np.zeros(p.n)
        e[k] = eps
        val = fd("b", p.b + e, p.b - e)
        if val is not None:
            assert abs(val - grad["b"][k]) <= 1e-6 * (1 + abs(val))
            checked += 1
    for m in range(p.n_contacts):
        e = np.zeros(p.n_contacts)
        e[m] = eps
        for name in ("phi", "mu", "mu2"):
            base = np.asarray(getattr(p, name))
            val = fd(name, base + e, base - e)
            if val is not None:
                assert abs(val - grad[name][m]) <= 1e-6 * (1 + abs(val)), (name, m, val, grad[name][m])
                checked += 1
    assert checked >= 10


def test_anisotropic_adjoint_zero_coefficient_one_sided():
    """With one friction coefficient zero (the elliptic cone flattens to a
    segment) the adjoint's gradient in that coefficient is the one-sided
    derivative of the converged step (mu >= 0), the others central."""
    p = scenes.random_problem(30, 14, 2, degree=4.0, phi_scale=0.4, mu_range=(0.2, 0.9), tag="adj")
    mu, mu2 = np.array(p.mu, dtype=np.float64), np.array(p.mu, dtype=np.float64) * 0.6
    mu[::3] = 0.0
    mu2[1::3] = 0.0
    p.mu, p.mu2 = mu, mu2
    f = _fwd(p)
    zero_slip = ((mu == 0) | (mu2 == 0)) & (f["branch"] == 2)
    assert zero_slip.sum() >= 3
    g = np.random.default_rng(21)
    gv, gl = g.normal(size=p.n), g.normal(size=3 * p.n_contacts)
    grad = adjoint(p, f, gv, gl)
    dense = adjoint_dense(p, f, gv, gl)
    for k in ("b", "phi", "mu", "mu2"):
        np.testing.assert_allclose(grad[k], dense[k], rtol=0, atol=1e-9 * (1 + np.abs(dense[k]).max()))

    def loss(**kw):
        q = scenes.Problem(**{**p.__dict__, **kw})
        fq = _fwd(q)
        return gv @ fq["v"] + gl @ fq["lam"].ravel(), fq["branch"]

    L0, _ = loss()
    checked = 0
    for m in np.nonzero(zero_slip)[0]:
        for name in ("mu", "mu2"):
            base = np.asarray(getattr(p, name))
            e = np.zeros(p.n_contacts)
            if base[m] == 0.0:
                h = 1e-8
                e[m] = h
                Lp, br = loss(**{name: base + e})
                if not np.array_equal(br, f["branch"]):
                    continue
                val = (Lp - L0) / h
                assert abs(val - grad[name][m]) <= 1e-5 * (1 + abs(val)), (name, m, val, grad[name][m])
            else:
                h = 1e-6
                e[m] = h
                (Lp, bp), (Lm, bm) = loss(**{name: base + e}), loss(**{name: base - e})
                if not (np.array_equal(bp, f["branch"]) and np.array_equal(bm, f["branch"])):
                    continue
                val = (Lp - Lm) / (2 * h)
                assert abs(val - grad[name][m]) <= 1e-6 * (1 + abs(val)), (name, m, val, grad[name][m])
            checked += 1
    assert checked >= 4
