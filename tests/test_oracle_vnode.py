"""Pins of the virtual-node formulation (eq. vforce, eq. vnode): Prop. 1
(the augmented matrix is SPD), eq. vnode3 at a solution (no extra force on
the original system), and Prop. 2 on the sliding box, whose contact error
against the closed-form solution falls like 1 / k_v."""
import numpy as np
import pytest

import oracle
import scenes
from oracle.delassus import pgs
from oracle.vnode import augment, augmented_matrix, jv_matrix


def _box_exact(vs):
    """Sliding box from rest under a horizontal force F > mu m g at its
    centre: no rotation, no vertical motion, v_y = h (F / m - mu g)."""
    m, h, g, mu, F = (vs.meta[k] for k in ("mass", "h", "g", "mu", "force"))
    assert F[1] > mu * m * g
    return np.array([0.0, h * (F[1] / m - mu * g), 0.0, 0.0, 0.0, 0.0])


@pytest.mark.parametrize("k_v", [1.0, 1e3, 1e6])
def test_prop1_augmented_matrix_spd(k_v):
    for vs in (scenes.rigid_box_on_floor(), scenes.particles_on_cloth(0)):
        A = augmented_matrix(vs, k_v).toarray()
        assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
        assert np.linalg.eigvalsh(A).min() > 0


def test_vnode3_no_additional_force():
    """At a solution, A_o v_o = b_o + J_v^T J_cv^T lambda_cv + J_co^T lambda_co:
    the tie only transmits the contact impulses (eq. vnode3)."""
    vs = scenes.particles_on_cloth(1)
    p = augment(vs, 1.0)
    r = oracle.vfpi(p, max_iters=200000, tol=1e-14)
    n3 = 3 * vs.n_o
    Ao = augmented_matrix(vs, 0.0)[:n3, :n3]
    J = oracle.contact_jacobian(p)
    f = J.T @ r["lam"].ravel()
    rhs = vs.b + f[:n3] + jv_matrix(vs).T @ f[n3:]
    res = Ao @ r["v"][:n3] - rhs
    assert np.abs(res).max() <= 1e-9 * np.abs(vs.b).max()
    assert np.abs(f[n3:]).max() > 1e-4  # particles do hit the cloth


def test_prop2_box_error_falls_like_one_over_kv():
    vs = scenes.rigid_box_on_floor()
    exact = _box_exact(vs)
    errs = []
    for k_v in (1e2, 1e3, 1e4, 1e5):
        p = augment(vs, k_v)
        q = pgs(p, tol=1e-15, max_sweeps=200000)
        errs.append(np.abs(q["v"][:6] - exact).max())
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 7) and np.all(ratios < 13), (errs, ratios)
    assert errs[-1] < 1e-6


def test_box_vfpi_matches_pgs_on_augmented_system():
    vs = scenes.rigid_box_on_floor()
    p = augment(vs, 10.0)
    r = oracle.vfpi(p, max_iters=500000, tol=1e-14)
    q = pgs(p, tol=1e-15, max_sweeps=200000)
    np.testing.assert_allclose(r["v"], q["v"], atol=1e-9)
