"""Pins of the step-size matrix W (Sec. IV-C.1) and of Prop. 3 (contact
diagonalization): checked against a generic minimizer and an explicit dense
product, not against the oracle's own formulas."""
import numpy as np
import scipy.optimize as so

import scenes
from oracle import contact_jacobian, frobenius_w, row_stats, surrogate_delassus, system_matrix
from oracle.core import contact_gamma, contact_groups


def _small(n_d=0, seed=0):
    return scenes.random_problem(9, 3 + n_d, seed, degree=4.0, n_d_contacts=n_d)


def test_frobenius_w_minimizes_frobenius_norm_generic_optimizer():
    p = _small(n_d=1, seed=5)
    A = system_matrix(p).toarray()
    n = p.n
    lab = contact_groups(p)
    # parametrize W by one value per free DOF and one per contact group
    groups = {}
    for node in range(p.n_nodes):
        for d in range(3):
            key = ("g", lab[node]) if lab[node] >= 0 else ("d", 3 * node + d)
            groups.setdefault(key, []).append(3 * node + d)
    keys = list(groups)

    def fro(theta):
        w = np.zeros(n)
        for k, t in zip(keys, theta):
            w[groups[k]] = t
        return np.sum((np.eye(n) - np.diag(w) @ A) ** 2)

    res = so.minimize(fro, np.full(len(keys), 0.1), method="BFGS", options={"gtol": 1e-12})
    w_opt = np.zeros(n)
    for k, t in zip(keys, res.x):
        w_opt[groups[k]] = t
    w = frobenius_w(p, *row_stats(system_matrix(p)))
    np.testing.assert_allclose(w, w_opt, rtol=1e-6)
    # equal entries on each contact node (the condition of Prop. 3)
    for m in range(p.n_contacts):
        i = p.c_node[m]
        assert np.ptp(w[3 * i:3 * i + 3]) == 0


def test_prop3_dense_product_is_diagonal():
    """J_c W J_c^T formed densely equals diag(gamma_m I_3), gamma = w_i (S) or
    w_i + w_j (D), for random orthonormal frames."""
    for seed in range(4):
        p = _small(n_d=2, seed=seed)
        w = frobenius_w(p, *row_stats(system_matrix(p)))
        J = contact_jacobian(p).toarray()
        G = J @ np.diag(w) @ J.T
        gam = contact_gamma(p, w)
        np.testing.assert_allclose(G, np.kron(np.diag(gam), np.eye(3)), rtol=0, atol=1e-15 * gam.max() * 8)
        sd = surrogate_delassus(contact_jacobian(p), w).toarray()
        np.testing.assert_allclose(sd, G, atol=1e-15 * gam.max() * 8)


def test_prop3_needs_equal_node_entries():
    """With unequal entries on a contact node Gamma is not diagonal: the
    condition of Prop. 3 is what the diagonalization rests on."""
    p = _small(seed=1)
    w = frobenius_w(p, *row_stats(system_matrix(p)))
    i = p.c_node[0]
    w[3 * i] *= 1.5
    J = contact_jacobian(p).toarray()
    G = J @ np.diag(w) @ J.T
    off = G[:3, :3] - np.diag(np.diag(G[:3, :3]))
    assert np.abs(off).max() > 1e-6 * w.max()
