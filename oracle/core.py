"""V-FPI oracle: plain float64 NumPy/SciPy, test infrastructure only.

Follows the paper step by step:

* problem  A v = b + J_c^T lambda  with SCC per contact        (Sec. II, eq. lindyn, eq. scc)
* nodal contact Jacobian, one SO(3) block (S) or R, -R (D)     (Sec. III-A, eq. jcnode)
* step-size matrix W, Frobenius-norm minimizing diagonal        (Sec. IV-C.1)
  with equal entries on each contact node (3 DOFs; 6 for a D pair)
* surrogate Delassus operator Gamma = J_c W J_c^T = diag(gamma I) (Sec. III-C, Prop. 3)
* V-FPI sweep: v* = v - W (A v - b)                            (eq. pgd1)
               eta = J_c v*                                     (eq. subp)
               lambda* = -(eta + phi e1) / gamma; ProjectFC     (Alg. 2, eq. operator)
               v^{l+1} = v* + W J_c^T lambda                    (eq. vup)
               theta = ||v^{l+1} - v^l||_2, stop if < tol or l = l_max  (Alg. 1)

The sparse products A v, J v, J^T lambda are SciPy library matvecs.

Readings where the paper is silent (each also listed in the design notes):
* theta is the absolute 2-norm over all DOFs; ``iters`` is l at the break.
* strict projection ties: lambda*_n <= 0 gives lambda = 0 (open);
  ||lambda*_t|| <= mu lambda_n is stick; no division when ||lambda*_t|| = 0.
* the printed expansion of ||I - WA||_F^2 drops a factor 2 and a square
  (Sec. IV-C.1); the minimizers printed after it are the ones of the correct
  expansion n - 2 sum w_ii a_ii + sum w_ii^2 ||A_i*||^2 and are used as printed.
* Barzilai-Borwein (Sec. IV-C.2): alpha^1 = 1 / max_i sum_j |a_ij| (Gershgorin),
  alpha^l for l >= 2 from s = v^l - v^{l-1}, z = A v^l - A v^{l-1}; the previous
  alpha is kept when s^T s = 0, s^T z <= 0 (or z^T z = 0 for BB2).

Pins (tests/test_oracle_*.py): closed-form projections; Prop. 3 by a dense
product; Frobenius W by a generic minimizer; n_c = 0 against a Cholesky solve;
the inclined-plane particle (analytic stick/slip); Prop. 4 per sweep; PGS and
mode enumeration on the Delassus form at convergence.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

BRANCH_OPEN, BRANCH_STICK, BRANCH_SLIP = 0, 1, 2


def system_matrix(p) -> sp.csr_matrix:
    """A (n x n) from its 3x3 block rows."""
    return sp.bsr_matrix((p.val, p.col_idx, p.row_ptr), shape=(p.n, p.n)).tocsr()


def contact_jacobian(p) -> sp.csr_matrix:
    """J_c (3 n_c x n), eq. jcnode: block row m holds R_m at node i and, for a
    D-contact, -R_m at node j."""
    nc = p.n_contacts
    a, bb = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")
    rows = (3 * np.arange(nc)[:, None, None] + a[None]).ravel()
    cols = (3 * p.c_node[:, None, None].astype(np.int64) + bb[None]).ravel()
    vals = p.R.ravel()
    d = np.nonzero(p.c_node_j >= 0)[0]
    if d.size:
        rows = np.concatenate([rows, (3 * d[:, None, None] + a[None]).ravel()])
        cols = np.concatenate([cols, (3 * p.c_node_j[d][:, None, None].astype(np.int64) + bb[None]).ravel()])
        vals = np.concatenate([vals, -p.R[d].ravel()])
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * nc, p.n))


class InvalidProblem(ValueError):
    def __init__(self, code, msg):
        super().__init__(f"{code}: {msg}")
        self.code = code


def validate(p, A=None, sym_tol=1e-12, orth_tol=1e-10):
    """The preconditions of the method: A symmetric with a positive diagonal
    (SPD, Sec. II-A); R_m orthonormal (eq. jcnode, used by Prop. 3); at most one
    contact per node (otherwise Gamma is not diagonal, Prop. 3); finite data."""
    A = system_matrix(p) if A is None else A
    for name in ("val", "b", "v0", "R", "phi", "mu"):
        if not np.all(np.isfinite(getattr(p, name))):
            raise InvalidProblem("NONFINITE", name)
    if np.any(A.diagonal() <= 0):
        raise InvalidProblem("NONPOS_DIAG", "a_ii <= 0")
    asym = abs(A - A.T).max() if A.nnz else 0.0
    if asym > sym_tol * max(abs(A).max(), 1e-300):
        raise InvalidProblem("NOT_SYMMETRIC", f"max |A - A^T| = {asym}")
    if p.n_contacts:
        err = np.abs(p.R @ p.R.transpose(0, 2, 1) - np.eye(3)).max()
        if err > orth_tol:
            raise InvalidProblem("NOT_ORTHONORMAL", f"max |R R^T - I| = {err}")
        nodes = np.concatenate([p.c_node, p.c_node_j[p.c_node_j >= 0]])
        if np.unique(nodes).shape[0] != nodes.shape[0]:
            raise InvalidProblem("SHARED_NODE", "a node is in more than one contact")
        if np.any(p.mu < 0):
            raise InvalidProblem("NEGATIVE_MU", "mu < 0")
    return A


def row_stats(A):
    """a_dd and ||A_d*||^2 per DOF (the two sums the Frobenius W needs)."""
    return A.diagonal().copy(), np.asarray(A.multiply(A).sum(axis=1)).ravel()


def contact_groups(p):
    """Group label per node: nodes joined by a contact (its node, or both
    nodes of a D pair, chained D pairs merged) share a label; -1 = no contact."""
    parent = np.arange(p.n_nodes)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for i, j in zip(p.c_node, p.c_node_j):
        if j >= 0:
            ri, rj = find(i), find(j)
            if ri != rj:
                parent[max(ri, rj)] = min(ri, rj)
    label = np.full(p.n_nodes, -1, dtype=np.int64)
    for i, j in zip(p.c_node, p.c_node_j):
        label[i] = find(i)
        if j >= 0:
            label[j] = find(j)
    return label


def frobenius_w(p, diag, rn2):
    """Diagonal W minimizing ||I - W A||_F (Sec. IV-C.1): w_dd = a_dd / ||A_d*||^2
    for DOFs of nodes without contact; one shared value
    sum_{d in G} a_dd / sum_{d in G} ||A_d*||^2 over the DOFs G of each contact
    group (3 DOFs for an S-contact node, 6 for a D pair)."""
    w = diag / rn2
    label = contact_groups(p)
    nodes = np.nonzero(label >= 0)[0]
    if nodes.size:
        dofs = (3 * nodes[:, None] + np.arange(3)).ravel()
        glab = np.repeat(label[nodes], 3)
        uniq, inv = np.unique(glab, return_inverse=True)
        num = np.bincount(inv, weights=diag[dofs], minlength=uniq.shape[0])
        den = np.bincount(inv, weights=rn2[dofs], minlength=uniq.shape[0])
        w[dofs] = (num / den)[inv]
    return w


def contact_gamma(p, w):
    """gamma_m of Prop. 3: w-bar of the contact node (S) or the sum of both
    nodes' w-bar (D)."""
    g = w[3 * p.c_node.astype(np.int64)].copy()
    d = p.c_node_j >= 0
    g[d] += w[3 * p.c_node_j[d].astype(np.int64)]
    return g


def surrogate_delassus(J, w):
    """Gamma_c = J_c W J_c^T (eq. subp), formed explicitly."""
    return (J @ sp.diags(w) @ J.T).tocsr()


def project_strict(lam_star, mu):
    """Strict ProjectFC (eq. operator): lambda_n = max(lambda*_n, 0), lambda_t =
    Euclidean projection of lambda*_t onto the disk of radius mu lambda_n.
    ``lam_star`` [m,3] = (n, t1, t2).  Returns (lambda [m,3], branch [m])."""
    lam_star = np.asarray(lam_star, dtype=np.float64)
    ln = np.maximum(lam_star[:, 0], 0.0)
    t = lam_star[:, 1:]
    s = np.sqrt(t[:, 0] ** 2 + t[:, 1] ** 2)
    rad = mu * ln
    inside = s <= rad
    scale = np.where(inside, 1.0, rad / np.where(s > 0, s, 1.0))
    lam = np.concatenate([ln[:, None], t * scale[:, None]], axis=1)
    branch = np.where(lam_star[:, 0] <= 0.0, BRANCH_OPEN, np.where(inside, BRANCH_STICK, BRANCH_SLIP))
    lam[lam_star[:, 0] <= 0.0] = 0.0
    return lam, branch.astype(np.int32)


def project_proximal(lam_star, mu):
    """Proximal ProjectFC (eq. operator): Euclidean projection onto the cone
    {lambda_n >= 0, ||lambda_t|| <= mu lambda_n} (second-order-cone projection)."""
    lam_star = np.asarray(lam_star, dtype=np.float64)
    n = lam_star[:, 0]
    t = lam_star[:, 1:]
    s = np.sqrt(t[:, 0] ** 2 + t[:, 1] ** 2)
    inside = (s <= mu * n) & (n >= 0)
    polar = (~inside) & (mu * s <= -n)
    nn = (n + mu * s) / (1.0 + mu * mu)
    scale = mu * nn / np.where(s > 0, s, 1.0)
    lam = np.concatenate([nn[:, None], t * scale[:, None]], axis=1)
    lam[inside] = lam_star[inside]
    lam[polar] = 0.0
    branch = np.where(polar, BRANCH_OPEN, np.where(inside, BRANCH_STICK, BRANCH_SLIP))
    return lam, branch.astype(np.int32)


def _ellipse_closest(y1, y2, a, b):
    """Closest point to (y1, y2) in the ellipse x1^2/a^2 + x2^2/b^2 <= 1 (a, b
    >= 0; a zero axis makes it a segment).  Outside, the Lagrange condition of
    min |x - y|^2 gives x_i = a_i^2 y_i / (a_i^2 + s) with s > 0 the root of
    sum_i (a_i y_i / (a_i^2 + s))^2 = 1; the left side falls from above 1 at
    s = 0 to at most 1 at s = a |y1| + b |y2|, and brentq brackets it there."""
    if a == 0.0 or b == 0.0:
        x1, x2 = min(max(y1, -a), a), min(max(y2, -b), b)
        return x1, x2, (x1 == y1 and x2 == y2)
    if (y1 * b) ** 2 + (y2 * a) ** 2 <= (a * b) ** 2:
        return y1, y2, True

    s = ellipse_root(y1, y2, a, b)
    return a * a * y1 / (a * a + s), b * b * y2 / (b * b + s), False


def ellipse_root(y1, y2, a, b):
    """The Lagrange multiplier s > 0 of the closest point to (y1, y2) outside
    the ellipse of semi-axes a, b > 0 (see _ellipse_closest)."""
    from scipy.optimize import brentq

    def F(s):
        return (a * y1 / (a * a + s)) ** 2 + (b * y2 / (b * b + s)) ** 2 - 1.0

    return brentq(F, 0.0, a * abs(y1) + b * abs(y2), xtol=1e-300, rtol=4 * np.finfo(float).eps, maxiter=500)


def project_strict_aniso(lam_star, mu1, mu2):
    """Strict ProjectFC for the elliptic friction cone of Sec. III-E
    (anisotropic friction, lambda_n^2 >= t1^2/mu1^2 + t2^2/mu2^2):
    lambda_n = max(lambda*_n, 0) and lambda_t = the closest point to
    lambda*_t in the ellipse of semi-axes mu1 lambda_n, mu2 lambda_n, which is
    the maximal-dissipation solution of the contact's surrogate problem
    (Prop. 6).  Branches as in project_strict."""
    lam_star = np.asarray(lam_star, dtype=np.float64)
    nc = lam_star.shape[0]
    lam = np.zeros((nc, 3))
    branch = np.full(nc, BRANCH_OPEN, dtype=np.int32)
    for m in range(nc):
        n = lam_star[m, 0]
        if n <= 0.0:
            continue
        x1, x2, inside = _ellipse_closest(lam_star[m, 1], lam_star[m, 2], mu1[m] * n, mu2[m] * n)
        lam[m] = (n, x1, x2)
        branch[m] = BRANCH_STICK if inside else BRANCH_SLIP
    return lam, branch


def gershgorin_alpha(A):
    return 1.0 / np.asarray(abs(A).sum(axis=1)).max()


def vfpi(p, *, max_iters=100, tol=0.0, fixed_iters=False, w_mode="frobenius", w_user=None,
         alpha_user=None, projection="strict", stats=None, history=False, omega=0.0):
    """Alg. 1 inner loop (the V-FPI) with Alg. 2 as its contact step.

    ``w_mode``: "frobenius" (Sec. IV-C.1), "diag" (user W, ``w_user``[n],
    equal over each contact group), "scalar" (W = alpha_user I),
    "bb1" / "bb2" (Sec. IV-C.2).  ``stats`` = (a_dd, ||A_d*||^2) reuses the
    row sums of an earlier A (W reuse across steps, Sec. IV-C, last paragraph).
    With ``fixed_iters`` exactly ``max_iters`` sweeps run regardless of ``tol``.
    ``omega`` > 0 is the invertible contact of Sec. III-E (eq. invt) with
    Omega_c = omega I: the surrogate problem uses Gamma_c + Omega_c, i.e. the
    contact step divides by gamma_m + omega.
    """
    A = validate(p)
    J = contact_jacobian(p)
    n, nc = p.n, p.n_contacts
    project = project_strict if projection == "strict" else project_proximal
    mu2 = getattr(p, "mu2", None)
    if mu2 is not None:  # anisotropic friction: strict operator on the elliptic cone
        if projection != "strict":
            raise ValueError("anisotropic friction is defined with the strict operator (Prop. 6)")

        def project(ls, mu1, _mu2=mu2):
            return project_strict_aniso(ls, mu1, _mu2)
    alpha = None
    if w_mode == "frobenius":
        diag, rn2 = row_stats(A) if stats is None else stats
        w = frobenius_w(p, diag, rn2)
    elif w_mode == "diag":
        w = np.asarray(w_user, dtype=np.float64).copy()
        lab = contact_groups(p)
        for gl in np.unique(lab[lab >= 0]):
            dofs = (3 * np.nonzero(lab == gl)[0][:, None] + np.arange(3)).ravel()
            if np.ptp(w[dofs]) != 0.0:
                raise ValueError("user W must be equal over each contact group (Prop. 3)")
    elif w_mode == "scalar":
        alpha = float(alpha_user)
        w = np.full(n, alpha)
    elif w_mode in ("bb1", "bb2"):
        alpha = gershgorin_alpha(A)
        w = np.full(n, alpha)
    else:
        raise ValueError(w_mode)
    if np.any(w <= 0):
        raise ValueError("W must be positive")
    gamma = contact_gamma(p, w) + omega
    phi_e1 = np.zeros(3 * nc)
    phi_e1[0::3] = p.phi
    v = p.v0.copy()
    v_prev = Av_prev = None
    hist = []
    lam = np.zeros((nc, 3))
    lam_star = np.zeros((nc, 3))
    branch = np.zeros(nc, dtype=np.int32)
    theta = np.inf
    it = 0
    for it in range(1, max_iters + 1):
        Av = A @ v
        if w_mode in ("bb1", "bb2") and it >= 2:
            s = v - v_prev
            z = Av - Av_prev
            ss, sz, zz = s @ s, s @ z, z @ z
            if w_mode == "bb1" and ss > 0 and sz > 0:
                alpha = ss / sz
            elif w_mode == "bb2" and sz > 0 and zz > 0:
                alpha = sz / zz
            w = np.full(n, alpha)
            gamma = contact_gamma(p, w) + omega
        vs = v - w * (Av - p.b)                                   # eq. pgd1
        eta = J @ vs                                              # eq. subp
        lam_star = (-(eta + phi_e1) / np.repeat(gamma, 3)).reshape(nc, 3)   # Alg. 2
        lam, branch = project(lam_star, p.mu)                     # eq. operator
        v_new = vs + w * (J.T @ lam.ravel())                      # eq. vup
        theta = float(np.linalg.norm(v_new - v))
        if history:
            hist.append(theta)
        v_prev, Av_prev, v = v, Av, v_new
        if not fixed_iters and theta < tol:
            break
    return {"v": v, "lam": lam, "iters": it, "theta": theta, "lam_star": lam_star,
            "branch": branch, "w": w, "gamma": gamma, "alpha": alpha, "history": hist,
            "projection": projection}
