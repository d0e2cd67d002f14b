"""The original contact problem in impulse space, solved the classical way.

Delassus form (eq. delassus):  J_c v = D lambda + J_c A^{-1} b  with
D = J_c A^{-1} J_c^T, computed here from a dense Cholesky factor of A (the
paper's I-FPI baselines factor A, Sec. V-C.1).  Solved by projected
Gauss-Seidel (PGS, the paper's first I-FPI baseline), contact by contact in
index order:

* normal:   lambda_n <- max(0, lambda_n - u_n / D_nn)
* tangent:  lambda_t <- proj_disk(mu lambda_n)(lambda_t - u_t / rho_m), u refreshed
            after the normal update, rho_m = largest eigenvalue of the 2x2
            tangential block D_tt,m

with u = D lambda + c, c = J_c A^{-1} b + phi e1.  The paper does not spell out
its PGS; a scalar tangential step makes every fixed point satisfy the SCC
exactly (friction exactly opposite the slip), which is what the pin needs.
The residual is mapped to velocity space through A^{-1} J_c^T (Sec. V-C.1):
theta = ||A^{-1} J_c^T (lambda^{l+1} - lambda^l)||.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .core import contact_jacobian, system_matrix, validate


def delassus(p):
    """Returns (D, c, Y, v_free): D = J A^-1 J^T, c = J A^-1 b + phi e1,
    Y = A^-1 J^T, v_free = A^-1 b (dense, for small problems)."""
    A = system_matrix(p)
    validate(p, A)
    Ad = A.toarray()
    J = contact_jacobian(p).toarray()
    cf = sla.cho_factor(Ad, lower=True)
    Y = sla.cho_solve(cf, J.T)
    v_free = sla.cho_solve(cf, p.b)
    D = J @ Y
    c = J @ v_free
    c[0::3] += p.phi
    return D, c, Y, v_free


def _disk(t, radius):
    s = np.hypot(t[0], t[1])
    return t if s <= radius else (t * (radius / s) if s > 0 else t)


def pgs(p, *, max_sweeps=10000, tol=1e-12, lam0=None, dl=None):
    """Projected Gauss-Seidel on the Delassus operator.  Returns a dict with
    v = A^-1 b + Y lambda, lambda [nc,3], sweeps, theta."""
    D, c, Y, v_free = delassus(p) if dl is None else dl
    nc = p.n_contacts
    lam = np.zeros(3 * nc) if lam0 is None else np.asarray(lam0, dtype=np.float64).ravel().copy()
    rho = np.zeros(nc)
    for m in range(nc):
        rho[m] = np.linalg.eigvalsh(D[3 * m + 1:3 * m + 3, 3 * m + 1:3 * m + 3]).max()
    theta = np.inf
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        old = lam.copy()
        for m in range(nc):
            k = 3 * m
            u_n = D[k] @ lam + c[k]
            lam[k] = max(0.0, lam[k] - u_n / D[k, k])
            u_t = D[k + 1:k + 3] @ lam + c[k + 1:k + 3]
            lam[k + 1:k + 3] = _disk(lam[k + 1:k + 3] - u_t / rho[m], p.mu[m] * lam[k])
        theta = float(np.linalg.norm(Y @ (lam - old)))
        if theta < tol:
            break
    return {"v": v_free + Y @ lam, "lam": lam.reshape(nc, 3), "sweeps": sweeps, "theta": theta}
