"""V-FPI with Chebyshev acceleration (Alg. 3), float64, test infrastructure.

Each iteration runs the plain V-FPI sweep of ``core.vfpi`` from v^l to get
v** (eq. pgd1, Alg. 2, eq. vup), then

    nu_{l+1} = 1                           if l <  l_s
             = 2 / (2 - rho^2)             if l == l_s
             = 4 / (4 - rho^2 nu_l)        if l >  l_s
    v^{l+1}  = nu_{l+1} (u (v** - v^l) + v^l - v^{l-1}) + v^{l-1}     (eq. chebyup)
    theta    = ||v^{l+1} - v^l||, stop if theta < tol or l = l_max   (Alg. 3)
    rho      = min(theta_l / theta_{l-1}, 1)                        (eq. varrho)

with v^0 = v^1 (so the first step is the plain sweep, under-relaxed by u).
Readings (the printed passage is terse): u is the under-relaxation factor the
text mentions but Alg. 3 does not show, placed on the new correction
v** - v^l (u = 1 gives eq. chebyup exactly); rho is computed after the stop
test of iteration l from the two latest residuals theta_l = ||v^{l+1} - v^l||
and theta_{l-1} (rho = 0 while only one residual exists or theta_{l-1} = 0).
lambda is the contact impulse of the sweep that produced the last v**.

Pins (tests/test_oracle_chebyshev.py): with l_s beyond l_max and u = 1 it is
the plain V-FPI exactly; on a linear system whose iteration matrix is
I - W A = r I and with rho held at r, the error after k accelerated steps is
the error at the start divided by the Chebyshev polynomial T_k(1/r) (the
textbook semi-iterative bound, attained for a scalar iteration matrix); there
the estimate of eq. varrho is exactly r before acceleration starts, so the
first accelerated nu is 2 / (2 - r^2); u < 1 gives the under-relaxed
iteration matrix; it converges to the plain V-FPI's solution.
"""
from __future__ import annotations

import numpy as np

from .core import (contact_gamma, contact_jacobian, frobenius_w, project_proximal, project_strict,
                   project_strict_aniso, row_stats,
                   validate)


def vfpi_chebyshev(p, *, max_iters=100, tol=0.0, fixed_iters=False, l_s=10, u=1.0, w_mode="frobenius",
                   alpha_user=None, projection="strict", history=False, rho_fixed=None, omega=0.0):
    """``rho_fixed`` replaces the estimate of eq. varrho by a constant (a test
    hook: with the exact spectral radius the classical error bound applies)."""
    A = validate(p)
    J = contact_jacobian(p)
    nc = p.n_contacts
    project = project_strict if projection == "strict" else project_proximal
    if getattr(p, "mu2", None) is not None:  # anisotropic friction (strict operator only)
        assert projection == "strict"

        def project(ls, mu1, _mu2=p.mu2):
            return project_strict_aniso(ls, mu1, _mu2)
    if w_mode == "frobenius":
        w = frobenius_w(p, *row_stats(A))
    elif w_mode == "scalar":
        w = np.full(p.n, float(alpha_user))
    else:
        raise ValueError(w_mode)
    gamma = contact_gamma(p, w) + omega
    phi_e1 = np.zeros(3 * nc)
    phi_e1[0::3] = p.phi
    v = p.v0.copy()
    v_prev = v.copy()
    nu = 1.0
    rho = 0.0
    theta_prev = None
    lam = np.zeros((nc, 3))
    lam_star = np.zeros((nc, 3))
    branch = np.zeros(nc, dtype=np.int32)
    theta = np.inf
    hist, it = [], 0
    for it in range(1, max_iters + 1):
        vs = v - w * (A @ v - p.b)                                    # eq. pgd1
        lam_star = (-(J @ vs + phi_e1) / np.repeat(gamma, 3)).reshape(nc, 3)
        lam, branch = project(lam_star, p.mu)                         # Alg. 2
        vss = vs + w * (J.T @ lam.ravel())                            # v** (eq. vup)
        if it < l_s:
            nu = 1.0
        elif it == l_s:
            nu = 2.0 / (2.0 - rho * rho)
        else:
            nu = 4.0 / (4.0 - rho * rho * nu)
        v_new = nu * (u * (vss - v) + v - v_prev) + v_prev              # eq. chebyup
        theta = float(np.linalg.norm(v_new - v))
        if history:
            hist.append((theta, nu))
        v_prev, v = v, v_new
        if not fixed_iters and theta < tol:
            break
        if rho_fixed is not None:
            rho = rho_fixed
        else:
            rho = min(theta / theta_prev, 1.0) if theta_prev else 0.0  # eq. varrho
        theta_prev = theta
    return {"v": v, "lam": lam, "iters": it, "theta": theta, "lam_star": lam_star, "branch": branch, "w": w,
            "gamma": gamma, "history": hist, "projection": projection}
