"""Brute-force solutions of the original contact problem on its Delassus form.

With u = D lambda + c (c = J_c A^{-1} b + phi e1, eq. delassus) the SCC of
eq. scc per contact m read: 0 <= lambda_n _|_ u_n >= 0; lambda in the cone;
stick => u_t = 0; slip => lambda_t = -mu lambda_n u_t / ||u_t||.

* ``lcp_enumerate``: frictionless case (mu = 0), every active set of the
  2^n_c, each one a linear solve (textbook LCP enumeration).
* ``mode_enumerate``: open / stick / slip for every contact (3^n_c modes); each
  mode's equations are solved by SciPy's root finder from several seeded
  starts, and a root is kept only if it satisfies every SCC inequality.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.optimize as so


def lcp_enumerate(Dn, cn, tol=1e-12):
    """All lambda_n >= 0 with u_n = Dn lambda_n + cn >= 0, lambda_n . u_n = 0."""
    m = cn.shape[0]
    sols = []
    scale = max(1.0, np.abs(cn).max())
    for mask in itertools.product((False, True), repeat=m):
        act = np.array(mask, dtype=bool)
        lam = np.zeros(m)
        if act.any():
            lam[act] = np.linalg.solve(Dn[np.ix_(act, act)], -cn[act])
        u = Dn @ lam + cn
        if np.all(lam >= -tol * scale) and np.all(u[~act] >= -tol * scale):
            sols.append(np.maximum(lam, 0.0))
    return sols


def _mode_residual(lam, D, c, mu, modes):
    u = D @ lam + c
    out = np.empty_like(lam)
    for m, md in enumerate(modes):
        k = 3 * m
        if md == 0:      # open
            out[k:k + 3] = lam[k:k + 3]
        elif md == 1:    # stick
            out[k:k + 3] = u[k:k + 3]
        else:            # slip
            ut = u[k + 1:k + 3]
            s = np.hypot(ut[0], ut[1])
            out[k] = u[k]
            out[k + 1:k + 3] = lam[k + 1:k + 3] + mu[m] * lam[k] * ut / max(s, 1e-300)
    return out


def scc_satisfied(lam, D, c, mu, modes, tol):
    u = D @ lam + c
    for m, md in enumerate(modes):
        k = 3 * m
        ln, lt = lam[k], lam[k + 1:k + 3]
        un, ut = u[k], u[k + 1:k + 3]
        if md == 0:
            if un < -tol or np.abs(lam[k:k + 3]).max() > tol:
                return False
        else:
            if ln < -tol or abs(un) > tol:
                return False
            if md == 1:
                if np.hypot(*lt) > mu[m] * ln + tol or np.abs(ut).max() > tol:
                    return False
            else:
                s = np.hypot(*ut)
                if s <= tol or ln <= tol:
                    return False
                if abs(np.hypot(*lt) - mu[m] * ln) > tol:
                    return False
                # friction opposite the slip velocity
                if lt @ ut > -(1 - 1e-9) * np.hypot(*lt) * s:
                    return False
    return True


def mode_enumerate(D, c, mu, *, n_starts=8, seed=0, tol=1e-10):
    """All solutions of the SCC on the Delassus form, by enumerating the
    3^n_c open/stick/slip modes.  Returns a list of (lambda, modes)."""
    nc = c.shape[0] // 3
    g = np.random.default_rng(seed)
    found = []
    scale = max(1.0, np.abs(c).max() / max(np.abs(np.diag(D)).min(), 1e-300))
    for modes in itertools.product((0, 1, 2), repeat=nc):
        starts = [np.linalg.solve(D, -c)] + [g.normal(size=3 * nc) * scale for _ in range(n_starts)]
        for x0 in starts:
            try:
                r = so.root(_mode_residual, x0, args=(D, c, mu, modes), method="hybr", tol=1e-14)
            except Exception:
                continue
            lam = r.x
            if np.abs(_mode_residual(lam, D, c, mu, modes)).max() > tol * scale:
                continue
            if not scc_satisfied(lam, D, c, mu, modes, tol * scale):
                continue
            if not any(np.abs(lam - f[0]).max() <= 1e-8 * scale for f in found):
                found.append((lam.copy(), modes))
            break
    return found
