"""Implicit differentiation of a converged V-FPI step (float64, test infrastructure).

The V-FPI map of the paper's convergence analysis (Sec. IV, Lemma 1 framing)
is f(v) = v* + W J_c^T lambda(v*), v* = v - W (A v - b),
lambda = P(-Gamma^{-1}(J_c v* + phi e1); mu) with P the strict projection
(eq. operator, Alg. 2).  At its fixed point the solution is independent of W
(consistency remark, Sec. III-B), so W is held constant.  Linearizing with
D_P the 3x3 Jacobian of P per contact (branch of the last projection:
open 0; stick I; slip dl_n/dn = 1, dl_t/dn = mu t/s, dl_t/dt = (mu n/s)(I - t t^T/s^2),
dl_t/dmu = n t/s, with (n, t) = lambda*, s = ||t||) and

    G = I - W J^T D_P Gamma^{-1} J

the adjoint u of a loss with gradients (g_v, g_lam) solves

    u = g~ + (I - A W) G^T u,        g~ = g_v - (I - A W) J^T Gamma^{-1} D_P^T g_lam

and then, with r = J W u + g_lam and q = u - J^T Gamma^{-1} D_P^T r:

    b_bar = W q,   A_bar_ij = -b_bar_i v_j (on the pattern of A),
    phi_bar_m = -(D_P,m^T r_m)_n / gamma_m,   mu_bar_m = (dP_m/dmu)^T r_m.

With the proximal operator (Euclidean projection onto the cone, eq. operator)
D_P on the slip branch is that of the second-order-cone projection
P = (n + mu s)/(1 + mu^2) (1, mu t/s): with c = 1/(1 + mu^2), h = t/s and
a = (n + mu s) c,
    dP_n/dn = c,  dP_n/dt = mu c h^T,  dP_t/dn = mu c h,
    dP_t/dt = mu^2 c h h^T + (mu a / s)(I - h h^T),
    dP_n/dmu = c (s - 2 mu a),  dP_t/dmu = (a + mu dP_n/dmu) h;
stick is I and open (the polar cone) is 0, as for the strict operator.

With anisotropic friction (strict operator on the elliptic cone, Sec. III-E)
the slip branch keeps lambda_n = n and x_i = A_i t_i / (A_i + s), A_i =
(mu_i n)^2, with s the root of F(s) = sum_i A_i t_i^2 / (A_i + s)^2 - 1.
Implicit differentiation (D_i = A_i + s, F_s = -2 sum_i A_i t_i^2 / D_i^3):
    ds = -(sum_i 2 A_i t_i / D_i^2 dt_i + sum_i t_i^2 (s - A_i) / D_i^3 dA_i) / F_s,
    dx_i = (t_i s / D_i^2) dA_i + (A_i / D_i) dt_i - (x_i / D_i) ds,
    dA_i = 2 mu_i^2 n dn + 2 mu_i n^2 dmu_i,
which gives D_P, dP/dmu1 and dP/dmu2 (mu2_bar = (dP/dmu2)^T r).  With one
coefficient zero the ellipse is a segment and P clamps each tangent component
to [-mu_i n, mu_i n]: a clamped component has dx_i/dn = sign(t_i) mu_i and
dx_i/dmu_i = sign(t_i) n, a free one dx_i/dt_i = 1; the derivative in the
zero coefficient is the one-sided one of the opening ellipse (ellipse_jacobian).

``adjoint`` solves for u by the transposed fixed-point iteration (SciPy
matvecs); ``adjoint_dense`` solves the same linear system with a dense LU.
Pins: the two agree; gradients match central finite differences of the
oracle's converged forward; they are the same for two different W; and the
sliding particle's closed form dx_N/dmu = -h^2 g cos(a) N(N+1)/2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .core import BRANCH_SLIP, BRANCH_STICK, contact_jacobian, ellipse_root, system_matrix


def ellipse_jacobian(n, t, mu1, mu2):
    """Slip branch of the strict operator on the elliptic cone: D_P [3,3],
    dP/dmu1 [3] and dP/dmu2 [3] at lambda* = (n, t)."""
    mu = np.array([mu1, mu2])
    DP = np.zeros((3, 3))
    dmu = np.zeros((2, 3))
    DP[0, 0] = 1.0
    if mu1 * n == 0.0 or mu2 * n == 0.0:   # a zero semi-axis, as the projection tests it
        # a zero semi-axis: the ellipse is a segment and P clamps each tangent
        # component to [-mu_i n, mu_i n] on its own
        for i in range(2):
            if abs(t[i]) > mu[i] * n:
                sg = np.sign(t[i])
                DP[1 + i, 0] = sg * mu[i]
                dmu[i, 1 + i] = sg * n
            else:
                DP[1 + i, 1 + i] = 1.0
        # the zero coefficient's derivative is one-sided (mu >= 0): the
        # ellipse's limit as its axis opens.  Past the tip (|t_j| > b) the
        # closest point stays at the tip to first order; beside the segment
        # s = a |t_i| / r + O(a^2), r = sqrt(1 - t_j^2 / b^2), so
        # dx_i/dmu_i = sign(t_i) n r and dx_j/dmu_i = -n t_j |t_i| / (b^2 r).
        i = 0 if mu1 * n == 0.0 else 1
        j = 1 - i
        dmu[i] = 0.0
        b = mu[j] * n
        if b > 0.0 and abs(t[j]) < b:
            r = np.sqrt(1.0 - (t[j] / b) ** 2)
            dmu[i, 1 + i] = np.sign(t[i]) * n * r
            dmu[i, 1 + j] = -n * t[j] * abs(t[i]) / (b * b * r)
        return DP, dmu[0], dmu[1]
    A = (mu * n) ** 2
    s = ellipse_root(t[0], t[1], mu1 * n, mu2 * n)
    D = A + s
    x = A * t / D
    F_s = -2.0 * np.sum(A * t * t / D ** 3)
    g_t = 2.0 * A * t / D ** 2
    g_A = t * t * (s - A) / D ** 3
    A_n = 2.0 * mu * mu * n          # dA_i / dn
    A_mu = 2.0 * mu * n * n          # dA_i / dmu_i
    ds_dn = -np.sum(g_A * A_n) / F_s
    ds_dt = -g_t / F_s
    ds_dmu = -g_A * A_mu / F_s
    for i in range(2):
        DP[1 + i, 0] = t[i] * s / D[i] ** 2 * A_n[i] - x[i] / D[i] * ds_dn
        for j in range(2):
            DP[1 + i, 1 + j] = (A[i] / D[i] if i == j else 0.0) - x[i] / D[i] * ds_dt[j]
            dmu[j, 1 + i] = (t[i] * s / D[i] ** 2 * A_mu[i] if i == j else 0.0) - x[i] / D[i] * ds_dmu[j]
    return DP, dmu[0], dmu[1]


def projection_jacobians(lam_star, branch, mu, projection="strict", mu2=None):
    """Per contact: D_P [nc,3,3], dP/dmu [nc,3] and (anisotropic friction)
    dP/dmu2 [nc,3] on the branch taken; dP/dmu2 is None without mu2."""
    nc = lam_star.shape[0]
    DP = np.zeros((nc, 3, 3))
    dmu = np.zeros((nc, 3))
    dmu2 = None if mu2 is None else np.zeros((nc, 3))
    st = branch == BRANCH_STICK
    DP[st] = np.eye(3)
    sl = np.nonzero(branch == BRANCH_SLIP)[0]
    if sl.size and mu2 is not None:
        for m in sl:
            DP[m], dmu[m], dmu2[m] = ellipse_jacobian(lam_star[m, 0], lam_star[m, 1:], mu[m], mu2[m])
    elif sl.size and projection == "proximal":
        n = lam_star[sl, 0]
        t = lam_star[sl, 1:]
        s = np.linalg.norm(t, axis=1)
        h = t / s[:, None]
        m = mu[sl]
        c = 1.0 / (1.0 + m * m)
        a = (n + m * s) * c
        DP[sl, 0, 0] = c
        DP[sl, 0, 1:] = (m * c)[:, None] * h
        DP[sl, 1:, 0] = (m * c)[:, None] * h
        hh = h[:, :, None] * h[:, None, :]
        DP[sl, 1:, 1:] = (m * m * c)[:, None, None] * hh + (m * a / s)[:, None, None] * (np.eye(2) - hh)
        da = c * (s - 2.0 * m * a)
        dmu[sl, 0] = da
        dmu[sl, 1:] = (a + m * da)[:, None] * h
    elif sl.size:
        n = lam_star[sl, 0]
        t = lam_star[sl, 1:]
        s = np.linalg.norm(t, axis=1)
        th = t / s[:, None]
        m = mu[sl]
        DP[sl, 0, 0] = 1.0
        DP[sl, 1:, 0] = m[:, None] * th
        DP[sl, 1:, 1:] = (m * n / s)[:, None, None] * (np.eye(2) - th[:, :, None] * th[:, None, :])
        dmu[sl, 1:] = n[:, None] * th
    return DP, dmu, dmu2


def _operators(p, fwd):
    mu2 = getattr(p, "mu2", None)
    if mu2 is not None and fwd.get("projection", "strict") != "strict":
        raise ValueError("anisotropic friction is defined for the strict operator only")
    A = system_matrix(p)
    J = contact_jacobian(p)
    DP, dmu, dmu2 = projection_jacobians(fwd["lam_star"], fwd["branch"], p.mu, fwd.get("projection", "strict"), mu2)
    DPb = sp.block_diag(list(DP), format="csr") if p.n_contacts else sp.csr_matrix((0, 0))
    ginv = np.repeat(1.0 / fwd["gamma"], 3)
    return A, J, DP, (dmu, dmu2), DPb, ginv


def _grads_from_u(p, fwd, u, g_lam, J, DP, dmus, DPb, ginv):
    dmu, dmu2 = dmus
    w = fwd["w"]
    nc = p.n_contacts
    r = J @ (w * u) + g_lam
    q = u - J.T @ (ginv * (DPb.T @ r))
    b_bar = w * q
    rm = r.reshape(nc, 3)
    dpr = np.einsum("mji,mj->mi", DP, rm)           # D_P^T r per contact
    phi_bar = -dpr[:, 0] / fwd["gamma"]
    mu_bar = np.einsum("mi,mi->m", dmu, rm)
    mu2_bar = None if dmu2 is None else np.einsum("mi,mi->m", dmu2, rm)
    # A_bar on the block pattern: block (i, c) = -b_bar_i v_c^T
    rows = np.repeat(np.arange(p.n_nodes), np.diff(p.row_ptr))
    A_bar = -b_bar.reshape(-1, 3)[rows][:, :, None] * fwd["v"].reshape(-1, 3)[p.col_idx][:, None, :]
    out = {"u": u, "b": b_bar, "A": A_bar, "phi": phi_bar, "mu": mu_bar}
    if mu2_bar is not None:
        out["mu2"] = mu2_bar
    return out


def adjoint(p, fwd, g_v, g_lam=None, *, tol=1e-14, max_iters=100000):
    A, J, DP, dmus, DPb, ginv = _operators(p, fwd)
    w = fwd["w"]
    nc = p.n_contacts
    g_lam = np.zeros(3 * nc) if g_lam is None else np.asarray(g_lam, dtype=np.float64).ravel()

    def i_minus_aw(x):
        return x - A @ (w * x)

    def gt(x):  # G^T x
        return x - J.T @ (ginv * (DPb.T @ (J @ (w * x))))

    g_t = g_v - i_minus_aw(J.T @ (ginv * (DPb.T @ g_lam)))
    u = g_t.copy()
    it = 0
    theta = np.inf
    for it in range(1, max_iters + 1):
        u_new = g_t + i_minus_aw(gt(u))
        theta = float(np.linalg.norm(u_new - u))
        u = u_new
        if theta < tol:
            break
    out = _grads_from_u(p, fwd, u, g_lam, J, DP, dmus, DPb, ginv)
    out.update(iters=it, theta=theta)
    return out


def adjoint_dense(p, fwd, g_v, g_lam=None):
    A, J, DP, dmus, DPb, ginv = _operators(p, fwd)
    w = fwd["w"]
    n, nc = p.n, p.n_contacts
    g_lam = np.zeros(3 * nc) if g_lam is None else np.asarray(g_lam, dtype=np.float64).ravel()
    Ad = A.toarray()
    W = np.diag(w)
    Jd = J.toarray()
    Gam_inv = np.diag(ginv)
    DPd = DPb.toarray() if nc else np.zeros((0, 0))
    G = np.eye(n) - W @ Jd.T @ DPd @ Gam_inv @ Jd
    IAW = np.eye(n) - Ad @ W
    g_t = g_v - IAW @ (Jd.T @ (Gam_inv @ (DPd.T @ g_lam)))
    u = np.linalg.solve(np.eye(n) - IAW @ G.T, g_t)
    return _grads_from_u(p, fwd, u, g_lam, J, DP, dmus, DPb, ginv)
