"""Pins of the Chebyshev-accelerated V-FPI oracle (Alg. 3)."""
import numpy as np
import pytest

import oracle
import scenes
from oracle.chebyshev import vfpi_chebyshev


def _diag_problem(n_nodes, a, seed):
    g = np.random.default_rng(seed)
    val = np.tile(a * np.eye(3), (n_nodes, 1, 1))
    return scenes.Problem(n_nodes=n_nodes, row_ptr=np.arange(n_nodes + 1), col_idx=np.arange(n_nodes), val=val,
                          b=g.normal(size=3 * n_nodes), v0=g.normal(size=3 * n_nodes), c_node=np.zeros(0),
                          c_node_j=np.zeros(0), R=np.zeros((0, 3, 3)), phi=np.zeros(0), mu=np.zeros(0))


@pytest.mark.parametrize("r,l_s", [(0.9, 3), (0.97, 5), (0.6, 4)])
def test_error_follows_chebyshev_polynomial(r, l_s):
    """For I - W A = r I and rho held at r, the accelerated error after k
    steps is e_0 / T_k(1/r), e_0 being the error of v^{l_s - 1} (textbook
    semi-iteration, attained for a scalar iteration matrix)."""
    a = 2.5
    p = _diag_problem(7, a, 1)
    x = p.b / a
    alpha = (1.0 - r) / a
    errs = []
    for L in range(1, l_s + 13):
        res = vfpi_chebyshev(p, max_iters=L, fixed_iters=True, l_s=l_s, w_mode="scalar", alpha_user=alpha,
                             rho_fixed=r)
        errs.append(np.linalg.norm(res["v"] - x))   # error of v^{L+1}
    e0 = errs[l_s - 3]  # v^{l_s - 1}, produced by iteration l_s - 2
    for k in range(1, 12):
        Tk = np.cosh(k * np.arccosh(1.0 / r))
        np.testing.assert_allclose(errs[l_s - 3 + k], e0 / Tk, rtol=1e-9)


@pytest.mark.parametrize("r,l_s", [(0.9, 3), (0.5, 6)])
def test_rho_estimate_is_exact_before_acceleration(r, l_s):
    """With a scalar iteration matrix the residual ratio of eq. varrho is r,
    so the first accelerated nu is 2 / (2 - r^2)."""
    a = 1.7
    p = _diag_problem(4, a, 3)
    res = vfpi_chebyshev(p, max_iters=l_s + 2, fixed_iters=True, l_s=l_s, w_mode="scalar",
                         alpha_user=(1.0 - r) / a, history=True)
    nus = [h[1] for h in res["history"]]
    assert nus[:l_s - 1] == [1.0] * (l_s - 1)
    np.testing.assert_allclose(nus[l_s - 1], 2.0 / (2.0 - r * r), rtol=1e-12)
    thetas = [h[0] for h in res["history"]]
    np.testing.assert_allclose(thetas[1] / thetas[0], r, rtol=1e-12)


def test_without_acceleration_it_is_plain_vfpi():
    sc, x, v = scenes.cloth_cfg1(0)
    p = sc.assemble(x, v)
    a = vfpi_chebyshev(p, max_iters=40, fixed_iters=True, l_s=1000)
    b = oracle.vfpi(p, max_iters=40, fixed_iters=True)
    # same iterates up to the rounding of nu (u (v** - v) + v - v_prev) + v_prev with nu = u = 1
    np.testing.assert_allclose(a["v"], b["v"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(a["lam"], b["lam"], rtol=0, atol=1e-13 * np.abs(b["lam"]).max())


def test_under_relaxation_on_linear_problem():
    """u < 1 without acceleration: v^{l+1} = v^l + u (v** - v^l), so the
    iteration matrix becomes (1 - u) I + u (I - W A)."""
    a, r, u = 2.0, 0.5, 0.7
    p = _diag_problem(5, a, 2)
    x = p.b / a
    res = [vfpi_chebyshev(p, max_iters=L, fixed_iters=True, l_s=1000, u=u, w_mode="scalar",
                          alpha_user=(1 - r) / a)["v"] for L in (1, 2, 3, 4)]
    e0 = np.linalg.norm(p.v0 - x)
    for k, vv in enumerate(res, start=1):
        np.testing.assert_allclose(np.linalg.norm(vv - x), e0 * (1 - u + u * r) ** k, rtol=1e-12)


@pytest.mark.parametrize("case", ["cloth10", "random"])
def test_converges_to_plain_solution_in_fewer_sweeps(case):
    if case == "cloth10":
        sc, x, v = scenes.cloth_cfg1(0)
        p = sc.assemble(x, v)
    else:
        p = scenes.random_problem(60, 25, 3, degree=5.0, phi_scale=0.4)
    plain = oracle.vfpi(p, max_iters=50000, tol=1e-12)
    acc = vfpi_chebyshev(p, max_iters=50000, tol=1e-12, l_s=10, u=1.0)
    np.testing.assert_allclose(acc["v"], plain["v"], atol=1e-9)
    assert acc["iters"] < plain["iters"]
