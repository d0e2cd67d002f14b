"""FP64 HIP path vs the FP64 oracle, element by element, at a fixed sweep
count (bar: 1e-9 relative on v and lambda), across every kernel variant,
ragged sizes, the full-size cloth and FEM workloads, and the edge cases."""
import numpy as np
import pytest
import torch

import oracle
import paper_2201_09212_amd as vf
import scenes
from paper_2201_09212_amd import _abi
from tests.gpu_util import fixed_parity, gate, gpu_step, say, solver_for, tape_parts, upload

pytestmark = pytest.mark.gpu
TOL = 1e-9

# kind | chunk slots << 8 | workgroup cap << 16 | LDS levels (kind 5: 1 off, 2 on) << 24
# | load group (kind 1, 8 slots: 1 = two levels) << 26
VARIANTS = {
    "wg1_node16": 3,
    "wg1_node4": 3 | (4 << 8),
    "wg1_row5": 4,
    "grid_node1": 1 | (1 << 8),
    "grid_node4": 1 | (4 << 8),
    "grid_row1": 2,
    "grid_row2": 2 | (2 << 8),
    "grid_node4_cap8": 1 | (4 << 8) | (8 << 16),
    "grid_row1_cap16": 2 | (16 << 16),
    "grid_row2_cap8": 2 | (2 << 8) | (8 << 16),
    "grid_node2_cap3": 1 | (2 << 8) | (3 << 16),
    "grid_node8": 1 | (8 << 8),
    "grid_node8_u2": 1 | (8 << 8) | (1 << 26),
    "grid_node16": 1 | (16 << 8),
    "grid_row4": 2 | (4 << 8),
    "regs_node1": 5 | (1 << 8),
    "regs_node2": 5 | (2 << 8),
    "regs_node4": 5 | (4 << 8),
    "regs_node5": 5 | (5 << 8),
    "regs_node6": 5 | (6 << 8),
    "regs_node8": 5 | (8 << 8),
    "regs_node1_grid16": 5 | (1 << 8) | (16 << 16),
    "regs_node2_lds_on": 5 | (2 << 8) | (2 << 24),
    "regs_node4_lds_on": 5 | (4 << 8) | (2 << 24),
    "regs_node5_lds_off": 5 | (5 << 8) | (1 << 24),
    "regs_node1_lds_off": 5 | (1 << 8) | (1 << 24),
}

CASES = [(1, 1), (5, 0), (5, 5), (63, 20), (64, 64), (65, 30), (130, 77), (700, 300)]


def _compare(p, L, variant, **kw):
    """GPU vs oracle at L sweeps: v, lambda and lambda* element by element
    (bar 1e-9), every contact's branch, and the branch counts."""
    okw = {k: v for k, v in kw.items() if k in ("w_mode", "w_user", "alpha_user", "projection")}
    ref = oracle.vfpi(p, max_iters=L, fixed_iters=True, **okw)
    gkw = {k: v for k, v in kw.items() if k in ("w_mode",)}
    if "w_user" in kw:
        gkw["w_user"] = torch.as_tensor(kw["w_user"], device="cuda")
    if "alpha_user" in kw:
        gkw["alpha"] = kw["alpha_user"]
    ev, el, st, ties = fixed_parity(p, ref, L, TOL, f"N={p.n_nodes} L={L} variant={variant:#x}",
                                    projection=kw.get("projection", "strict"), variant=variant, **gkw)
    say(f"  N={p.n_nodes} nc={p.n_contacts} L={L} variant={variant:#x} rel_v={ev:.2e} rel_lam={el:.2e} "
        f"branch ties={ties}")
    return st


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("n,nc", CASES)
def test_random_parity_all_variants(n, nc, variant):
    p = scenes.random_problem(n, nc, 11 * n + nc, degree=5.0, phi_scale=0.5)
    for L in (1, 7, 40):
        _compare(p, L, VARIANTS[variant])


@pytest.mark.parametrize("mode", ["diag", "scalar", "proximal"])
def test_user_w_and_proximal_parity(mode):
    p = scenes.random_problem(300, 120, 5, degree=5.0, phi_scale=0.5)
    kw = {}
    if mode == "diag":
        w = oracle.frobenius_w(p, *oracle.row_stats(oracle.system_matrix(p))) * 0.8
        kw = {"w_mode": "diag", "w_user": w}
    elif mode == "scalar":
        kw = {"w_mode": "scalar", "alpha_user": 0.9 * oracle.core.gershgorin_alpha(oracle.system_matrix(p))}
    else:
        kw = {"projection": "proximal"}
    for variant in (3, 2, 1 | (4 << 8)):
        _compare(p, 25, variant, **kw)


def test_cloth10_fixed_and_converged():
    sc, x, v = scenes.cloth_cfg1(0)
    p = sc.assemble(x, v)
    for variant in (0, 3, 4, 2, 5 | (1 << 8)):
        _compare(p, 50, variant)
    ref = oracle.vfpi(p, max_iters=1000, tol=1e-10)
    v_, lam, st, _ = gpu_step(p, max_iters=1000, tol=1e-10)
    say(f"  cloth10 converged: oracle {ref['iters']} sweeps, gpu {st['iters']}, theta {st['theta']:.2e}")
    assert st["status"] == _abi.VFPI_S_CONVERGED
    assert abs(st["iters"] - ref["iters"]) <= 1
    gate(v_, ref["v"], 1e-9, "cloth10 converged v")


def test_cloth128_full_size():
    sc, x, v = scenes.cloth_cfg2(0)
    p = sc.assemble(x, v)
    for variant in (0, 1 | (4 << 8), 2 | (2 << 8), 2, 1 | (1 << 8), 5 | (1 << 8), 5 | (2 << 8), 5 | (4 << 8)):
        _compare(p, 50, variant)


def test_fem_full_size():
    sc, x, v = scenes.fem_cfg3(0)
    p = sc.assemble(x, v)
    for variant in (0, 1 | (4 << 8), 2, 1 | (2 << 8), 5 | (5 << 8), 5 | (6 << 8), 5 | (8 << 8)):
        _compare(p, 20, variant)


@pytest.mark.parametrize("variant", [k for k in VARIANTS if k.startswith("regs")])
def test_long_rows_register_lds_and_streamed_levels(variant):
    """Rows of 4 to 34 blocks (S- and D-contacts): each register-resident
    instance keeps the first levels in registers, the next ones in LDS and
    streams the rest."""
    for n, nc, nd in ((700, 300, 0), (130, 60, 20)):
        p = scenes.random_problem(n, nc, 7 * n + nc, degree=18.0, phi_scale=0.5, n_d_contacts=nd)
        assert np.diff(p.row_ptr).max() > 17
        for L in (1, 9):
            _compare(p, L, VARIANTS[variant])


def test_fem_paper_size_block():
    """16 x 16 x 4 cells: rows of up to 19 blocks, more than the register and
    LDS levels of the one- and two-slot register-resident kernels."""
    sc, x, v = scenes.fem_ctx(0)
    p = sc.assemble(x, v)
    for variant in (0, 1 | (2 << 8), 3, 5 | (1 << 8), 5 | (2 << 8), 5 | (4 << 8), 5 | (5 << 8)):
        _compare(p, 30, variant)


def test_inclined_plane_analytic_on_gpu():
    alpha = np.array([0.2, 0.2, 0.6, 0.6])
    mu = np.tan(alpha) + np.array([-1e-6, 1e-6, -1e-6, 1e-6])
    p = scenes.inclined_plane_particles(alpha, mu, mass=2.0, h=0.01, g=9.81)
    v, lam, st, _ = gpu_step(p, max_iters=3, fixed_iters=True)
    for k in range(4):
        slide = mu[k] < np.tan(alpha[k])
        sp = 0.01 * 9.81 * (np.sin(alpha[k]) - mu[k] * np.cos(alpha[k])) if slide else 0.0
        exp = sp * np.array([np.cos(alpha[k]), 0.0, -np.sin(alpha[k])])
        np.testing.assert_allclose(v[3 * k:3 * k + 3], exp, atol=1e-15)
    assert [st["n_open"], st["n_stick"], st["n_slip"]] == [0, 2, 2]


def test_deterministic_bitwise():
    sc, x, v = scenes.cloth_cfg2(1)
    p = sc.assemble(x, v)
    s = solver_for(p)
    a = gpu_step(p, solver=s, max_iters=30, fixed_iters=True)
    b = gpu_step(p, solver=s, max_iters=30, fixed_iters=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2]["theta"] == b[2]["theta"]


def test_zero_iterations_and_no_contacts():
    p = scenes.random_problem(100, 40, 3)
    v, lam, st, _ = gpu_step(p, max_iters=0)
    assert np.array_equal(v, p.v0) and np.all(lam == 0) and st["iters"] == 0
    p0 = scenes.random_problem(100, 0, 3)
    _compare(p0, 10, 0)
    ref = oracle.vfpi(p0, max_iters=5000, tol=1e-13)
    v, lam, st, _ = gpu_step(p0, max_iters=5000, tol=1e-13)
    gate(v, ref["v"], 1e-9, "no contacts, converged v")


def _status_of(p, **kw):
    v, lam, st, _ = gpu_step(p, max_iters=10, **kw)
    assert st["iters"] == 0 and np.array_equal(v, p.v0) and np.all(lam == 0)
    return st["status"]


def test_device_detected_data_errors():
    p = scenes.random_problem(80, 10, 2)
    bad = scenes.Problem(**{**p.__dict__, "c_node": np.array([1, 1] + list(p.c_node[2:]))})
    assert _status_of(bad) & _abi.VFPI_S_SHARED_NODE
    R = p.R.copy()
    R[3, 0, 0] += 1e-6
    assert _status_of(scenes.Problem(**{**p.__dict__, "R": R})) & _abi.VFPI_S_NOT_ORTHONORMAL
    b = p.b.copy()
    b[7] = np.inf
    assert _status_of(scenes.Problem(**{**p.__dict__, "b": b})) & _abi.VFPI_S_NONFINITE
    val = p.val.copy()
    d = p.row_ptr[4] + int(np.nonzero(p.col_idx[p.row_ptr[4]:p.row_ptr[5]] == 4)[0][0])
    val[d, 1, 1] = -1.0
    assert _status_of(scenes.Problem(**{**p.__dict__, "val": val})) & _abi.VFPI_S_NONPOS_DIAG
    col = p.col_idx.copy()
    col[5] = 80
    assert _status_of(scenes.Problem(**{**p.__dict__, "col_idx": col})) & _abi.VFPI_S_BAD_PATTERN
    mu = p.mu.copy()
    mu[0] = -0.1
    assert _status_of(scenes.Problem(**{**p.__dict__, "mu": mu})) & _abi.VFPI_S_BAD_MU
    w = np.full(p.n, 0.1)
    w[3 * p.c_node[0]] = 0.2
    assert _status_of(p, w_mode="diag", w_user=torch.as_tensor(w, device="cuda")) & _abi.VFPI_S_BAD_W


def test_synchronous_argument_errors():
    small = vf.Solver(10, 10, 1)
    p2 = scenes.random_problem(50, 5, 4)
    A, Jc, b, v = upload(p2)
    with pytest.raises(vf.VfpiError, match="capacity"):
        small.step(A, b, Jc, v)
    s2 = solver_for(p2)
    with pytest.raises(vf.VfpiError, match="invalid option"):
        s2.step(A, b, Jc, v, max_iters=-1)
    with pytest.raises(vf.VfpiError, match="invalid option"):
        s2.step(A, b, Jc, v, w_mode="scalar", alpha=0.0)


def test_beyond_register_resident_grid():
    """140,000 nodes (2,188 chunks) need more than one workgroup per CU even
    with 8 chunk slots: the register-resident launch is refused with
    VFPI_E_OPTS, and the library default takes the streaming kernel."""
    p = scenes.random_problem(140000, 20000, 3, degree=5.0, phi_scale=0.5)
    s = solver_for(p)
    A, Jc, b, v = upload(p)
    v_in = v.clone()
    st = vf.new_stats(1, torch.device("cuda", 0))
    st.fill_(7)
    sentinel = st.clone()
    with pytest.raises(vf.VfpiError, match="invalid option"):
        s.step(A, b, Jc, v, stats=st, max_iters=3, fixed_iters=True, variant=5 | (8 << 8))
    torch.cuda.synchronize()
    # refused before anything was enqueued: v and the stats record untouched
    assert torch.equal(v, v_in) and torch.equal(st, sentinel)
    for variant in (0, 1 | (4 << 8), 1 | (8 << 8), 1 | (16 << 8)):
        _compare(p, 10, variant)


@pytest.mark.parametrize("which", ["cloth384", "fem128x64x16"])
def test_streaming_default_at_scale(which):
    """Past the register-resident grid (more than 2,048 chunks) the library
    default is the streaming kernel with eight chunk slots: a 384 x 384 cloth
    draped over spheres (147,456 nodes) and a 128 x 64 x 16-cell FEM block
    (142,545 nodes), 10 sweeps, element by element against the oracle."""
    if which == "cloth384":
        sc, x, v = scenes.cloth_drape(384, 0)
    else:
        sc, x, v = scenes.fem_block((128, 64, 16), 0)
    p = sc.assemble(x, v)
    assert (p.n_nodes + 63) // 64 > 2048
    for variant in (0, 1 | (16 << 8)):
        _compare(p, 10, variant)


def test_reuse_w_matches_oracle_with_previous_row_sums():
    sc, x, v = scenes.cloth_cfg1(0)
    p1 = sc.assemble(x, v)
    x2 = x + 0.001 * np.random.default_rng(0).normal(size=x.shape)
    p2 = sc.assemble(x2, v)
    s = vf.Solver(p2.n_nodes, p2.nnzb, p2.n_nodes)
    gpu_step(p1, solver=s, max_iters=5)
    v2, lam2, st, _ = gpu_step(p2, solver=s, max_iters=40, fixed_iters=True, reuse_w=True)
    stats1 = oracle.row_stats(oracle.system_matrix(p1))
    ref = oracle.vfpi(p2, max_iters=40, fixed_iters=True, stats=stats1)
    gate(v2, ref["v"], TOL, "reuse_w v")
    gate(lam2, ref["lam"], TOL, "reuse_w lambda")


def _step_all(p, **opt):
    v, lam, st, tp = gpu_step(p, tape=True, **opt)
    t = tape_parts(tp, p.n_nodes, p.n_contacts) if p.n_contacts else None
    return v, lam, st, t


@pytest.mark.parametrize("which", ["cloth128", "fem16x16x4", "fem16x16x4_regs5", "fem16x16x4_regs6",
                                   "fem16x16x4_regs8", "random700_regs1", "random700_regs5", "random700_regs6",
                                   "random700_regs8", "cloth_pair64_d", "random700_d_regs1", "random700_d_regs2"])
def test_lagged_residual_matches_synchronous(which):
    """The register-resident kernel takes the stop test of sweep l after
    sweep l + 1 and synchronizes each workgroup with its neighbours only (and,
    with D-contacts, with the workgroups that own a contact's partner node);
    with the sync bit it reduces over the whole grid after every sweep.  Both
    must stop on the same sweep with the same results, bit for bit: converged
    at several tolerances, stopped by max_iters (also at 1 and 2 sweeps), and
    at a fixed sweep count; the converged runs also against the oracle."""
    variant = 0
    if which == "cloth128":
        sc, x, v = scenes.cloth_cfg2(0)
        p = sc.assemble(x, v)
    elif which.startswith("fem16x16x4"):
        # (with 5, 6 and 8 chunk slots the lagged form keeps more levels on
        # chip than the synchronous one and streams the rest in other groups:
        # the same sums in the same order)
        sc, x, v = scenes.fem_ctx(0)
        p = sc.assemble(x, v)
        if which != "fem16x16x4":
            variant = 5 | (int(which[-1]) << 8) | (2 << 24)
    elif which == "cloth_pair64_d":
        p = scenes.cloth_pair_collision(0, side=64)
    elif which.startswith("random700_d"):
        p = scenes.random_problem(700, 300, 4, degree=5.0, phi_scale=0.5, n_d_contacts=120)
        variant = 5 | (int(which[-1]) << 8)
    else:
        p = scenes.random_problem(700, 300, 71, degree=5.0, phi_scale=0.5)
        nw = int(which[len("random700_regs"):])
        variant = 5 | (nw << 8) | ((1 << 24) if nw > 1 else 0)  # (LDS levels off: the short-row instances)
    sync = variant | (1 << 28)
    cases = [dict(max_iters=5000, tol=t) for t in (1e-3, 1e-5, 1e-8)]
    cases += [dict(max_iters=37, tol=1e-30), dict(max_iters=1, tol=1e-3), dict(max_iters=2, tol=1e-30),
              dict(max_iters=2, tol=1e30), dict(max_iters=25, fixed_iters=True)]
    for opt in cases:
        a = _step_all(p, variant=variant, **opt)
        b = _step_all(p, variant=sync, **opt)
        assert a[2] == b[2], (which, opt, a[2], b[2])
        assert np.array_equal(a[0].view(np.int64), b[0].view(np.int64)), (which, opt)
        assert np.array_equal(a[1].view(np.int64), b[1].view(np.int64)), (which, opt)
        if p.n_contacts:
            for k in ("w", "v", "lam_star", "branch"):
                assert np.array_equal(np.asarray(a[3][k]).view(np.uint8), np.asarray(b[3][k]).view(np.uint8)), k
        say(f"  {which} {opt}: iters={a[2]['iters']} status={a[2]['status']} theta={a[2]['theta']:.3e} "
            f"lagged == synchronous")
        if not opt.get("fixed_iters") and opt["max_iters"] == 5000:
            ref = oracle.vfpi(p, max_iters=opt["max_iters"], tol=opt["tol"])
            assert a[2]["status"] == _abi.VFPI_S_CONVERGED and abs(a[2]["iters"] - ref["iters"]) <= 1
            if a[2]["iters"] == ref["iters"]:
                gate(a[0], ref["v"], TOL, f"{which} tol={opt['tol']} v")
