"""Barzilai-Borwein step sizes (Sec. IV-C.2) on the GPU vs the FP64 oracle:
1e-9 at fixed sweep counts up to 30 (beyond that the quotients are formed from
differences near the rounding floor, where any two summation orders part), the
one-eigenspace closed form, and the converged solution against Frobenius W."""
import numpy as np
import pytest

import oracle
import paper_2201_09212_amd as vf
import scenes
from paper_2201_09212_amd import _abi
from tests.gpu_util import fixed_parity, gate, gpu_step, rel, say, solver_for, upload

pytestmark = pytest.mark.gpu

# kind | chunk slots << 8 | workgroup cap << 16
VARIANTS = {"grid_node1": 1 | (1 << 8), "grid_node2": 1 | (2 << 8), "grid_node4_cap8": 1 | (4 << 8) | (8 << 16),
            "wg1_node4": 3 | (4 << 8), "wg1_node16": 3 | (16 << 8), "default": 0,
            "regs_node1": 5 | (1 << 8), "regs_node2": 5 | (2 << 8), "regs_node5": 5 | (5 << 8),
            "regs_node8": 5 | (8 << 8), "regs_node2_lds_on": 5 | (2 << 8) | (2 << 24)}


def _problems():
    sc, x, v = scenes.cloth_cfg1(0)
    yield "cloth10", sc.assemble(x, v), 12
    yield "random700", scenes.random_problem(700, 300, 4, degree=5.0, phi_scale=0.5), 30
    sc, x, v = scenes.cloth_cfg2(0)
    yield "cloth128", sc.assemble(x, v), 30


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("mode", ["bb1", "bb2"])
def test_bb_fixed_sweeps_parity(variant, mode):
    for name, p, L in _problems():
        if name == "cloth128" and variant.startswith("wg1"):
            continue
        ref = oracle.vfpi(p, max_iters=L, fixed_iters=True, w_mode=mode)
        ev, el, st, ties = fixed_parity(p, ref, L, 1e-9, f"{name} {variant} {mode}", w_mode=mode,
                                        variant=VARIANTS[variant])
        say(f"  {name} {variant} {mode} L={L}: rel_v={ev:.2e} rel_lam={el:.2e} alpha={ref['alpha']:.4e} "
            f"branch ties={ties}")


@pytest.mark.parametrize("mode", ["bb1", "bb2"])
def test_bb_one_eigenspace_closed_form(mode):
    p, x = scenes.two_level_diagonal(300, 0)
    for var in (VARIANTS["grid_node1"], VARIANTS["wg1_node4"], VARIANTS["regs_node2"]):
        v, _, st, _ = gpu_step(p, max_iters=3, fixed_iters=True, w_mode=mode, variant=var)
        say(f"  two_level300 {mode} variant {var:#x}: |v - x*| = {np.abs(v.ravel() - x).max():.2e}")
        assert np.abs(v.ravel() - x).max() <= 1e-14 and st["theta"] <= 1e-14


def test_bb_converged_matches_frobenius_and_omega():
    p = scenes.random_problem(700, 300, 4, degree=5.0, phi_scale=0.5)
    ref = gpu_step(p, max_iters=100000, tol=1e-12)
    for mode in ("bb1", "bb2"):
        v, lam, st, _ = gpu_step(p, max_iters=100000, tol=1e-12, w_mode=mode)
        say(f"  random700 {mode}: {st['iters']} sweeps (Frobenius {ref[2]['iters']}), "
            f"rel_v={rel(v, ref[0]):.2e}")
        assert st["status"] == _abi.VFPI_S_CONVERGED
        gate(v, ref[0], 1e-9, f"{mode} converged v")
        gate(lam, ref[1], 1e-8, f"{mode} converged lambda")
    L = 25
    o = oracle.vfpi(p, max_iters=L, fixed_iters=True, w_mode="bb1", omega=0.05)
    fixed_parity(p, o, L, 1e-9, "bb1 omega", w_mode="bb1", omega=0.05)


def test_bb_unsupported_combinations():
    p = scenes.random_problem(100, 20, 1)
    s = solver_for(p)
    A, Jc, b, v = upload(p)
    with pytest.raises(vf.VfpiError, match="not supported"):
        s.step(A, b, Jc, v, w_mode="bb1", cheby_ls=5)
    for kind in (2, 4):
        with pytest.raises(vf.VfpiError, match="not supported"):
            s.step(A, b, Jc, v.clone(), w_mode="bb2", variant=kind)
