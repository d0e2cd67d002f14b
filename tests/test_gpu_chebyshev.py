"""Chebyshev-accelerated V-FPI (Alg. 3) on the GPU vs the FP64 oracle
(oracle/chebyshev.py): 1e-9 relative at a fixed sweep count for the FP64
kernels, 1e-4 per environment for the batched FP32 kernel."""
import numpy as np
import pytest

import scenes
from oracle.chebyshev import vfpi_chebyshev
from paper_2201_09212_amd import _abi
from tests.gpu_util import fixed_parity, gate, gpu_step, say
from tests.test_gpu_batched import run_batched

pytestmark = pytest.mark.gpu

VARIANTS = {"grid_node2": 1 | (2 << 8), "grid_row1": 2, "regs2": 5 | (2 << 8), "wg1_node16": 3, "wg1_row5": 4}


def _problems():
    sc, x, v = scenes.cloth_cfg1(0)
    yield "cloth10", sc.assemble(x, v)
    yield "random700", scenes.random_problem(700, 300, 4, degree=5.0, phi_scale=0.5)
    sc, x, v = scenes.cloth_cfg2(0)
    yield "cloth128", sc.assemble(x, v)


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("ls,u", [(3, 1.0), (5, 0.8)])
def test_chebyshev_fixed_sweeps_parity(variant, ls, u):
    for name, p in _problems():
        if name == "cloth128" and variant.startswith("wg1"):
            continue
        L = 40
        ref = vfpi_chebyshev(p, max_iters=L, fixed_iters=True, l_s=ls, u=u)
        ev, el, st, ties = fixed_parity(p, ref, L, 1e-9, f"{name} {variant}", variant=VARIANTS[variant],
                                        cheby_ls=ls, cheby_u=u)
        say(f"  {name} {variant} ls={ls} u={u}: rel_v={ev:.2e} rel_lam={el:.2e} branch ties={ties}")


def test_chebyshev_converged_fewer_sweeps():
    sc, x, v = scenes.cloth_cfg2(0)
    p = sc.assemble(x, v)
    ref = vfpi_chebyshev(p, max_iters=5000, tol=1e-8, l_s=10)
    vv, lam, st, _ = gpu_step(p, max_iters=5000, tol=1e-8, cheby_ls=10)
    plain = gpu_step(p, max_iters=5000, tol=1e-8)[2]
    say(f"  cloth128 to 1e-8: plain {plain['iters']} sweeps, Chebyshev {st['iters']} (oracle {ref['iters']})")
    assert st["status"] == _abi.VFPI_S_CONVERGED and abs(st["iters"] - ref["iters"]) <= 1
    gate(vv, ref["v"], 1e-7, "cloth128 Chebyshev converged v")
    assert st["iters"] < plain["iters"]


@pytest.mark.parametrize("variant", [0, 4 | (16 << 8)])
def test_batched_chebyshev_parity(variant):
    from tests.test_gpu_batched import _envs_small
    envs = _envs_small()
    batch = scenes.concat_problems(envs)
    L = 30
    v, lam, st = run_batched(batch, max_iters=L, fixed_iters=True, cheby_ls=4, cheby_u=0.9, variant=variant)
    for e, pe in enumerate(envs):
        ref = vfpi_chebyshev(pe, max_iters=L, fixed_iters=True, l_s=4, u=0.9)
        n0, n1 = batch.env_node_off[e], batch.env_node_off[e + 1]
        m0, m1 = batch.env_con_off[e], batch.env_con_off[e + 1]
        gate(v[3 * n0:3 * n1], ref["v"], 1e-4, f"env {e} v")
        gate(lam[3 * m0:3 * m1], ref["lam"], 1e-4, f"env {e} lambda")
