"""A seeded sweep over problem shapes and options on the HIP path vs the FP64
oracle at a fixed sweep count (bar 1e-9 element by element, branches per contact): node counts from 1 to a few
thousand (ragged last chunks), row lengths from 2 to ~40 blocks, S- and
D-contacts, both projections, omega, anisotropic friction, Chebyshev and BB
step sizes, and every launch kind, including workgroup caps."""
import numpy as np
import pytest

import oracle
import scenes
from oracle.chebyshev import vfpi_chebyshev
from tests.gpu_util import fixed_parity, say

pytestmark = pytest.mark.gpu

KINDS = [0, 1 | (1 << 8), 1 | (4 << 8) | (8 << 16), 2 | (2 << 8), 3 | (4 << 8), 4,
         5 | (1 << 8), 5 | (2 << 8), 5 | (4 << 8) | (2 << 24), 5 | (5 << 8), 5 | (6 << 8) | (1 << 24), 5 | (8 << 8),
         5 | (2 << 8) | (12 << 16)]


def _config(k):
    g = np.random.default_rng(1000 + k)
    n = int(g.choice([1, 3, 63, 64, 65, 129, 200, 511, 640, 1500, 3000]))
    nc = int(g.integers(0, n + 1))
    nd = int(g.integers(0, min(nc, n - nc) + 1)) if g.random() < 0.4 and n > 1 else 0
    deg = float(g.choice([2.0, 6.0, 12.0, 24.0]))
    p = scenes.random_problem(n, nc, 50 + k, degree=deg, phi_scale=0.5, n_d_contacts=nd)
    opt = {}
    r = g.random()
    if r < 0.15:
        opt["projection"] = "proximal"
    elif r < 0.3 and nd == 0 and nc > 0:
        p.mu2 = np.asarray(p.mu) * g.uniform(0.2, 1.5, size=nc)
    if g.random() < 0.3:
        opt["omega"] = float(g.choice([1e-3, 0.2]))
    accel = g.random()
    if accel < 0.2:
        opt["cheby_ls"] = int(g.integers(1, 6))
    elif accel < 0.35 and p.mu2 is None:
        opt["w_mode"] = str(g.choice(["bb1", "bb2"]))
    kind = int(g.choice(KINDS))
    if "w_mode" in opt and (kind & 0xff) not in (0, 1, 3, 5):
        kind = 0
    if p.mu2 is not None and opt.get("projection") == "proximal":
        opt.pop("projection")
    return p, opt, kind


@pytest.mark.parametrize("k", range(40))
def test_seeded_config_parity(k):
    p, opt, kind = _config(k)
    L = 9
    if "cheby_ls" in opt:
        ref = vfpi_chebyshev(p, max_iters=L, fixed_iters=True, l_s=opt["cheby_ls"], u=1.0,
                             omega=opt.get("omega", 0.0), projection=opt.get("projection", "strict"))
    else:
        ref = oracle.vfpi(p, max_iters=L, fixed_iters=True, **{a: b for a, b in opt.items()})
    o = dict(opt)
    proj = o.pop("projection", "strict")
    ev, el, st, ties = fixed_parity(p, ref, L, 1e-9, f"cfg {k}", projection=proj, variant=kind, **o)
    say(f"  cfg {k}: N={p.n_nodes} nc={p.n_contacts} D={int((p.c_node_j >= 0).sum())} "
        f"max row {int(np.diff(p.row_ptr).max()) if p.n_nodes else 0} variant={kind:#x} opt={opt} "
        f"aniso={p.mu2 is not None}: rel_v={ev:.2e} rel_lam={el:.2e} branch ties={ties}")
