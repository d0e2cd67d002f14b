"""Mass-spring cloth scenes (stand-ins for the paper's deformable workloads).

A square s x s grid of nodes, spacing 1 cm, node mass 0.01 kg, structural
(rest 1 cm) and shear (rest sqrt(2) cm) springs of stiffness k.  Each step is
the backward-Euler linearization of the spring potential with the
outer-product Hessian and no damping term (paper eq. gen_psi / hess_psi with
E = 0):

    A = M + h^2 K,   K = sum_springs k J_e^T J_e,   J_e = [d^T, -d^T]
    b = M v_k + h (f_spring(x_k) + M g)

This is the integrator the scenes use in place of the paper's midpoint form
(eq. akbk); the solver only needs A SPD and b.  ``lambda`` is then an impulse.

The block pattern is the 9-point node stencil, so every block row holds 4, 6
or 9 blocks and nnzb = (3s - 2)^2.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .geometry import contacts_from_gaps
from .problem import Problem, rng

GRAVITY = np.array([0.0, 0.0, -9.81])
# stencil offsets (dr, dc) -> slot (dr+1)*3 + (dc+1); slots are in column order
_SPRING_OFFSETS = [(0, 1), (1, 0), (1, 1), (1, -1)]


def _slot(dr, dc):
    return (dr + 1) * 3 + (dc + 1)


@dataclasses.dataclass
class ClothScene:
    side: int
    spacing: float = 0.01
    mass: float = 0.01
    k: float = 1.0e3
    h: float = 1.0 / 240.0
    delta: float = 0.005
    obstacles: list = dataclasses.field(default_factory=list)
    mu_node: np.ndarray | None = None
    damping: float = 0.0  # mass-proportional (air) damping c, 1/s, taken implicitly: A += h c M

    def __post_init__(self):
        s = self.side
        if self.mu_node is None:
            self.mu_node = np.full(s * s, 0.5)
        r, c = np.meshgrid(np.arange(s), np.arange(s), indexing="ij")
        self.rc = np.stack([r.ravel(), c.ravel()], axis=1)
        ex = np.zeros((s * s, 9), dtype=bool)
        for dr in (-1, 0, 1):
            for dc in (-1, 0, 1):
                rr, cc = self.rc[:, 0] + dr, self.rc[:, 1] + dc
                ex[:, _slot(dr, dc)] = (rr >= 0) & (rr < s) & (cc >= 0) & (cc < s)
        self.exists = ex
        nb = np.zeros((s * s, 9), dtype=np.int64)
        for dr in (-1, 0, 1):
            for dc in (-1, 0, 1):
                nb[:, _slot(dr, dc)] = (self.rc[:, 0] + dr) * s + (self.rc[:, 1] + dc)
        self.col_idx = nb[ex].astype(np.int32)
        self.row_ptr = np.zeros(s * s + 1, dtype=np.int32)
        np.cumsum(ex.sum(axis=1), out=self.row_ptr[1:])
        springs = []
        for dr, dc in _SPRING_OFFSETS:
            rr, cc = self.rc[:, 0] + dr, self.rc[:, 1] + dc
            ok = (rr >= 0) & (rr < s) & (cc >= 0) & (cc < s)
            p = np.nonzero(ok)[0]
            springs.append((dr, dc, p, rr[ok] * s + cc[ok]))
        self.springs = springs

    @property
    def n_nodes(self):
        return self.side * self.side

    def rest_positions(self, z0=0.0):
        s = self.side
        x = np.zeros((s * s, 3))
        x[:, 0] = (self.rc[:, 1] - (s - 1) / 2.0) * self.spacing
        x[:, 1] = (self.rc[:, 0] - (s - 1) / 2.0) * self.spacing
        x[:, 2] = z0
        return x

    def assemble(self, x: np.ndarray, v: np.ndarray, with_contacts=True) -> Problem:
        s2 = self.n_nodes
        K9 = np.zeros((s2, 9, 3, 3))
        f = np.zeros((s2, 3))
        for dr, dc, p, q in self.springs:
            rest = self.spacing * np.hypot(dr, dc)
            dx = x[p] - x[q]
            ln = np.linalg.norm(dx, axis=1)
            d = dx / ln[:, None]
            kb = self.k * d[:, :, None] * d[:, None, :]
            K9[p, 4] += kb
            K9[q, 4] += kb
            K9[p, _slot(dr, dc)] -= kb
            K9[q, _slot(-dr, -dc)] -= kb
            fs = -self.k * (ln - rest)[:, None] * d
            # p (and q) are distinct within one spring direction
            f[p] += fs
            f[q] -= fs
        A9 = (self.h * self.h) * K9
        A9[:, 4] += self.mass * (1.0 + self.h * self.damping) * np.eye(3)
        val = A9[self.exists]
        f += self.mass * GRAVITY
        b = self.mass * v.reshape(-1, 3) + self.h * f
        if with_contacts:
            cn, R, phi, mu = contacts_from_gaps(x, self.obstacles, self.delta, self.h, self.mu_node)
        else:
            cn, R, phi, mu = (np.zeros(0, np.int32), np.zeros((0, 3, 3)), np.zeros(0), np.zeros(0))
        return Problem(
            n_nodes=s2, row_ptr=self.row_ptr, col_idx=self.col_idx, val=val,
            b=b.reshape(-1), v0=v.reshape(-1).copy(), c_node=cn,
            c_node_j=np.full(cn.shape[0], -1, dtype=np.int32), R=R, phi=phi, mu=mu,
            meta={"scene": "cloth", "side": self.side, "h": self.h},
        )

    def advance(self, x, v_new):
        return x + self.h * v_new.reshape(-1, 3)


def cloth_cfg1(seed: int = 0, landing: bool = True):
    """10x10 cloth, mu = 0.5, plane z = 0, h = 1/240, jitter +-1 mm in x/y.

    Returns (scene, x, v).  With ``landing`` the state is the moment of
    touchdown after a 2 cm drop (every node within the 5 mm contact margin,
    falling at sqrt(2 g 0.02)), else the initial state 2 cm up at rest."""
    g = rng("cloth10", seed, "state")
    sc = ClothScene(side=10, obstacles=[("plane", (0, 0, 0), (0, 0, 1))])
    x = sc.rest_positions(0.02)
    x[:, :2] += g.uniform(-1e-3, 1e-3, size=(sc.n_nodes, 2))
    v = np.zeros((sc.n_nodes, 3))
    if landing:
        x[:, 2] = g.uniform(-5e-4, 4e-3, size=sc.n_nodes)
        v[:, 2] = -np.sqrt(2 * 9.81 * 0.02)
        v += g.normal(0.0, 0.01, size=v.shape)
    return sc, x, v


def cloth_cfg2(seed: int = 0):
    """128x128 cloth draped over 16 fixed spheres (r ~ U[5,15] cm, centres at
    z = 0, seeded, non-overlapping in xy), per-node mu ~ U[0.2, 0.8], no floor.

    Returns (scene, x, v): a draped snapshot built procedurally (no solver
    involved): over each sphere the cloth follows the cap (plus a gap in
    [-0.5, 1] mm) out to 0.92 r, then falls off along the cap's tangent; the
    height is the max over spheres.  Nodes hanging between spheres move
    downward at ~0.1 m/s."""
    s = 128
    g = rng("cloth128", seed, "scene")
    half = (s - 1) / 2 * 0.01
    centers, radii = [], []
    while len(centers) < 16:
        r = g.uniform(0.05, 0.15)
        c = g.uniform(-half + 0.05, half - 0.05, size=2)
        if all(np.hypot(*(c - c2)) > r + r2 + 0.01 for c2, r2 in zip(centers, radii)):
            centers.append(c)
            radii.append(r)
    obstacles = [("sphere", (c[0], c[1], 0.0), r) for c, r in zip(centers, radii)]
    mu = g.uniform(0.2, 0.8, size=s * s)
    sc = ClothScene(side=s, obstacles=obstacles, mu_node=mu)
    x = sc.rest_positions(0.0)
    gap = g.uniform(-5e-4, 1e-3, size=s * s)
    z = np.full(s * s, -1.0)
    for c, r in zip(centers, radii):
        rho = np.hypot(x[:, 0] - c[0], x[:, 1] - c[1])
        r1 = 0.92 * r
        z1 = np.sqrt(r * r - r1 * r1)
        slope = r1 / z1
        cap = np.where(rho <= r1, np.sqrt(np.maximum(r * r - rho * rho, 0.0)), z1 - slope * (rho - r1))
        z = np.maximum(z, cap)
    x[:, 2] = np.maximum(z, -0.3) + gap
    v = g.normal(0.0, 0.02, size=(s * s, 3))
    v[:, 2] -= np.where(z < 0.0, 0.1, 0.0)
    return sc, x, v


def cloth_cfg2_drop(seed: int = 0, damping: float = 5.0):
    """The 128x128 cloth of ``cloth_cfg2`` (same 16 spheres, same per-node mu),
    flat and at rest 5 mm above the highest sphere, to be dropped onto them:
    the rollout form of that workload.  Contacts appear as the cloth lands
    and reach about 5,000.  ``damping`` is a mass-proportional damping
    coefficient (1/s, air drag, taken implicitly); without it the undamped
    drop stops converging after about 60 steps, in the oracle as on the GPU.
    Returns (scene, x, v)."""
    sc, _, _ = cloth_cfg2(seed)
    sc.damping = float(damping)
    top = max(o[2] for o in sc.obstacles)
    x = sc.rest_positions(top + 0.005)
    return sc, x, np.zeros_like(x)


def cloth_drape(side: int, seed: int = 0):
    """A side x side cloth draped over fixed spheres, for the size sweep: the
    cloth128 recipe (r ~ U[5,15] cm, centres at z = 0, non-overlapping in xy,
    per-node mu ~ U[0.2, 0.8], cap plus a gap in [-0.5, 1] mm out to 0.92 r,
    then the tangent fall-off, hanging parts clipped at -0.3 m and falling at
    0.1 m/s) with the sphere count scaled with the area, 16 per 128 x 128.
    Each sphere only shapes the nodes its cap and fall-off reach.  Returns
    (scene, x, v)."""
    s = int(side)
    g = rng("cloth_drape", seed, f"side{s}")
    half = (s - 1) / 2 * 0.01
    n_sph = max(1, int(round(16 * (s / 128.0) ** 2)))
    centers, radii = [], []
    tries = 0
    while len(centers) < n_sph and tries < 200 * n_sph:
        tries += 1
        r = g.uniform(0.05, min(0.15, half - 0.01))
        c = g.uniform(-half + r, half - r, size=2)
        if all(np.hypot(*(c - c2)) > r + r2 + 0.01 for c2, r2 in zip(centers, radii)):
            centers.append(c)
            radii.append(r)
    obstacles = [("sphere", (c[0], c[1], 0.0), r) for c, r in zip(centers, radii)]
    mu = g.uniform(0.2, 0.8, size=s * s)
    sc = ClothScene(side=s, obstacles=obstacles, mu_node=mu)
    x = sc.rest_positions(0.0)
    gap = g.uniform(-5e-4, 1e-3, size=s * s)
    z = np.full((s, s), -0.3)
    xs = x[:, 0].reshape(s, s)
    ys = x[:, 1].reshape(s, s)
    for c, r in zip(centers, radii):
        r1 = 0.92 * r
        z1 = np.sqrt(r * r - r1 * r1)
        slope = r1 / z1
        reach = r1 + (z1 + 0.3) / slope
        c0 = max(0, int(np.floor((c[0] - reach + half) / 0.01)))
        c1 = min(s, int(np.ceil((c[0] + reach + half) / 0.01)) + 1)
        r0 = max(0, int(np.floor((c[1] - reach + half) / 0.01)))
        r1i = min(s, int(np.ceil((c[1] + reach + half) / 0.01)) + 1)
        rho = np.hypot(xs[r0:r1i, c0:c1] - c[0], ys[r0:r1i, c0:c1] - c[1])
        cap = np.where(rho <= r1, np.sqrt(np.maximum(r * r - rho * rho, 0.0)), z1 - slope * (rho - r1))
        z[r0:r1i, c0:c1] = np.maximum(z[r0:r1i, c0:c1], cap)
    z = z.ravel()
    x[:, 2] = z + gap
    v = g.normal(0.0, 0.02, size=(s * s, 3))
    v[:, 2] -= np.where(z < 0.0, 0.1, 0.0)
    return sc, x, v


def cloth_cfg4_envs(seed: int = 0, n_env: int = 2048, smin: int = 8, smax: int = 48):
    """Batched cloth environments: side s ~ U{smin..smax}, mu_env ~ U[0.1, 0.9],
    drop height H ~ U[0, 5] cm onto the plane z = 0, h = 1/240.

    Each environment is a snapshot of its drop: the cloth (tilted by up to 3
    degrees) sits at height H - 2.5 cm clipped below at 0.5 mm, so about half
    of the environments rest on the plane (all or part of their nodes inside
    the 5 mm margin) and the rest are still falling with no contacts.
    Returns a list of (scene, x, v)."""
    g = rng("cloth_batched", seed, "envs")
    out = []
    for e in range(n_env):
        s = int(g.integers(smin, smax + 1))
        mu_env = g.uniform(0.1, 0.9)
        H = g.uniform(0.0, 0.05)
        tilt = np.tan(np.deg2rad(g.uniform(-3.0, 3.0, size=2)))
        sc = ClothScene(side=s, obstacles=[("plane", (0, 0, 0), (0, 0, 1))], mu_node=np.full(s * s, mu_env))
        x = sc.rest_positions(0.0)
        zc = max(H - 0.025, 0.0)
        x[:, 2] = zc + tilt[0] * x[:, 0] + tilt[1] * x[:, 1]
        x[:, 2] -= min(x[:, 2].min() - 5e-4, 0.0) if zc == 0.0 else 0.0
        x[:, :2] += g.uniform(-1e-3, 1e-3, size=(s * s, 2))
        v = g.normal(0.0, 0.01, size=(s * s, 3))
        v[:, 2] -= np.sqrt(2 * 9.81 * max(H - zc, 0.0))
        out.append((sc, x, v))
    return out


def cloth_cfg5_scene(seed: int = 0, side: int = 64):
    """64x64 cloth dropped 2 cm onto the plane z = 0, mu = 0.5, k = 1e3,
    initial velocities ~ N(0, 0.05 m/s).  Returns (scene, x0, v0)."""
    g = rng("cloth64_adjoint", seed, "state")
    sc = ClothScene(side=side, obstacles=[("plane", (0, 0, 0), (0, 0, 1))], mu_node=np.full(side * side, 0.5))
    x = sc.rest_positions(0.02)
    x[:, :2] += g.uniform(-1e-3, 1e-3, size=(sc.n_nodes, 2))
    v = g.normal(0.0, 0.05, size=(sc.n_nodes, 3))
    return sc, x, v


def cloth_pair_collision(seed: int = 0, side: int = 32, speed: float = 0.3):
    """Two equal cloth sheets meeting in free fall (no obstacles): the lower
    one at z = 0 moving up, the upper one a few mm above moving down, with
    +-1 mm x/y jitter.  Every upper node within the 5 mm margin of the lower
    node under it is in a D-contact with it (normal +z, R on the upper node,
    -R on the lower one, phi = gap / h, mu = 0.5).  Returns the Problem over
    both sheets (lower sheet first)."""
    g = rng(f"cloth_pair{side}", seed, "state")
    sc = ClothScene(side=side)
    n = sc.n_nodes
    xl = sc.rest_positions(0.0)
    xu = sc.rest_positions(0.0)
    xu[:, :2] += g.uniform(-1e-3, 1e-3, size=(n, 2))
    xu[:, 2] = g.uniform(1e-3, 7e-3, size=n)
    vl = np.tile([0.0, 0.0, speed], (n, 1)) + g.normal(size=(n, 3)) * 0.02
    vu = np.tile([0.0, 0.0, -speed], (n, 1)) + g.normal(size=(n, 3)) * 0.02
    pl = sc.assemble(xl, vl, with_contacts=False)
    pu = sc.assemble(xu, vu, with_contacts=False)
    gap = xu[:, 2] - xl[:, 2]
    hit = np.nonzero(gap <= sc.delta)[0]
    from .geometry import onb_duff
    R = onb_duff(np.tile([0.0, 0.0, 1.0], (hit.shape[0], 1)))
    row_ptr = np.concatenate([pl.row_ptr, pl.row_ptr[-1] + pu.row_ptr[1:]])
    return Problem(
        n_nodes=2 * n, row_ptr=row_ptr, col_idx=np.concatenate([pl.col_idx, pu.col_idx + n]),
        val=np.concatenate([pl.val, pu.val]), b=np.concatenate([pl.b, pu.b]), v0=np.concatenate([pl.v0, pu.v0]),
        c_node=n + hit, c_node_j=hit, R=R, phi=gap[hit] / sc.h, mu=np.full(hit.shape[0], 0.5),
        meta={"scene": "cloth_pair", "side": side, "seed": seed})
