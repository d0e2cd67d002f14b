"""Co-rotated linear FEM soft block (stand-in for the paper's co-rotational
FEM scenes: soft mat, soft ball, soft gripper).

The block is a grid of nx x ny x nz hexahedral cells of 1 cm, each split into 5
tetrahedra with alternating parity so that face diagonals match.  Per tet the
linear stiffness is K_e = V (lam g_a g_b^T + mu g_b g_a^T + mu (g_a.g_b) I) for
shape-function gradients g_a; it is co-rotated with the rotation R_e of the polar
decomposition of the deformation gradient: K = sum R_e K_e R_e^T and elastic
force f = -R_e K_e (R_e^T x - X).  Mass is lumped (rho V / 4 per tet node).
The step matrix is the same backward-Euler form as the cloth:
A = M + h^2 K, b = M v + h (f + M g).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .cloth import GRAVITY
from .geometry import contacts_from_gaps
from .problem import Problem, rng

_EVEN = [(0, 1, 2, 4), (3, 2, 1, 7), (5, 4, 7, 1), (6, 7, 4, 2), (1, 2, 4, 7)]
_ODD = [(1, 0, 3, 5), (2, 3, 0, 6), (4, 5, 6, 0), (7, 6, 5, 3), (0, 3, 5, 6)]


def assemble_blocks(n_nodes, rows, cols, blocks):
    """Sum 3x3 block contributions into sorted block-sparse rows."""
    key = rows.astype(np.int64) * n_nodes + cols.astype(np.int64)
    uniq, inv = np.unique(key, return_inverse=True)
    flat = blocks.reshape(-1, 9)
    val = np.empty((uniq.shape[0], 9))
    for e in range(9):
        val[:, e] = np.bincount(inv, weights=flat[:, e], minlength=uniq.shape[0])
    r = (uniq // n_nodes).astype(np.int64)
    c = (uniq % n_nodes).astype(np.int32)
    row_ptr = np.zeros(n_nodes + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n_nodes), out=row_ptr[1:])
    return row_ptr.astype(np.int32), c, val.reshape(-1, 3, 3)


def polar_rotation(F):
    U, _, Vt = np.linalg.svd(F)
    d = np.sign(np.linalg.det(U @ Vt))
    U[:, :, 2] *= d[:, None]
    return U @ Vt


@dataclasses.dataclass
class FemScene:
    cells: tuple = (64, 64, 16)
    spacing: float = 0.01
    young: float = 1.0e5
    poisson: float = 0.4
    rho: float = 1000.0
    h: float = 1.0e-3
    delta: float = 0.03
    obstacles: list = dataclasses.field(default_factory=list)
    mu: float = 0.6

    def __post_init__(self):
        cx, cy, cz = self.cells
        nx, ny, nz = cx + 1, cy + 1, cz + 1
        self.dims = (nx, ny, nz)
        gi, gj, gk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        # node index: k-major slabs? use (k, j, i) ordering: i fastest
        self.X = np.zeros((nx * ny * nz, 3))
        idx = lambda i, j, k: (k * ny + j) * nx + i
        ii, jj, kk = gi.ravel(), gj.ravel(), gk.ravel()
        self.X[idx(ii, jj, kk)] = np.stack([ii, jj, kk], axis=1) * self.spacing
        self.X[:, 0] -= cx * self.spacing / 2
        self.X[:, 1] -= cy * self.spacing / 2
        ci, cj, ck = np.meshgrid(np.arange(cx), np.arange(cy), np.arange(cz), indexing="ij")
        ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
        corner = np.stack([idx(ci + (b & 1), cj + ((b >> 1) & 1), ck + ((b >> 2) & 1)) for b in range(8)], axis=1)
        parity = (ci + cj + ck) & 1
        tets = []
        for par, table in ((0, _EVEN), (1, _ODD)):
            sel = corner[parity == par]
            for t in table:
                tets.append(sel[:, list(t)])
        self.tets = np.concatenate(tets).astype(np.int64)
        Xt = self.X[self.tets]
        Dm = np.stack([Xt[:, 1] - Xt[:, 0], Xt[:, 2] - Xt[:, 0], Xt[:, 3] - Xt[:, 0]], axis=2)
        self.vol = np.abs(np.linalg.det(Dm)) / 6.0
        self.Dm_inv = np.linalg.inv(Dm)
        gr = self.Dm_inv  # rows are grad N_1..3
        g0 = -gr.sum(axis=1)
        self.grads = np.concatenate([g0[:, None, :], gr], axis=1)  # [T,4,3]
        lam = self.young * self.poisson / ((1 + self.poisson) * (1 - 2 * self.poisson))
        mu_l = self.young / (2 * (1 + self.poisson))
        G = self.grads
        gg = np.einsum("tai,tbi->tab", G, G)
        Ke = (lam * np.einsum("tai,tbj->tabij", G, G)
              + mu_l * np.einsum("tbi,taj->tabij", G, G)
              + mu_l * gg[:, :, :, None, None] * np.eye(3))
        self.Ke = Ke * self.vol[:, None, None, None, None]  # [T,4,4,3,3]
        self.mass = np.zeros(self.X.shape[0])
        np.add.at(self.mass, self.tets.ravel(), np.repeat(self.rho * self.vol / 4.0, 4))
        self.rows = np.repeat(self.tets, 4, axis=1).ravel()
        self.cols = np.tile(self.tets, (1, 4)).ravel()

    @property
    def n_nodes(self):
        return self.X.shape[0]

    def assemble(self, x: np.ndarray, v: np.ndarray) -> Problem:
        xt = x[self.tets]
        Ds = np.stack([xt[:, 1] - xt[:, 0], xt[:, 2] - xt[:, 0], xt[:, 3] - xt[:, 0]], axis=2)
        Re = polar_rotation(Ds @ self.Dm_inv)
        Kc = np.einsum("tij,tabjk,tlk->tabil", Re, self.Ke, Re, optimize=True)
        # f_a = -R sum_b K_ab (R^T x_b - X_b)
        loc = np.einsum("tji,tbj->tbi", Re, xt) - self.X[self.tets]
        fe = -np.einsum("tij,tabjk,tbk->tai", Re, self.Ke, loc, optimize=True)
        f = np.zeros_like(x)
        np.add.at(f, self.tets.ravel(), fe.reshape(-1, 3))
        blocks = (self.h * self.h) * Kc.reshape(-1, 3, 3)
        n = self.n_nodes
        rows = np.concatenate([self.rows, np.arange(n)])
        cols = np.concatenate([self.cols, np.arange(n)])
        blocks = np.concatenate([blocks, self.mass[:, None, None] * np.eye(3)])
        row_ptr, col_idx, val = assemble_blocks(n, rows, cols, blocks)
        f += self.mass[:, None] * GRAVITY
        b = self.mass[:, None] * v + self.h * f
        cn, R, phi, mu = contacts_from_gaps(x, self.obstacles, self.delta, self.h, np.full(n, self.mu))
        return Problem(
            n_nodes=n, row_ptr=row_ptr, col_idx=col_idx, val=val, b=b.reshape(-1), v0=v.reshape(-1).copy(),
            c_node=cn, c_node_j=np.full(cn.shape[0], -1, np.int32), R=R, phi=phi, mu=mu,
            meta={"scene": "fem", "cells": self.cells, "h": self.h},
        )


def _fem_snapshot(cells, n_spheres, rmin, rmax, delta, seed, tag):
    g = rng(tag, seed, "scene")
    cx, cy, cz = cells
    hx, hy = cx * 0.01 / 2, cy * 0.01 / 2
    spheres = []
    while len(spheres) < n_spheres:
        r = g.uniform(rmin, rmax)
        c = g.uniform([-hx + r, -hy + r], [hx - r, hy - r])
        if all(np.hypot(*(c - c2)) > r + r2 for c2, r2, _ in spheres):
            spheres.append((c, r, g.uniform(0.002, 0.006)))
    obstacles = [("plane", (0, 0, 0), (0, 0, 1))]
    obstacles += [("sphere", (c[0], c[1], p - r), r) for c, r, p in spheres]
    sc = FemScene(cells=cells, delta=delta, obstacles=obstacles)
    X = sc.X
    x = X.copy()
    x[:, 2] += 0.001
    H = cz * 0.01
    bump = np.zeros(X.shape[0])
    for c, r, p in spheres:
        rho2 = (X[:, 0] - c[0]) ** 2 + (X[:, 1] - c[1]) ** 2
        top = np.sqrt(np.maximum(r * r - rho2, 0.0)) - (r - p)
        bump = np.maximum(bump, top + 0.0005)
    x[:, 2] += np.maximum(bump - 0.001, 0.0) * (1.0 - X[:, 2] / H)
    # slight sag under gravity plus noise
    x[:, 2] -= 0.0005 * (X[:, 2] / H) * (1.0 - X[:, 2] / H)
    x += g.normal(0.0, 1e-4, size=x.shape)
    v = g.normal(0.0, 0.005, size=x.shape)
    v[:, 2] -= 0.05
    return sc, x, v


def fem_cfg3(seed: int = 0):
    """64 x 64 x 16 cells (71,825 nodes), E = 1e5 Pa, nu = 0.4, rho = 1000,
    h = 1e-3 s, plane z = 0 plus 8 spheres (r ~ U[2,6] cm) protruding 2-6 mm
    through it, mu = 0.6.  The block rests 1 mm above the plane, bent over the
    sphere caps.  Speculative contact margin 2.5 cm."""
    return _fem_snapshot((64, 64, 16), 8, 0.02, 0.06, 0.025, seed, "fem64x64x16")


def fem_ctx(seed: int = 0):
    """Paper-size block: 16 x 16 x 4 cells (1,445 nodes, 4,335 DOF), same
    material and obstacles scaled down (2 spheres)."""
    return _fem_snapshot((16, 16, 4), 2, 0.02, 0.04, 0.025, seed, "fem16x16x4")


def fem_block(cells, seed: int = 0):
    """FEM block of any size for the size sweep: the FEM-block recipe (same
    material, h, margin and obstacle sizes) with the sphere count scaled with
    the footprint, 8 per 64 x 64 cells (at least 2)."""
    cx, cy, cz = (int(c) for c in cells)
    n_sph = max(2, int(round(8 * cx * cy / (64.0 * 64.0))))
    return _fem_snapshot((cx, cy, cz), n_sph, 0.02, 0.06, 0.025, seed, f"fem{cx}x{cy}x{cz}")
