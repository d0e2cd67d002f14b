"""Collision geometry for the synthetic scenes: analytic planes and spheres,
closest-obstacle nodal contacts, and the contact frame.

Contact nodalization (paper Sec. III-A): every contact acts on a mesh node, so
the contact Jacobian row is ``[0 .. R .. 0]`` with ``R`` in SO(3).  The paper
does not say how the tangent basis is chosen; any orthonormal completion of the
normal works (the velocity solution is basis-invariant).  Here it is the
branch-free construction of Duff et al., "Building an Orthonormal Basis,
Revisited" (JCGT 2017).  The normal offset ``phi`` is not given a formula in the
paper (eq. scc only calls it a penetration-compensation term); these scenes use
phi = d / h, d being the signed gap at the start of the step, which is the
backward-Euler non-penetration condition for x_{k+1} = x_k + h v.
"""
from __future__ import annotations

import numpy as np


def onb_duff(nrm: np.ndarray) -> np.ndarray:
    """Rows [n, t1, t2] for unit normals ``nrm[m,3]`` -> ``R[m,3,3]`` in SO(3)."""
    nx, ny, nz = nrm[:, 0], nrm[:, 1], nrm[:, 2]
    sign = np.where(nz >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + nz)
    bb = nx * ny * a
    t1 = np.stack([1.0 + sign * nx * nx * a, sign * bb, -sign * nx], axis=1)
    t2 = np.stack([bb, sign + ny * ny * a, -ny], axis=1)
    return np.stack([nrm, t1, t2], axis=1)


def plane_gap(x: np.ndarray, point, normal):
    normal = np.asarray(normal, dtype=np.float64)
    normal = normal / np.linalg.norm(normal)
    d = (x - np.asarray(point, dtype=np.float64)) @ normal
    return d, np.broadcast_to(normal, x.shape)


def sphere_gap(x: np.ndarray, center, radius):
    r = x - np.asarray(center, dtype=np.float64)
    dist = np.linalg.norm(r, axis=1)
    nrm = r / np.maximum(dist, 1e-12)[:, None]
    return dist - radius, nrm


def _sphere_bins(x: np.ndarray, cell: float):
    """Nodes binned on an xy grid of ``cell``-sized squares: (sorted order,
    bin keys in that order, x/y bin origin)."""
    ij = np.floor(x[:, :2] / cell).astype(np.int64)
    o = ij.min(axis=0)
    ij -= o
    ny = int(ij[:, 1].max()) + 1
    key = ij[:, 0] * ny + ij[:, 1]
    order = np.argsort(key, kind="stable")
    return order, key[order], o, ny


def contacts_from_gaps(x: np.ndarray, obstacles: list, delta: float, h: float, mu_node: np.ndarray):
    """One contact per node, with the closest obstacle, if its signed gap is
    at most ``delta`` (speculative contacts).  ``obstacles`` is a list of
    ("plane", point, normal) / ("sphere", center, radius).  Returns
    (c_node, R, phi, mu) sorted by node index.

    With many spheres each one is only tested against the nodes whose xy bin
    lies within radius + delta of its centre; a node outside that window has a
    gap above delta for that sphere, so the contacts are the same as testing
    every node against every obstacle."""
    n_nodes = x.shape[0]
    best_d = np.full(n_nodes, np.inf)
    best_n = np.zeros((n_nodes, 3))
    radii = [float(ob[2]) for ob in obstacles if ob[0] == "sphere"]
    bins = None
    if len(radii) > 8 and n_nodes > 0:
        cell = max(radii) + delta
        bins = _sphere_bins(x, cell)
    for ob in obstacles:
        if ob[0] == "plane":
            d, nrm = plane_gap(x, ob[1], ob[2])
            idx = None
        elif ob[0] == "sphere":
            if bins is None:
                d, nrm = sphere_gap(x, ob[1], ob[2])
                idx = None
            else:
                order, keys, o, ny = bins
                reach = float(ob[2]) + delta
                c = np.asarray(ob[1], dtype=np.float64)
                lo = np.floor((c[:2] - reach) / cell).astype(np.int64) - o
                hi = np.floor((c[:2] + reach) / cell).astype(np.int64) - o
                parts = []
                for bx in range(max(lo[0], 0), hi[0] + 1):
                    a = np.searchsorted(keys, bx * ny + max(lo[1], 0), "left")
                    b = np.searchsorted(keys, bx * ny + min(hi[1], ny - 1), "right")
                    parts.append(order[a:b])
                idx = np.sort(np.concatenate(parts)) if parts else np.zeros(0, np.int64)
                d, nrm = sphere_gap(x[idx], ob[1], ob[2])
        else:
            raise ValueError(ob[0])
        if idx is None:
            closer = d < best_d
            best_d = np.where(closer, d, best_d)
            best_n[closer] = nrm[closer]
        else:
            closer = d < best_d[idx]
            best_d[idx[closer]] = d[closer]
            best_n[idx[closer]] = nrm[closer]
    nodes = np.nonzero(best_d <= delta)[0].astype(np.int32)
    R = onb_duff(best_n[nodes])
    phi = best_d[nodes] / h
    return nodes, R, phi, np.asarray(mu_node, dtype=np.float64)[nodes]
