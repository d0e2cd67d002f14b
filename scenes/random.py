"""Random and analytic small problems for parity and edge-case tests."""
from __future__ import annotations

import numpy as np

from .fem import assemble_blocks
from .geometry import onb_duff
from .problem import Problem, rng


def random_problem(n_nodes: int, n_contacts: int, seed: int, *, degree: float = 6.0,
                   stiff: float = 1.0, phi_scale: float = 1.0, mu_range=(0.0, 1.0),
                   n_d_contacts: int = 0, tag: str = "random") -> Problem:
    """Random SPD block-sparse A of the form  diag(m_i I) + sum_edges L(B_e B_e^T)
    (a graph Laplacian of PSD 3x3 couplings, so A is SPD), with ``stiff``
    setting the coupling-to-mass ratio.  The node degree varies (ragged rows).
    Contacts: distinct random nodes with random unit normals; ``n_d_contacts``
    of them are node-node (D) contacts on further distinct nodes."""
    g = rng(tag, seed, f"{n_nodes}/{n_contacts}/{n_d_contacts}")
    n_edges = int(round(degree * n_nodes / 2))
    p = g.integers(0, n_nodes, size=n_edges)
    q = g.integers(0, n_nodes, size=n_edges)
    ok = p != q
    p, q = p[ok], q[ok]
    B = g.normal(size=(p.shape[0], 3, 3)) * np.sqrt(stiff / 3.0 / max(degree, 1.0))
    Kb = B @ B.transpose(0, 2, 1)
    mass = g.uniform(0.5, 2.0, size=n_nodes)
    rows = np.concatenate([p, q, p, q, np.arange(n_nodes)])
    cols = np.concatenate([p, q, q, p, np.arange(n_nodes)])
    blocks = np.concatenate([Kb, Kb, -Kb, -Kb, mass[:, None, None] * np.eye(3)])
    row_ptr, col_idx, val = assemble_blocks(n_nodes, rows, cols, blocks)
    b = g.normal(size=3 * n_nodes)
    v0 = g.normal(size=3 * n_nodes) * 0.5
    n_s = n_contacts - n_d_contacts
    assert n_s >= 0 and n_contacts + n_d_contacts <= n_nodes
    perm = g.permutation(n_nodes)
    c_node = perm[:n_contacts].astype(np.int32)
    c_j = np.full(n_contacts, -1, dtype=np.int32)
    if n_d_contacts:
        c_j[n_s:] = perm[n_contacts:n_contacts + n_d_contacts]
    nrm = g.normal(size=(n_contacts, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    R = onb_duff(nrm)
    phi = g.uniform(-phi_scale, phi_scale, size=n_contacts)
    mu = g.uniform(mu_range[0], mu_range[1], size=n_contacts)
    order = np.argsort(c_node, kind="stable")
    return Problem(n_nodes=n_nodes, row_ptr=row_ptr, col_idx=col_idx, val=val, b=b, v0=v0,
                   c_node=c_node[order], c_node_j=c_j[order], R=R[order], phi=phi[order], mu=mu[order],
                   meta={"scene": "random", "seed": seed})


def inclined_plane_particles(alpha, mu, mass=1.0, h=0.01, g=9.81, v_k=None, phi=None, mu2=None) -> Problem:
    """Independent particles, each resting on its own inclined plane through the
    origin with normal (sin a, 0, cos a) under gravity (0, 0, -g): A = m I,
    b = m (v_k + h g_vec), one S-contact per particle.  The tangent basis is
    rows 2-3 of the Duff frame of the normal."""
    alpha = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), alpha.shape).copy()
    mass = np.broadcast_to(np.asarray(mass, dtype=np.float64), alpha.shape).copy()
    n_p = alpha.shape[0]
    if v_k is None:
        v_k = np.zeros((n_p, 3))
    nrm = np.stack([np.sin(alpha), np.zeros_like(alpha), np.cos(alpha)], axis=1)
    R = onb_duff(nrm)
    gvec = np.array([0.0, 0.0, -g])
    b = mass[:, None] * (v_k + h * gvec)
    val = mass[:, None, None] * np.eye(3)
    return Problem(n_nodes=n_p, row_ptr=np.arange(n_p + 1), col_idx=np.arange(n_p), val=val,
                   b=b.reshape(-1), v0=np.asarray(v_k, dtype=np.float64).reshape(-1),
                   c_node=np.arange(n_p), c_node_j=np.full(n_p, -1),
                   R=R, phi=np.zeros(n_p) if phi is None else phi, mu=mu,
                   meta={"scene": "inclined_plane", "h": h, "g": g}, mu2=mu2)


def two_level_diagonal(n_nodes: int, seed: int, *, low=1.0, high=4.0, in_low_space=True) -> tuple:
    """Contact-free problem with A = diag(low on the first half of the nodes,
    high on the rest) and a warm start whose error x* - v0 lies in the `low`
    eigenspace only (or in both with ``in_low_space=False``).  Returns
    (problem, x*) with x* = A^-1 b.  Gershgorin gives alpha^1 = 1/high."""
    g = rng("two_level", seed, "vectors")
    half = n_nodes // 2
    dvec = np.where(np.arange(3 * n_nodes) < 3 * half, low, high)
    val = np.zeros((n_nodes, 3, 3))
    for k in range(3):
        val[:, k, k] = dvec[k::3]
    x = g.normal(size=3 * n_nodes)
    e = g.normal(size=3 * n_nodes)
    if in_low_space:
        e[3 * half:] = 0.0
    p = Problem(n_nodes, np.arange(n_nodes + 1), np.arange(n_nodes), val, dvec * x, x - e,
                np.zeros(0), np.zeros(0), np.zeros((0, 3, 3)), np.zeros(0), np.zeros(0),
                meta={"name": f"two_level{n_nodes}"})
    return p, x


def colliding_particle_pairs(m_i, m_j, normal, v_i, v_j, mu, h=0.01, g=9.81) -> Problem:
    """K independent particle pairs (i = 2k, j = 2k + 1), each pair in one
    D-contact whose frame R has ``normal`` (pointing from j to i) as its first
    row: A = diag(m I), b = m (v_k + h g), phi = 0."""
    m_i, m_j, mu = (np.atleast_1d(np.asarray(x, dtype=np.float64)) for x in (m_i, m_j, mu))
    K = m_i.shape[0]
    nrm = np.asarray(normal, dtype=np.float64).reshape(K, 3)
    nrm = nrm / np.linalg.norm(nrm, axis=1, keepdims=True)
    mass = np.stack([m_i, m_j], 1).reshape(-1)
    val = mass[:, None, None] * np.eye(3)
    vk = np.stack([np.asarray(v_i).reshape(K, 3), np.asarray(v_j).reshape(K, 3)], 1).reshape(-1, 3)
    b = (mass[:, None] * (vk + h * np.array([0.0, 0.0, -g]))).reshape(-1)
    n = 2 * K
    return Problem(n_nodes=n, row_ptr=np.arange(n + 1), col_idx=np.arange(n), val=val, b=b, v0=vk.reshape(-1),
                   c_node=2 * np.arange(K), c_node_j=2 * np.arange(K) + 1, R=onb_duff(nrm), phi=np.zeros(K),
                   mu=mu, meta={"scene": "particle_pairs"})
