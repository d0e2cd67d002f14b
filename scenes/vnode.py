"""Scenes whose contacts sit on virtual nodes (Sec. III-A, eq. vforce):
points that are not nodes of the model get a temporary node, tied to the
point's velocity J_v v_o.  A scene gives the original system (A_o, b_o), the
rows of J_v (one 3-row block row per virtual node, over the original nodes),
and contacts in the numbering [original nodes, virtual nodes].  Building the
augmented system of eq. vnode is left to the consumer."""
from __future__ import annotations

import dataclasses

import numpy as np

from .cloth import GRAVITY, cloth_cfg1
from .geometry import onb_duff
from .problem import rng


@dataclasses.dataclass
class VirtualScene:
    n_o: int                 # original nodes
    row_ptr: np.ndarray      # A_o, BSR 3x3
    col_idx: np.ndarray
    val: np.ndarray
    b: np.ndarray            # b_o [3 n_o]
    v0: np.ndarray           # warm start of the original nodes [3 n_o]
    jv_ptr: np.ndarray       # J_v block rows [n_v + 1]
    jv_col: np.ndarray       # original node of each block
    jv_val: np.ndarray       # [nnz_v, 3, 3]
    c_node: np.ndarray       # contacts over n_o + n_v nodes
    c_node_j: np.ndarray
    R: np.ndarray
    phi: np.ndarray
    mu: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_v(self) -> int:
        return int(self.jv_ptr.shape[0] - 1)


def _skew(r):
    return np.array([[0.0, -r[2], r[1]], [r[2], 0.0, -r[0]], [-r[1], r[0], 0.0]])


def rigid_box_on_floor(force=(0.0, 2.0, 0.0), mass=0.5, side=0.2, mu=0.2, h=0.01, g=9.81, v_k=(0, 0, 0),
                       w_k=(0, 0, 0)) -> VirtualScene:
    """A cube (edge ``side``, uniform density) resting on the floor z = 0 with a
    constant force at its centre; its velocity is two 3-DOF nodes (linear,
    angular), A_o = diag(m I, I_b I) with I_b = m side^2 / 6, b_o = A_o
    (v_k, w_k) + h (m g + F, 0).  The four bottom vertices carry the contacts,
    each on a virtual node with J_v = [I, -[r]_x] (velocity of the point at
    offset r from the centre)."""
    Ib = mass * side * side / 6.0
    val = np.stack([mass * np.eye(3), Ib * np.eye(3)])
    vk, wk = np.asarray(v_k, float), np.asarray(w_k, float)
    b = np.concatenate([mass * vk + h * (mass * np.array([0.0, 0.0, -g]) + np.asarray(force, float)), Ib * wk])
    hs = side / 2
    corners = np.array([[sx * hs, sy * hs, -hs] for sx in (-1, 1) for sy in (-1, 1)])
    jv_val = np.concatenate([np.stack([np.eye(3), -_skew(r)]) for r in corners])
    n_v = corners.shape[0]
    return VirtualScene(
        n_o=2, row_ptr=np.array([0, 1, 2]), col_idx=np.array([0, 1]), val=val, b=b,
        v0=np.concatenate([vk, wk]), jv_ptr=2 * np.arange(n_v + 1), jv_col=np.tile([0, 1], n_v), jv_val=jv_val,
        c_node=2 + np.arange(n_v), c_node_j=np.full(n_v, -1), R=onb_duff(np.tile([0.0, 0.0, 1.0], (n_v, 1))),
        phi=np.zeros(n_v), mu=np.full(n_v, mu),
        meta={"scene": "rigid_box", "mass": mass, "side": side, "force": tuple(force), "h": h, "g": g, "mu": mu})


def particles_on_cloth(seed: int, n_particles: int = 6, m_p: float = 0.05, speed: float = 0.5) -> VirtualScene:
    """The 10 x 10 landing cloth (S-contacts with the floor) with particles
    falling onto it: each particle is above a random point of a random
    triangle of the cloth grid, and its contact is a D-contact with a virtual
    node at that point (J_v = barycentric weights times I over the triangle's
    three nodes); normal +z, phi = gap / h."""
    sc, x, v = cloth_cfg1(seed)
    p = sc.assemble(x, v)
    g = rng("particles_on_cloth", seed, "placement")
    n = sc.side
    N = p.n_nodes
    cells = g.choice((n - 1) * (n - 1), size=n_particles, replace=False)
    ci, cj = cells // (n - 1), cells % (n - 1)
    upper = g.integers(0, 2, size=n_particles)
    tri = np.where(upper[:, None] == 0,
                   np.stack([ci * n + cj, ci * n + cj + 1, (ci + 1) * n + cj], 1),
                   np.stack([(ci + 1) * n + cj + 1, (ci + 1) * n + cj, ci * n + cj + 1], 1))
    bary = g.dirichlet(np.ones(3), size=n_particles)
    xs = x.reshape(-1, 3)
    pts = np.einsum("kt,ktd->kd", bary, xs[tri])
    gap = g.uniform(0.0, 3e-3, n_particles)
    px = pts + gap[:, None] * np.array([0.0, 0.0, 1.0])
    h = sc.h
    grav = GRAVITY
    pv = np.tile([0.0, 0.0, -speed], (n_particles, 1)) + g.normal(size=(n_particles, 3)) * 0.05
    # original system: cloth nodes, then particle nodes (A = m_p I)
    rp = np.concatenate([p.row_ptr, p.row_ptr[-1] + 1 + np.arange(n_particles)])
    col = np.concatenate([p.col_idx, N + np.arange(n_particles)])
    val = np.concatenate([p.val, np.tile(m_p * np.eye(3), (n_particles, 1, 1))])
    b = np.concatenate([p.b, (m_p * (pv + h * grav)).reshape(-1)])
    v0 = np.concatenate([p.v0, pv.reshape(-1)])
    n_o = N + n_particles
    jv_ptr = 3 * np.arange(n_particles + 1)
    jv_col = tri.reshape(-1)
    jv_val = bary.reshape(-1)[:, None, None] * np.eye(3)
    c_node = np.concatenate([p.c_node, N + np.arange(n_particles)])
    c_node_j = np.concatenate([np.full(p.n_contacts, -1), n_o + np.arange(n_particles)])
    R = np.concatenate([p.R, onb_duff(np.tile([0.0, 0.0, 1.0], (n_particles, 1)))])
    phi = np.concatenate([p.phi, gap / h])
    mu = np.concatenate([p.mu, np.full(n_particles, 0.4)])
    return VirtualScene(n_o=n_o, row_ptr=rp, col_idx=col, val=val, b=b, v0=v0, jv_ptr=jv_ptr, jv_col=jv_col,
                        jv_val=jv_val, c_node=c_node, c_node_j=c_node_j, R=R, phi=phi, mu=mu,
                        meta={"scene": "particles_on_cloth", "seed": seed, "triangles": tri})
