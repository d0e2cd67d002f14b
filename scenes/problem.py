"""Container for one time step's contact problem and its batched concatenation.

Layout (the same one the C ABI takes, see include/vfpi.h):

* ``A`` in block-sparse row form with 3x3 blocks (one block row per node):
  ``row_ptr[N+1]`` (int32), ``col_idx[nnzb]`` (int32, sorted within a row),
  ``val[nnzb,3,3]`` row-major blocks.  A is symmetric positive definite
  (paper Sec. II-A, eq. akbk and the remark after it).
* ``b``, ``v0``: node-major ``[3N]`` (x, y, z of node 0, then node 1, ...).
* contacts (paper eq. jcnode): contact m acts on node ``c_node[m]``; for a
  D-contact also on ``c_node_j[m]`` (else -1).  ``R[m]`` is the SO(3) frame whose
  first row is the contact normal and rows 2-3 the tangents, so that the contact
  Jacobian block row is ``[.. R ..]`` (S) or ``[.. R .. -R ..]`` (D).
  ``phi[m]`` is the normal offset term, ``mu[m]`` the friction coefficient
  (eq. scc).
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np


def rng(config: str, seed: int, purpose: str) -> np.random.Generator:
    """Independent PCG64 stream keyed by (config, seed, purpose)."""
    key = hashlib.sha256(f"{config}|{seed}|{purpose}".encode()).digest()
    words = np.frombuffer(key, dtype=np.uint32)
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(words.tolist())))


@dataclasses.dataclass
class Problem:
    n_nodes: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    b: np.ndarray
    v0: np.ndarray
    c_node: np.ndarray
    c_node_j: np.ndarray
    R: np.ndarray
    phi: np.ndarray
    mu: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)
    mu2: np.ndarray | None = None  # anisotropic friction: coefficient along tangent 2 (mu along tangent 1)

    def __post_init__(self):
        self.row_ptr = np.ascontiguousarray(self.row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(self.col_idx, dtype=np.int32)
        self.val = np.ascontiguousarray(self.val, dtype=np.float64).reshape(-1, 3, 3)
        self.b = np.ascontiguousarray(self.b, dtype=np.float64).reshape(-1)
        self.v0 = np.ascontiguousarray(self.v0, dtype=np.float64).reshape(-1)
        self.c_node = np.ascontiguousarray(self.c_node, dtype=np.int32).reshape(-1)
        self.c_node_j = np.ascontiguousarray(self.c_node_j, dtype=np.int32).reshape(-1)
        self.R = np.ascontiguousarray(self.R, dtype=np.float64).reshape(-1, 3, 3)
        self.phi = np.ascontiguousarray(self.phi, dtype=np.float64).reshape(-1)
        self.mu = np.ascontiguousarray(self.mu, dtype=np.float64).reshape(-1)
        if self.mu2 is not None:
            self.mu2 = np.ascontiguousarray(self.mu2, dtype=np.float64).reshape(-1)
            assert self.mu2.shape == self.mu.shape
        n = 3 * self.n_nodes
        assert self.row_ptr.shape == (self.n_nodes + 1,)
        assert self.col_idx.shape == (self.nnzb,)
        assert self.b.shape == (n,) and self.v0.shape == (n,)
        nc = self.c_node.shape[0]
        assert self.c_node_j.shape == (nc,) and self.R.shape == (nc, 3, 3)
        assert self.phi.shape == (nc,) and self.mu.shape == (nc,)

    @property
    def nnzb(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n_contacts(self) -> int:
        return int(self.c_node.shape[0])

    @property
    def n(self) -> int:
        return 3 * self.n_nodes

    def jc_bsr(self):
        """J_c as a block-sparse matrix: one block row per contact holding R at
        column ``c_node`` and, for a D-contact, -R at column ``c_node_j`` (in that
        storage order).  Returns (row_ptr[nc+1], col_idx[nnzb_c], val[nnzb_c,3,3])."""
        nc = self.n_contacts
        is_d = self.c_node_j >= 0
        counts = 1 + is_d.astype(np.int32)
        row_ptr = np.zeros(nc + 1, dtype=np.int32)
        np.cumsum(counts, out=row_ptr[1:])
        col = np.empty(int(row_ptr[-1]), dtype=np.int32)
        val = np.empty((int(row_ptr[-1]), 3, 3), dtype=np.float64)
        col[row_ptr[:-1]] = self.c_node
        val[row_ptr[:-1]] = self.R
        dpos = row_ptr[:-1][is_d] + 1
        col[dpos] = self.c_node_j[is_d]
        val[dpos] = -self.R[is_d]
        return row_ptr, col, val

    def cast(self, dtype) -> dict:
        """Arrays of the problem in ``dtype`` (indices stay int32)."""
        return {k: getattr(self, k).astype(dtype) for k in ("val", "b", "v0", "R", "phi", "mu")}


@dataclasses.dataclass
class Batch:
    """Block-diagonal concatenation of independent environments."""
    problem: Problem          # concatenated problem with global node indices
    env_node_off: np.ndarray  # [E+1]
    env_blk_off: np.ndarray   # [E+1]
    env_con_off: np.ndarray   # [E+1]
    envs: list

    @property
    def n_env(self) -> int:
        return len(self.envs)


def concat_problems(problems: list) -> Batch:
    node_off = np.zeros(len(problems) + 1, dtype=np.int64)
    blk_off = np.zeros(len(problems) + 1, dtype=np.int64)
    con_off = np.zeros(len(problems) + 1, dtype=np.int64)
    for e, p in enumerate(problems):
        node_off[e + 1] = node_off[e] + p.n_nodes
        blk_off[e + 1] = blk_off[e] + p.nnzb
        con_off[e + 1] = con_off[e] + p.n_contacts
    assert node_off[-1] < 2**31 and blk_off[-1] < 2**31
    row_ptr = np.concatenate([p.row_ptr[:-1] + blk_off[e] for e, p in enumerate(problems)] + [blk_off[-1:]])
    col = np.concatenate([p.col_idx + node_off[e] for e, p in enumerate(problems)])
    cn = np.concatenate([p.c_node + node_off[e] for e, p in enumerate(problems)])
    cj = np.concatenate([np.where(p.c_node_j >= 0, p.c_node_j + node_off[e], -1) for e, p in enumerate(problems)])
    big = Problem(
        n_nodes=int(node_off[-1]), row_ptr=row_ptr, col_idx=col,
        val=np.concatenate([p.val for p in problems]),
        b=np.concatenate([p.b for p in problems]),
        v0=np.concatenate([p.v0 for p in problems]),
        c_node=cn, c_node_j=cj,
        R=np.concatenate([p.R for p in problems]),
        phi=np.concatenate([p.phi for p in problems]),
        mu=np.concatenate([p.mu for p in problems]),
        meta={"batched": True},
        mu2=(np.concatenate([p.mu if p.mu2 is None else p.mu2 for p in problems])
             if any(p.mu2 is not None for p in problems) else None),
    )
    return Batch(big, node_off.astype(np.int32), blk_off.astype(np.int32), con_off.astype(np.int32), problems)
