"""Virtual nodes (Sec. III-A): the augmented system of eq. vnode, test
infrastructure only.

With the viscous tie f_v = -k_v (J_v v_o - v_v) of eq. vforce between each
virtual node and the point it sits on, the velocities [v_o; v_v] solve

    [ A_o + k_v J_v^T J_v   -k_v J_v^T ] [v_o]   [b_o]
    [ -k_v J_v               k_v I     ] [v_v] = [ 0 ] + J_c^T lambda,

the same structure as eq. lindyn, so V-FPI runs on it unchanged (Prop. 1: it
is SPD).  The virtual nodes' warm start is the velocity of their points,
J_v v_o (a reading: the paper does not state it).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .core import system_matrix  # noqa: F401  (same BSR convention)


def jv_matrix(vs) -> sp.csr_matrix:
    """J_v (3 n_v x 3 n_o) from its block rows."""
    return sp.bsr_matrix((vs.jv_val, vs.jv_col, vs.jv_ptr), shape=(3 * vs.n_v, 3 * vs.n_o)).tocsr()


def augmented_matrix(vs, k_v) -> sp.csr_matrix:
    Ao = sp.bsr_matrix((vs.val, vs.col_idx, vs.row_ptr), shape=(3 * vs.n_o, 3 * vs.n_o)).tocsr()
    Jv = jv_matrix(vs)
    return sp.bmat([[Ao + k_v * (Jv.T @ Jv), -k_v * Jv.T],
                    [-k_v * Jv, k_v * sp.identity(3 * vs.n_v)]], format="csr")


def augment(vs, k_v):
    """The eq. vnode problem as a Problem over n_o + n_v nodes (3x3 blocks of
    the augmented matrix, columns sorted within each block row)."""
    from scenes import Problem  # container only

    A = augmented_matrix(vs, k_v)
    B = A.tobsr(blocksize=(3, 3))
    B.sort_indices()
    n = vs.n_o + vs.n_v
    b = np.concatenate([vs.b, np.zeros(3 * vs.n_v)])
    v0 = np.concatenate([vs.v0, jv_matrix(vs) @ vs.v0])
    return Problem(n_nodes=n, row_ptr=B.indptr, col_idx=B.indices, val=B.data, b=b, v0=v0, c_node=vs.c_node,
                   c_node_j=vs.c_node_j, R=vs.R, phi=vs.phi, mu=vs.mu, meta={"k_v": k_v, **vs.meta})
