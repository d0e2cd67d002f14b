"""Differentiable (PyTorch) form of the mass-spring cloth step assembly, for
rollouts whose gradient flows through the scene parameters (spring stiffness
k, per-node friction mu) and the initial state.

Same physics as ``scenes.cloth.ClothScene.assemble`` (backward-Euler,
outer-product spring Hessian, plane z = 0 with speculative contacts inside
delta, phi = gap / h); the contact set is chosen from the current positions
and is not differentiated (it is piecewise constant).
"""
from __future__ import annotations

import numpy as np
import torch

from .cloth import GRAVITY, ClothScene, _slot
from .geometry import onb_duff


class TorchCloth:
    def __init__(self, scene: ClothScene, device, dtype=torch.float64):
        self.sc = scene
        self.device = torch.device(device)
        self.dtype = dtype
        ex = scene.exists
        # block index of (row i, stencil slot s) in the block-row layout
        before = np.cumsum(ex, axis=1) - ex
        blk = scene.row_ptr[:-1, None].astype(np.int64) + before
        d = torch.device(device)
        self.row_ptr = torch.as_tensor(scene.row_ptr, device=d)
        self.col_idx = torch.as_tensor(scene.col_idx, device=d)
        self.nnzb = int(scene.row_ptr[-1])
        self.diag_blk = torch.as_tensor(blk[:, 4], device=d)
        self.springs = []
        for dr, dc, p, q in scene.springs:
            self.springs.append((
                torch.as_tensor(p, device=d), torch.as_tensor(q, device=d),
                torch.as_tensor(blk[p, 4], device=d), torch.as_tensor(blk[q, 4], device=d),
                torch.as_tensor(blk[p, _slot(dr, dc)], device=d), torch.as_tensor(blk[q, _slot(-dr, -dc)], device=d),
                scene.spacing * float(np.hypot(dr, dc))))
        self.gravity = torch.as_tensor(GRAVITY, device=d, dtype=dtype)
        nrm = np.array([[0.0, 0.0, 1.0]])
        self.R_plane = torch.as_tensor(onb_duff(nrm)[0], device=d, dtype=dtype)

    @property
    def n_nodes(self):
        return self.sc.n_nodes

    @property
    def h(self):
        return self.sc.h

    def assemble(self, x, v, k, mu_node):
        """x, v: [N,3]; k: scalar tensor; mu_node: [N].  Returns A values
        [nnzb,3,3], b [3N], contact nodes (int32), R [nc,3,3], phi [nc], mu [nc]."""
        sc = self.sc
        h = sc.h
        val = torch.zeros(self.nnzb, 3, 3, device=self.device, dtype=self.dtype)
        f = torch.zeros_like(x)
        for p, q, bpp, bqq, bpq, bqp, rest in self.springs:
            dx = x[p] - x[q]
            ln = torch.linalg.norm(dx, dim=1)
            dd = dx / ln[:, None]
            kb = k * dd[:, :, None] * dd[:, None, :]
            val = val.index_add(0, bpp, kb).index_add(0, bqq, kb).index_add(0, bpq, -kb).index_add(0, bqp, -kb)
            fs = -k * (ln - rest)[:, None] * dd
            f = f.index_add(0, p, fs).index_add(0, q, -fs)
        eye = torch.eye(3, device=self.device, dtype=self.dtype)
        A = (h * h) * val
        A = A.index_add(0, self.diag_blk, (sc.mass * eye).expand(self.n_nodes, 3, 3))
        f = f + sc.mass * self.gravity
        b = (sc.mass * v + h * f).reshape(-1)
        gap = x[:, 2]
        nodes = torch.nonzero(gap.detach() <= sc.delta).squeeze(1)
        phi = gap[nodes] / h
        mu = mu_node[nodes]
        R = self.R_plane.expand(nodes.shape[0], 3, 3).contiguous()
        return A, b, nodes.to(torch.int32), R, phi, mu
