"""Helpers for the GPU tests: move a seeded problem to the device, run the
HIP path through the C ABI, compare with the oracle."""
import sys

import numpy as np
import torch

import paper_2201_09212_amd as vf


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(x, y):
    """||x - y|| / ||y||; when y = 0 the absolute max of x."""
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    ny = np.linalg.norm(y)
    if ny == 0.0:
        return float(np.abs(x).max()) if x.size else 0.0
    return float(np.linalg.norm(x - y) / ny)


def upload(p, dtype=torch.float64):
    dev = torch.device("cuda", 0)
    A = vf.bsr_from_arrays(p.n_nodes, p.row_ptr, p.col_idx, p.val, dtype=dtype, device=dev)
    crp, ccol, cval = p.jc_bsr()
    Jc = vf.contacts_from_arrays(crp, ccol, cval, p.phi, p.mu, dtype=dtype, device=dev, mu2=p.mu2)
    b = torch.as_tensor(p.b, device=dev).to(dtype)
    v = torch.as_tensor(p.v0, device=dev).to(dtype)
    return A, Jc, b, v


def solver_for(p, max_envs=0):
    return vf.Solver(max(p.n_nodes, 1), max(p.nnzb, 1), max(p.n_contacts, 1), max_envs)


def gpu_step(p, solver=None, tape=False, **opt):
    """Runs vfpi_step on p; returns (v, lambda, stats dict, tape tensor)."""
    s = solver or solver_for(p)
    A, Jc, b, v = upload(p)
    tp = s.tape(p.n_nodes, p.n_contacts) if tape else None
    lam, st = s.step(A, b, Jc, v, tape=tp, **opt)
    torch.cuda.synchronize()
    return v.cpu().numpy(), lam.cpu().numpy().reshape(-1, 3), vf.read_stats(st)[0], tp
