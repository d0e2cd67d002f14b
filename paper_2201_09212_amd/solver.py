"""Torch-facing wrappers around the C ABI: device buffers in, device buffers
out.  PyTorch provides memory and streams only; every step of the solve runs
in the HIP library."""
from __future__ import annotations

import atexit
import ctypes
import dataclasses
import sys
import weakref

import numpy as np
import torch

from . import _abi

W_MODES = {"frobenius": _abi.VFPI_W_FROBENIUS, "diag": _abi.VFPI_W_USER_DIAG,
           "scalar": _abi.VFPI_W_USER_SCALAR, "bb1": _abi.VFPI_W_BB1, "bb2": _abi.VFPI_W_BB2}
PROJECTIONS = {"strict": _abi.VFPI_PROJ_STRICT, "proximal": _abi.VFPI_PROJ_PROXIMAL}
STATS_BYTES = ctypes.sizeof(_abi.vfpi_stats)


def _dev(device):
    return torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check(t, dtype, n, name):
    if t.dtype != dtype or not t.is_contiguous() or t.device.type != "cuda" or t.numel() != n:
        raise ValueError(f"{name}: need contiguous {dtype} cuda tensor with {n} elements, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


@dataclasses.dataclass
class Bsr:
    """Block-sparse rows with 3x3 blocks on the device."""
    n_nodes: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor

    @property
    def nnzb(self):
        return int(self.col_idx.numel())

    def desc(self):
        _check(self.row_ptr, torch.int32, self.n_nodes + 1, "row_ptr")
        _check(self.col_idx, torch.int32, self.nnzb, "col_idx")
        if self.val.numel() != 9 * self.nnzb or not self.val.is_contiguous():
            raise ValueError("val must hold 9 * nnzb contiguous values")
        return _abi.vfpi_bsr(self.n_nodes, self.nnzb, _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.val))


@dataclasses.dataclass
class Contacts:
    """Nodal contact Jacobian rows ([R] for an S-contact, [R, -R] for a D-contact), phi,
    mu and, for anisotropic friction, mu2."""
    n_contacts: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor
    phi: torch.Tensor
    mu: torch.Tensor
    mu2: torch.Tensor | None = None  # anisotropic friction (tangent 2); None: isotropic

    def desc(self):
        _check(self.row_ptr, torch.int32, self.n_contacts + 1, "Jc.row_ptr")
        nnzb = int(self.col_idx.numel())
        if self.mu2 is not None and (self.mu2.numel() != self.n_contacts or self.mu2.dtype != self.mu.dtype):
            raise ValueError("mu2 must match mu")
        return _abi.vfpi_contacts(self.n_contacts, nnzb, _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.val),
                                  _ptr(self.phi), _ptr(self.mu), _ptr(self.mu2))


def bsr_from_arrays(n_nodes, row_ptr, col_idx, val, dtype=torch.float64, device=None) -> Bsr:
    d = _dev(device)
    return Bsr(n_nodes, torch.as_tensor(np.ascontiguousarray(row_ptr, np.int32), device=d),
               torch.as_tensor(np.ascontiguousarray(col_idx, np.int32), device=d),
               torch.as_tensor(np.ascontiguousarray(val).reshape(-1), device=d).to(dtype).contiguous())


def contacts_from_arrays(row_ptr, col_idx, val, phi, mu, dtype=torch.float64, device=None, mu2=None) -> Contacts:
    d = _dev(device)
    nc = len(row_ptr) - 1
    return Contacts(nc, torch.as_tensor(np.ascontiguousarray(row_ptr, np.int32), device=d),
                    torch.as_tensor(np.ascontiguousarray(col_idx, np.int32), device=d),
                    torch.as_tensor(np.ascontiguousarray(val).reshape(-1), device=d).to(dtype).contiguous(),
                    torch.as_tensor(np.ascontiguousarray(phi), device=d).to(dtype).contiguous(),
                    torch.as_tensor(np.ascontiguousarray(mu), device=d).to(dtype).contiguous(),
                    None if mu2 is None else
                    torch.as_tensor(np.ascontiguousarray(mu2), device=d).to(dtype).contiguous())


def make_opts(max_iters=100, tol=0.0, fixed_iters=False, w_mode="frobenius", w_user=None, alpha=0.0,
              projection="strict", reuse_w=False, variant=0, cheby_ls=0, cheby_u=1.0, omega=0.0) -> _abi.vfpi_opts:
    return _abi.vfpi_opts(int(max_iters), int(bool(fixed_iters)), float(tol), W_MODES[w_mode],
                          PROJECTIONS[projection], _ptr(w_user), float(alpha or 0.0), int(bool(reuse_w)),
                          int(variant), int(cheby_ls), float(cheby_u), float(omega))


def new_stats(n=1, device=None):
    return torch.zeros(n * STATS_BYTES, dtype=torch.uint8, device=_dev(device))


def read_stats(stats: torch.Tensor):
    raw = stats.cpu().numpy().tobytes()
    out = []
    for k in range(len(raw) // STATS_BYTES):
        s = _abi.vfpi_stats.from_buffer_copy(raw[k * STATS_BYTES:(k + 1) * STATS_BYTES])
        out.append({"iters": s.iters, "status": s.status, "theta": s.theta, "n_open": s.n_open,
                    "n_stick": s.n_stick, "n_slip": s.n_slip})
    return out


def stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    """Release every context still open when the program ends, while the HIP
    runtime, torch and any profiler attached to the process are still alive
    (atexit handlers run before the interpreter tears modules down)."""
    for s in list(_LIVE):
        s.close()


class Solver:
    """Owns one library context (device workspace for problems up to the
    given sizes).  Release it with ``close()`` (or a ``with`` block); a
    context still open at exit is released by an atexit handler.  The
    finalizer frees it too, except during interpreter shutdown, when no HIP
    call is made (the process's memory goes with it)."""

    def __init__(self, max_nodes, max_nnzb, max_contacts, max_envs=0, device=None):
        self.ctx = None
        self.device = _dev(device)
        with torch.cuda.device(self.device):
            self.ctx = _abi.vfpi_create(int(max_nodes), int(max_nnzb), int(max_contacts), int(max_envs))
        self.capacity = (max_nodes, max_nnzb, max_contacts, max_envs)
        _LIVE.add(self)

    def close(self):
        if self.ctx:
            ctx, self.ctx = self.ctx, None
            _LIVE.discard(self)
            _abi.vfpi_destroy(ctx)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        if sys.is_finalizing() or not getattr(self, "ctx", None):
            return
        try:
            self.close()
        except Exception:
            pass

    def tape(self, n_nodes, n_contacts):
        return torch.empty(_abi.vfpi_tape_bytes(n_nodes, n_contacts), dtype=torch.uint8, device=self.device)

    def step(self, A: Bsr, b, Jc: Contacts, v, lam=None, *, stats=None, tape=None, stream=None, **opt):
        """FP64 solve; ``v`` (warm start) is overwritten with the solution.
        Returns (lambda, stats tensor)."""
        n = 3 * A.n_nodes
        _check(b, torch.float64, n, "b")
        _check(v, torch.float64, n, "v")
        if lam is None:
            lam = torch.empty(3 * Jc.n_contacts, dtype=torch.float64, device=self.device)
        stats = new_stats(1, self.device) if stats is None else stats
        o = make_opts(**opt)
        rc = _abi.vfpi_step(self.ctx, A.desc(), _ptr(b), Jc.desc(), _ptr(v), _ptr(lam), o, _ptr(stats),
                            _ptr(tape), stream_handle(stream))
        _abi.check(rc, "vfpi_step")
        return lam, stats

    def step_batched(self, n_env, env_node_off, env_con_off, A: Bsr, b, Jc: Contacts, v, lam=None, *,
                     env_order=None, stats=None, stream=None, **opt):
        n = 3 * A.n_nodes
        _check(b, torch.float32, n, "b")
        _check(v, torch.float32, n, "v")
        _check(env_node_off, torch.int32, n_env + 1, "env_node_off")
        _check(env_con_off, torch.int32, n_env + 1, "env_con_off")
        if lam is None:
            lam = torch.empty(3 * Jc.n_contacts, dtype=torch.float32, device=self.device)
        stats = new_stats(n_env, self.device) if stats is None else stats
        o = make_opts(**opt)
        rc = _abi.vfpi_step_batched(self.ctx, int(n_env), _ptr(env_node_off), _ptr(env_con_off), _ptr(env_order),
                                    A.desc(), _ptr(b), Jc.desc(), _ptr(v), _ptr(lam), o, _ptr(stats),
                                    stream_handle(stream))
        _abi.check(rc, "vfpi_step_batched")
        return lam, stats

    def step_backward(self, A: Bsr, Jc: Contacts, tape, grad_v, grad_lambda=None, *, want_A=False, stats=None,
                      stream=None, **opt):
        n = 3 * A.n_nodes
        _check(grad_v, torch.float64, n, "grad_v")
        dev = self.device
        gb = torch.empty(n, dtype=torch.float64, device=dev)
        gA = torch.empty(9 * A.nnzb, dtype=torch.float64, device=dev) if want_A else None
        gphi = torch.empty(Jc.n_contacts, dtype=torch.float64, device=dev)
        gmu = torch.empty(Jc.n_contacts, dtype=torch.float64, device=dev)
        gmu2 = torch.empty(Jc.n_contacts, dtype=torch.float64, device=dev) if Jc.mu2 is not None else None
        stats = new_stats(1, dev) if stats is None else stats
        o = make_opts(**opt)
        rc = _abi.vfpi_step_backward(self.ctx, A.desc(), Jc.desc(), _ptr(tape), _ptr(grad_v), _ptr(grad_lambda),
                                     _ptr(gb), _ptr(gA), _ptr(gphi), _ptr(gmu), _ptr(gmu2), o, _ptr(stats),
                                     stream_handle(stream))
        _abi.check(rc, "vfpi_step_backward")
        out = {"b": gb, "A": gA, "phi": gphi, "mu": gmu, "stats": stats}
        if gmu2 is not None:
            out["mu2"] = gmu2
        return out


def vnode_augment(A_o: Bsr, b_o, v_o, jv_ptr, jv_col, jv_val, k_v, stream=None):
    """System of eq. vnode for virtual nodes tied to the points J_v v_o with
    gain k_v: returns (A, b, v) over n_o + n_v nodes (virtual node q is node
    n_o + q).  The block pattern comes from ``vfpi_vnode_pattern`` on host
    copies of the index arrays, the values from ``vfpi_vnode_values`` on the
    device."""
    dev = b_o.device
    n_o = A_o.n_nodes
    n_v = int(jv_ptr.numel()) - 1
    rp_h = A_o.row_ptr.detach().to("cpu", torch.int32).contiguous()
    ci_h = A_o.col_idx.detach().to("cpu", torch.int32).contiguous()
    jp_h = jv_ptr.detach().to("cpu", torch.int32).contiguous()
    jc_h = jv_col.detach().to("cpu", torch.int32).contiguous()
    g_ptr = torch.empty(n_o + n_v + 1, dtype=torch.int32)
    nnz = _abi.vfpi_vnode_pattern(n_o, rp_h.data_ptr(), ci_h.data_ptr(), n_v, jp_h.data_ptr(), jc_h.data_ptr(),
                                  g_ptr.data_ptr(), None, 0)
    g_col = torch.empty(max(nnz, 1), dtype=torch.int32)
    _abi.vfpi_vnode_pattern(n_o, rp_h.data_ptr(), ci_h.data_ptr(), n_v, jp_h.data_ptr(), jc_h.data_ptr(),
                            g_ptr.data_ptr(), g_col.data_ptr(), nnz)
    rp = g_ptr.to(dev)
    ci = g_col[:nnz].to(dev)
    val = torch.empty(9 * max(nnz, 1), dtype=torch.float64, device=dev)
    n = 3 * (n_o + n_v)
    b = torch.empty(n, dtype=torch.float64, device=dev)
    v = torch.empty(n, dtype=torch.float64, device=dev)
    jvp = jv_ptr.to(dev, torch.int32).contiguous()
    jvc = jv_col.to(dev, torch.int32).contiguous()
    jvv = jv_val.to(dev, torch.float64).contiguous()
    _check(b_o, torch.float64, 3 * n_o, "b_o")
    _check(v_o, torch.float64, 3 * n_o, "v_o")
    with torch.cuda.device(dev):
        rc = _abi.vfpi_vnode_values(A_o.desc(), _ptr(b_o), _ptr(v_o), n_v, _ptr(jvp), _ptr(jvc), _ptr(jvv), k_v,
                                    _ptr(rp), _ptr(ci), _ptr(val), _ptr(b), _ptr(v), stream_handle(stream))
    _abi.check(rc, "vfpi_vnode_values")
    return Bsr(n_o + n_v, rp, ci, val[:9 * nnz]), b, v
