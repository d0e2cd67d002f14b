"""ctypes mirror of include/vfpi.h: structs, constants and the entry points
under the same names.  Argument marshalling only; all computation happens in
the HIP library.  Loading fails loudly if the library has not been built."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvfpi.so")

VFPI_OK = 0
VFPI_E_NULL = -1
VFPI_E_SHAPE = -2
VFPI_E_OPTS = -3
VFPI_E_CAPACITY = -4
VFPI_E_UNSUPPORTED = -5
VFPI_E_HIP = -6
VFPI_E_NO_TAPE = -7

VFPI_S_CONVERGED = 0x000
VFPI_S_MAXITER = 0x001
VFPI_S_NONFINITE = 0x010
VFPI_S_NOT_NODAL = 0x020
VFPI_S_NOT_ORTHONORMAL = 0x040
VFPI_S_SHARED_NODE = 0x080
VFPI_S_NONPOS_DIAG = 0x100
VFPI_S_BAD_PATTERN = 0x200
VFPI_S_BAD_W = 0x400
VFPI_S_BAD_MU = 0x800

VFPI_W_FROBENIUS = 0
VFPI_W_USER_DIAG = 1
VFPI_W_USER_SCALAR = 2
VFPI_W_BB1 = 3
VFPI_W_BB2 = 4

VFPI_PROJ_STRICT = 0
VFPI_PROJ_PROXIMAL = 1

ENTRY_POINTS = ("vfpi_create", "vfpi_destroy", "vfpi_tape_bytes", "vfpi_step", "vfpi_step_batched",
                "vfpi_step_backward", "vfpi_vnode_pattern", "vfpi_vnode_values", "vfpi_timing_enable",
                "vfpi_timing_read", "vfpi_error_string", "vfpi_step_noalloc")

VFPI_NOALLOC_SCRATCH_BYTES = 32 << 20


class vfpi_bsr(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("nnzb", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class vfpi_contacts(ctypes.Structure):
    _fields_ = [("n_contacts", ctypes.c_int32), ("nnzb", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p), ("phi", ctypes.c_void_p),
                ("mu", ctypes.c_void_p), ("mu2", ctypes.c_void_p)]


class vfpi_opts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("fixed_iters", ctypes.c_int32), ("tol", ctypes.c_double),
                ("w_mode", ctypes.c_int32), ("projection", ctypes.c_int32), ("w_user", ctypes.c_void_p),
                ("alpha_user", ctypes.c_double), ("reuse_w", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("cheby_ls", ctypes.c_int32), ("cheby_u", ctypes.c_double), ("omega", ctypes.c_double)]


class vfpi_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("theta", ctypes.c_double),
                ("n_open", ctypes.c_int32), ("n_stick", ctypes.c_int32), ("n_slip", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


assert ctypes.sizeof(vfpi_stats) == 32
assert ctypes.sizeof(vfpi_opts) == 72

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the built library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"V-FPI HIP library not built: {path} is missing "
                           "(run `python -m paper_2201_09212_amd.build`)")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I32 = ctypes.c_int32
    lib.vfpi_create.argtypes = [ctypes.POINTER(P), I32, I32, I32, I32]
    lib.vfpi_create.restype = ctypes.c_int
    lib.vfpi_destroy.argtypes = [P]
    lib.vfpi_destroy.restype = ctypes.c_int
    lib.vfpi_tape_bytes.argtypes = [I32, I32]
    lib.vfpi_tape_bytes.restype = ctypes.c_int64
    lib.vfpi_step.argtypes = [P, ctypes.POINTER(vfpi_bsr), P, ctypes.POINTER(vfpi_contacts), P, P,
                              ctypes.POINTER(vfpi_opts), P, P, P]
    lib.vfpi_step.restype = ctypes.c_int
    lib.vfpi_step_noalloc.argtypes = [ctypes.POINTER(vfpi_bsr), P, ctypes.POINTER(vfpi_contacts), P, P,
                                      ctypes.POINTER(vfpi_opts), P, P, P]
    lib.vfpi_step_noalloc.restype = ctypes.c_int
    lib.vfpi_step_batched.argtypes = [P, I32, P, P, P, ctypes.POINTER(vfpi_bsr), P, ctypes.POINTER(vfpi_contacts),
                                      P, P, ctypes.POINTER(vfpi_opts), P, P]
    lib.vfpi_step_batched.restype = ctypes.c_int
    lib.vfpi_step_backward.argtypes = [P, ctypes.POINTER(vfpi_bsr), ctypes.POINTER(vfpi_contacts), P, P, P, P, P,
                                       P, P, P, ctypes.POINTER(vfpi_opts), P, P]
    lib.vfpi_step_backward.restype = ctypes.c_int
    lib.vfpi_vnode_pattern.argtypes = [I32, P, P, I32, P, P, P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    lib.vfpi_vnode_pattern.restype = ctypes.c_int
    lib.vfpi_vnode_values.argtypes = [ctypes.POINTER(vfpi_bsr), P, P, I32, P, P, P, ctypes.c_double, P, P, P, P, P,
                                      P]
    lib.vfpi_vnode_values.restype = ctypes.c_int
    lib.vfpi_timing_enable.argtypes = [P, I32]
    lib.vfpi_timing_enable.restype = ctypes.c_int
    lib.vfpi_timing_read.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
    lib.vfpi_timing_read.restype = ctypes.c_int
    lib.vfpi_error_string.argtypes = [ctypes.c_int]
    lib.vfpi_error_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


class VfpiError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().vfpi_error_string(code).decode()
        super().__init__(f"{where}: {msg} ({code})")
        self.code = code


def check(rc: int, where: str):
    if rc != VFPI_OK:
        raise VfpiError(rc, where)


# ---- entry points under their C names (pointers as ints) -------------------

def vfpi_create(max_nodes: int, max_nnzb: int, max_contacts: int, max_envs: int = 0) -> int:
    h = ctypes.c_void_p()
    check(load().vfpi_create(ctypes.byref(h), max_nodes, max_nnzb, max_contacts, max_envs), "vfpi_create")
    return h.value


def vfpi_destroy(ctx: int) -> None:
    check(load().vfpi_destroy(ctx), "vfpi_destroy")


def vfpi_tape_bytes(n_nodes: int, n_contacts: int) -> int:
    return int(load().vfpi_tape_bytes(n_nodes, n_contacts))


def vfpi_error_string(code: int) -> str:
    return load().vfpi_error_string(code).decode()


def vfpi_step(ctx, A: vfpi_bsr, b, Jc: vfpi_contacts, v, lam, opts: vfpi_opts, stats, tape, stream) -> int:
    return load().vfpi_step(ctx, ctypes.byref(A), b, ctypes.byref(Jc), v, lam, ctypes.byref(opts), stats, tape,
                            stream)


def vfpi_step_noalloc(A: vfpi_bsr, b, Jc: vfpi_contacts, v, lam, opts: vfpi_opts, stats, tape, stream) -> int:
    return load().vfpi_step_noalloc(ctypes.byref(A), b, ctypes.byref(Jc), v, lam, ctypes.byref(opts), stats, tape,
                                    stream)


def vfpi_step_batched(ctx, n_env, env_node_off, env_con_off, env_order, A: vfpi_bsr, b, Jc: vfpi_contacts, v, lam,
                      opts: vfpi_opts, stats, stream) -> int:
    return load().vfpi_step_batched(ctx, n_env, env_node_off, env_con_off, env_order, ctypes.byref(A), b,
                                    ctypes.byref(Jc), v, lam, ctypes.byref(opts), stats, stream)


def vfpi_step_backward(ctx, A: vfpi_bsr, Jc: vfpi_contacts, tape, grad_v, grad_lambda, grad_b, grad_A_val,
                       grad_phi, grad_mu, grad_mu2, opts: vfpi_opts, stats, stream) -> int:
    return load().vfpi_step_backward(ctx, ctypes.byref(A), ctypes.byref(Jc), tape, grad_v, grad_lambda, grad_b,
                                     grad_A_val, grad_phi, grad_mu, grad_mu2, ctypes.byref(opts), stats, stream)


def vfpi_vnode_pattern(n_o, row_ptr, col_idx, n_v, jv_ptr, jv_col, aug_row_ptr, aug_col_idx, cap) -> int:
    """Host arrays (pointers as ints); returns the number of blocks."""
    nnz = ctypes.c_int64()
    check(load().vfpi_vnode_pattern(n_o, row_ptr, col_idx, n_v, jv_ptr, jv_col, aug_row_ptr, aug_col_idx, cap,
                                    ctypes.byref(nnz)), "vfpi_vnode_pattern")
    return nnz.value


def vfpi_vnode_values(A_o: vfpi_bsr, b_o, v_o, n_v, jv_ptr, jv_col, jv_val, k_v, aug_row_ptr, aug_col_idx, aug_val,
                      b, v, stream) -> int:
    return load().vfpi_vnode_values(ctypes.byref(A_o), b_o, v_o, n_v, jv_ptr, jv_col, jv_val, float(k_v),
                                    aug_row_ptr, aug_col_idx, aug_val, b, v, stream)


def vfpi_timing_enable(ctx, on: bool) -> None:
    check(load().vfpi_timing_enable(ctx, int(bool(on))), "vfpi_timing_enable")


def vfpi_timing_read(ctx):
    """(setup_ms, solve_ms) of the last timed call (waits for its events)."""
    a, b = ctypes.c_float(), ctypes.c_float()
    check(load().vfpi_timing_read(ctx, ctypes.byref(a), ctypes.byref(b)), "vfpi_timing_read")
    return a.value, b.value
