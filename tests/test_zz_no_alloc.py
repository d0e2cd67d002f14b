"""vfpi_step_noalloc (the plain FP64 solve with its workspace in the
library's fixed device array) against vfpi_step with a context, through the
C ABI: two calls in a row, the second on a smaller problem, each compared
element by element (and bit for bit: the kernels are the same) with the
context entry point's v, lambda, tape and stats."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2201_09212_amd as vf
import scenes
from paper_2201_09212_amd import _abi
from tests.gpu_util import gate, say, solver_for, tape_parts, upload

pytestmark = pytest.mark.gpu
TOL = 1e-9


def _problem(which):
    if which == "cloth128":
        sc, x, v = scenes.cloth_cfg2(0)
    else:
        sc, x, v = scenes.cloth_cfg1(0)
    return sc.assemble(x, v)


def _run(p, noalloc, **opt):
    A, Jc, b, v = upload(p)
    lam = torch.full((3 * p.n_contacts,), np.nan, dtype=torch.float64, device="cuda")
    stats = vf.new_stats(1, "cuda")
    tape = torch.zeros(vf.vfpi_tape_bytes(p.n_nodes, p.n_contacts), dtype=torch.uint8, device="cuda")
    o = vf.make_opts(**opt)
    stream = torch.cuda.current_stream().cuda_stream
    if noalloc:
        rc = _abi.vfpi_step_noalloc(A.desc(), b.data_ptr(), Jc.desc(), v.data_ptr(), lam.data_ptr(), o,
                                    stats.data_ptr(), tape.data_ptr(), stream)
        _abi.check(rc, "vfpi_step_noalloc")
    else:
        s = solver_for(p)
        try:
            s.step(A, b, Jc, v, lam, stats=stats, tape=tape, **opt)
            torch.cuda.synchronize()
        finally:
            s.close()
    torch.cuda.synchronize()
    return (v.cpu().numpy(), lam.cpu().numpy(), vf.read_stats(stats)[0],
            tape_parts(tape, p.n_nodes, p.n_contacts))


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_context_entry_point(order):
    cases = [("cloth128", dict(max_iters=100, fixed_iters=True)),
             ("cloth10", dict(max_iters=500, tol=1e-6, cheby_ls=10))]
    for name, opt in cases:
        p = _problem(name)
        say(f"  noalloc: {name} N={p.n_nodes} nnzb={p.nnzb} nc={p.n_contacts} opts={opt}")
        v1, l1, s1, t1 = _run(p, True, **opt)
        v0, l0, s0, t0 = _run(p, False, **opt)
        assert s1 == s0, (name, s1, s0)
        gate(v1, v0, TOL, f"{name} v")
        gate(l1, l0, TOL, f"{name} lambda")
        gate(t1["lam_star"], t0["lam_star"], TOL, f"{name} lambda*")
        assert np.array_equal(t1["branch"], t0["branch"]), name
        # same kernels on the same inputs: the same bits
        assert np.array_equal(v1.view(np.int64), v0.view(np.int64)), name
        assert np.array_equal(l1.view(np.int64), l0.view(np.int64)), name
        assert np.array_equal(t1["w"].view(np.int64), t0["w"].view(np.int64)), name
        say(f"    iters={s1['iters']} theta={s1['theta']:.3e} status={s1['status']} bitwise equal")


def test_noalloc_rejects_what_does_not_fit():
    lib = vf.load()
    o = vf.make_opts()
    big = _abi.vfpi_bsr(1 << 20, 9 << 20, None, None, None)
    Jc = _abi.vfpi_contacts(0, 0, None, None, None, None, None)
    dummy = ctypes.c_void_p(1)
    assert lib.vfpi_step_noalloc(ctypes.byref(big), dummy, ctypes.byref(Jc), dummy, None, ctypes.byref(o), dummy,
                                 None, None) == _abi.VFPI_E_CAPACITY
    o.reuse_w = 1
    small = _abi.vfpi_bsr(4, 4, None, None, None)
    assert lib.vfpi_step_noalloc(ctypes.byref(small), dummy, ctypes.byref(Jc), dummy, None, ctypes.byref(o), dummy,
                                 None, None) == _abi.VFPI_E_OPTS
