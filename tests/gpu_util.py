"""Helpers for the GPU tests: move a seeded problem to the device, run the
HIP path through the C ABI, compare with the oracle element by element."""
import sys

import numpy as np
import torch

import paper_2201_09212_amd as vf


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(x, y):
    """||x - y|| / ||y||; when y = 0 the absolute max of x (reported next to
    the element-wise gate, never the gate by itself)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    ny = np.linalg.norm(y)
    if ny == 0.0:
        return float(np.abs(x).max()) if x.size else 0.0
    return float(np.linalg.norm(x - y) / ny)


def gate(x, y, tol, what=""):
    """Element-wise parity gate at relative bar ``tol``: every entry must
    satisfy |x_i - y_i| <= tol |y_i| + tol max_j |y_j| (so a single wrong
    entry fails however long the vector), and the norm-wise rel(x, y) <= tol
    as well.  An all-zero reference requires exact zeros.  Returns rel(x, y)
    for the log line."""
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    assert x.shape == y.shape, (what, x.shape, y.shape)
    if x.size == 0:
        return 0.0
    assert np.all(np.isfinite(x)), (what, "non-finite entries")
    scale = float(np.abs(y).max())
    np.testing.assert_allclose(x, y, rtol=tol, atol=tol * scale, err_msg=f"{what} (element-wise, bar {tol:g})")
    r = rel(x, y)
    assert r <= tol, (what, r, tol)
    return r


def tape_parts(tape, n_nodes, n_contacts):
    """The forward tape's fields (byte layout of the C ABI's tape: w[3N] f64,
    v[3N] f64, lambda*[3 n_c] f64, branch[n_c] i32), as host arrays."""
    raw = tape.cpu().numpy().tobytes()
    n = 3 * n_nodes
    w = np.frombuffer(raw, np.float64, n, 0)
    v = np.frombuffer(raw, np.float64, n, 8 * n)
    ls = np.frombuffer(raw, np.float64, 3 * n_contacts, 16 * n).reshape(-1, 3)
    br = np.frombuffer(raw, np.int32, n_contacts, 16 * n + 24 * n_contacts)
    return {"w": w, "v": v, "lam_star": ls, "branch": br}


def branch_margin(lam_star, mu, mu2=None, projection="strict"):
    """How far each contact's lambda* is from the nearest branch boundary of
    the projection, relative to |lambda*|: the normal clamp (lambda*_n = 0)
    and the cone / disk / ellipse boundary.  A branch may differ between two
    FP64 evaluations only where this is at the rounding level."""
    ls = np.asarray(lam_star, dtype=np.float64).reshape(-1, 3)
    n, t1, t2 = ls[:, 0], ls[:, 1], ls[:, 2]
    s = np.hypot(t1, t2)
    scale = np.maximum(np.abs(ls).max(axis=1), 1e-300)
    mu = np.asarray(mu, dtype=np.float64)
    if projection == "proximal":
        m1 = np.abs(s - mu * n)
        m2 = np.abs(mu * s + n)
        return np.minimum(m1, m2) / scale
    m_n = np.abs(n)
    ln = np.maximum(n, 0.0)
    if mu2 is None:
        m_t = np.abs(s - mu * ln)
    else:
        a, b = mu * ln, np.asarray(mu2, dtype=np.float64) * ln
        # distance-like measure of the ellipse test (t1/a)^2 + (t2/b)^2 = 1
        with np.errstate(divide="ignore", invalid="ignore"):
            f = np.sqrt((t1 / np.where(a > 0, a, 1.0)) ** 2 * (a > 0) + (t2 / np.where(b > 0, b, 1.0)) ** 2 * (b > 0))
        m_t = np.abs(f - 1.0) * np.minimum(np.where(a > 0, a, np.inf), np.where(b > 0, b, np.inf))
        m_t = np.where(np.isfinite(m_t), m_t, s)
    return np.minimum(m_n, m_t) / scale


def check_branches(br_gpu, ref, mu, mu2=None, projection="strict", what="", tie=1e-10):
    """Per-contact branch (open / stick / slip) equality with the oracle.  A
    mismatch is accepted only at a tie: where the oracle's lambda* lies within
    ``tie`` (relative) of that branch boundary, so that the two sides' last
    rounding decides it.  Returns the number of such ties."""
    br_gpu = np.asarray(br_gpu).ravel()
    br_ref = np.asarray(ref["branch"]).ravel()
    assert br_gpu.shape == br_ref.shape, (what, br_gpu.shape, br_ref.shape)
    bad = np.nonzero(br_gpu != br_ref)[0]
    if bad.size == 0:
        return 0
    margin = branch_margin(ref["lam_star"], mu, mu2, projection)[bad]
    assert np.all(margin <= tie), (what, "branch differs away from a tie", bad[margin > tie][:10].tolist(),
                                   br_gpu[bad][:10].tolist(), br_ref[bad][:10].tolist())
    return int(bad.size)


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


def fixed_parity(p, ref, L, tol=1e-9, what="", projection="strict", **opt):
    """vfpi_step at a fixed sweep count L against an oracle result ``ref`` of
    the same sweeps: v, lambda and the taped lambda* element by element,
    each contact's branch, the branch counts, and the residual theta of the
    last sweep (Alg. 1's reduction: relative bar tol, plus 1e-12 of |v| for
    the rounding of the last sweep's difference).  Returns (rel_v, rel_lam,
    stats, ties)."""
    v, lam, st, tp = gpu_step(p, tape=True, max_iters=L, fixed_iters=True, projection=projection, **opt)
    assert st["iters"] == L and st["status"] == 1, (what, st)
    vnorm = float(np.linalg.norm(ref["v"]))
    assert abs(st["theta"] - ref["theta"]) <= tol * ref["theta"] + 1e-12 * vnorm, (what, st["theta"], ref["theta"])
    ev = gate(v, ref["v"], tol, f"{what} v")
    el = gate(lam, ref["lam"], tol, f"{what} lambda")
    ties = 0
    if p.n_contacts:
        t = tape_parts(tp, p.n_nodes, p.n_contacts)
        gate(t["lam_star"], ref["lam_star"], tol, f"{what} lambda*")
        ties = check_branches(t["branch"], ref, p.mu, getattr(p, "mu2", None), projection, what)
    counts = np.bincount(ref["branch"], minlength=3) if p.n_contacts else np.zeros(3, int)
    if ties == 0:
        assert [st["n_open"], st["n_stick"], st["n_slip"]] == counts.tolist(), what
    return ev, el, st, ties
