#!/usr/bin/env python3
"""Benchmark of the V-FPI contact solve on one MI355X.

One step = one vfpi_step call (setup + the whole V-FPI loop, every row of the
hot path) on the 128x128 cloth draped over 16 spheres (49,152 DOF, ~5.2k
contacts, FP64), with a fixed number of sweeps per step and the inputs already
resident in HBM.  Prints one JSON line:

  value        contact-iterations per second (sum of n_c * sweeps / solver time)
  roofline     the persistent sweep kernel: algorithmic bytes per launch over
               its average duration (HIP events on the launch stream)
  cpu_baseline the CPU FP64 oracle on the same input, bounded sample, one
               core (cpu_baseline_multicore: one oracle process per core)
  fem, cloth10 the FEM soft block and the 10x10 cloth, fixed sweeps
  context      sweeps and time to theta < tol (plain and Chebyshev) on the
               128x128 cloth and the paper-size FEM block
  extensions   per-sweep cost of the proximal operator, the invertible
               contact, anisotropic friction, Chebyshev, BB1, node-node
               contacts and virtual nodes
  batched      batched FP32 environments (env-steps/s), when enabled
  adjoint      backward/forward time ratio, when enabled
  cpu_context  oracle V-FPI vs PGS (Delassus), the oracle adjoint step, and
               the batched FP32 result's error on a sample of environments

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sweeps L]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "contact-iters/sec + HBM GB/s (% peak); batched env-steps/s; bwd/fwd time"
HBM_PEAK_GBPS = 8000.0


def sweep_bytes(n_nodes, nnzb, n_contacts, w):
    """Algorithmic bytes of one sweep: A read once (values + column index),
    row offsets, v / b / W read and v written once per DOF, the node->contact
    map, and per contact its packed record (R, phi, mu, gamma) read and lambda
    written."""
    return (nnzb * (9 * w + 4) + 4 * (n_nodes + 1) + 3 * n_nodes * 4 * w + 4 * n_nodes
            + n_contacts * (12 * w + 3 * w))


def kernel_name(variant):
    """The persistent sweep kernel a vfpi_step variant runs."""
    kind = variant & 0xff
    return {1: "k_vfpi_grid<1,NW> (lane per node, grid)", 2: "k_vfpi_grid<3,NW> (lane per row, grid)",
            3: "k_vfpi_grid<1,NW> (one workgroup)", 4: "k_vfpi_grid<3,5> (one workgroup)",
            5: "k_vfpi_regs (A's first levels in registers, grid)"}.get(kind, f"kind {kind}")


def kernel_sources_hash():
    """Hash of the HIP sources of the forward and batched kernels with
    comments and whitespace removed, so that the stored byte counters stay
    valid across documentation edits but not across code changes.  The
    backward (adjoint.hip) and the virtual-node builder (vnode.hip) are
    included after those kernels in the one translation unit and define
    nothing they use, so they are left out."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2201_09212_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f in ("adjoint.hip", "vnode.hip"):
            continue
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(f.encode() + " ".join(src.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(name, per_launch_units):
    """HBM traffic per launch from a committed rocprofv3 --pmc summary, or None
    when the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("sources_hash") != kernel_sources_hash():
        return None
    return t.get("bytes_per_launch")


def dist(xs):
    """Mean, median and 90th percentile of a list of timings."""
    s = sorted(xs)
    return {"mean": sum(s) / len(s), "median": s[len(s) // 2], "p90": s[min(len(s) - 1, int(0.9 * len(s)))]}


def copy_peak(torch, nbytes=1 << 30, reps=5):
    """Measured device-to-device copy rate (read + write bytes per second),
    the practical HBM ceiling next to the 8 TB/s specification."""
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del x, y
    return 2 * nbytes / (dist(ms)["median"] * 1e-3) / 1e9


def upload(torch, vf, p):
    """Device copies of one problem: A, b, J_c, v (warm start), lambda, stats."""
    dev = torch.device("cuda", 0)
    A = vf.bsr_from_arrays(p.n_nodes, p.row_ptr, p.col_idx, p.val, device=dev)
    crp, ccol, cval = p.jc_bsr()
    Jc = vf.contacts_from_arrays(crp, ccol, cval, p.phi, p.mu, device=dev)
    b = torch.as_tensor(p.b, device=dev)
    vv = torch.as_tensor(p.v0, device=dev).clone()
    lam = torch.empty(3 * p.n_contacts, dtype=torch.float64, device=dev)
    return A, b, Jc, vv, lam, vf.new_stats(1, dev)


def converge_runs(torch, vf, p, tols=(1e-4, 1e-6), cheby=(0, 10), reps=3, fixed=()):
    """Iterations and solver time to reach theta < tol from the step's warm
    start, plain and with Chebyshev acceleration (l_s = 10, u = 1), with the
    library's default launch; optionally also fixed sweep counts."""
    A, b, Jc, vv, lam, stats = upload(torch, vf, p)
    v0 = vv.clone()
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)
    runs = [dict(tol=t, cheby_ls=c) for c in cheby for t in tols] + [dict(fixed=L) for L in fixed]
    out = []
    vf.vfpi_timing_enable(s.ctx, True)
    for r in runs:
        if "fixed" in r:
            opt = dict(max_iters=r["fixed"], fixed_iters=True)
        else:
            opt = dict(max_iters=100000, tol=r["tol"], cheby_ls=r["cheby_ls"])
        ms, sms = [], []
        for _ in range(reps + 1):
            vv.copy_(v0)
            s.step(A, b, Jc, vv, lam, stats=stats, **opt)
            a_, c_ = vf.vfpi_timing_read(s.ctx)
            sms.append(a_)
            ms.append(c_)
        st = vf.read_stats(stats)[0]
        out.append({**r, "iters": st["iters"], "status": st["status"], "theta": st["theta"],
                    "setup_ms": dist(sms[1:])["median"], "solve_ms": dist(ms[1:])["median"]})
    vf.vfpi_timing_enable(s.ctx, False)
    s.close()
    return out


def plain_bench(args, torch, vf, scenes, p=None, variant=None, traffic_name="cloth128"):
    if p is None:
        sc, x, v = scenes.cloth_cfg2(args.seed)
        p = sc.assemble(x, v)
    A, b, Jc, vv, lam, stats = upload(torch, vf, p)
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)
    L = args.sweeps
    variant = args.variant if variant is None else variant
    if variant == 0:
        from paper_2201_09212_amd import autotune
        variant = autotune.best_step_variant(s, A, b, Jc, vv, lam, stats)
    opt = dict(max_iters=L, fixed_iters=True, variant=variant)
    for _ in range(args.warmup):
        s.step(A, b, Jc, vv, lam, stats=stats, **opt)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        s.step(A, b, Jc, vv, lam, stats=stats, **opt)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    st = vf.read_stats(stats)[0]
    assert st["iters"] == L, st
    # per-kernel durations: events recorded by the library around setup / solve
    vf.vfpi_timing_enable(s.ctx, True)
    setup_ms, solve_ms = [], []
    for _ in range(args.steps):
        s.step(A, b, Jc, vv, lam, stats=stats, **opt)
        a, c = vf.vfpi_timing_read(s.ctx)
        setup_ms.append(a)
        solve_ms.append(c)
    vf.vfpi_timing_enable(s.ctx, False)
    s.close()
    solve_avg = sum(solve_ms) / len(solve_ms)
    setup_avg = sum(setup_ms) / len(setup_ms)
    per_sweep = sweep_bytes(p.n_nodes, p.nnzb, p.n_contacts, 8)
    achieved = per_sweep * L / (solve_avg * 1e-3) / 1e9
    traffic = load_traffic(traffic_name, L) if traffic_name else None
    sd = dist(solve_ms)
    return p, {
        "ms_per_step": ms_total / args.steps,
        "wall_s": wall,
        "value": p.n_contacts * L * args.steps / (ms_total * 1e-3),
        "stats": st,
        "setup_ms": setup_avg,
        "solve_ms": solve_avg,
        "solve_ms_median": sd["median"],
        "solve_ms_p90": sd["p90"],
        "sweep_us": solve_avg * 1e3 / L,
        "variant": variant,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": kernel_name(variant),
                     "bytes_per_launch": per_sweep * L,
                     "dram_gbps": None if traffic is None else traffic / (solve_avg * 1e-3) / 1e9},
    }


def batched_bench(args, torch, vf, scenes):
    """2048 cloth environments (side 8..48), FP32 with FP64 residual, one
    persistent launch per step captured in a HIP graph, largest-first queue."""
    import numpy as np
    envs = [sc.assemble(x, v) for sc, x, v in scenes.cloth_cfg4_envs(args.seed)]
    batch = scenes.concat_problems(envs)
    p = batch.problem
    dev = torch.device("cuda", 0)
    A = vf.bsr_from_arrays(p.n_nodes, p.row_ptr, p.col_idx, p.val, dtype=torch.float32, device=dev)
    crp, ccol, cval = p.jc_bsr()
    Jc = vf.contacts_from_arrays(crp, ccol, cval, p.phi, p.mu, dtype=torch.float32, device=dev)
    b = torch.as_tensor(p.b, device=dev).float()
    v = torch.as_tensor(p.v0, device=dev).float()
    no = torch.as_tensor(batch.env_node_off, device=dev)
    co = torch.as_tensor(batch.env_con_off, device=dev)
    order = torch.as_tensor(np.argsort([-e.nnzb for e in envs]).astype(np.int32), device=dev)
    lam = torch.empty(3 * p.n_contacts, dtype=torch.float32, device=dev)
    stats = vf.new_stats(batch.n_env, dev)
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts, batch.n_env)
    L = args.sweeps
    variant = args.batched_variant
    if variant == 0:
        from paper_2201_09212_amd import autotune
        variant = autotune.best_batched_variant(s, batch, A, b, Jc, v, lam, stats, no, co, order, L)
    opt = dict(max_iters=L, fixed_iters=True, variant=variant)
    run = lambda: s.step_batched(batch.n_env, no, co, A, b, Jc, v, lam, env_order=order, stats=stats, **opt)
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    # kernel duration from the library's own events (eager launches)
    vf.vfpi_timing_enable(s.ctx, True)
    kms = []
    for _ in range(max(3, args.steps // 4)):
        run()
        kms.append(vf.vfpi_timing_read(s.ctx)[1])
    vf.vfpi_timing_enable(s.ctx, False)
    # timed region: graph replays
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    st = vf.read_stats(stats)
    assert all(x["iters"] == L for x in st)
    # one fresh step from the warm start, kept for the oracle comparison of a
    # sample of environments (done in the CPU leg)
    v.copy_(torch.as_tensor(p.v0, device=dev).float())
    run()
    torch.cuda.synchronize()
    sizes = np.argsort([e.n_nodes for e in envs])
    pick = sorted(set(int(sizes[k]) for k in np.linspace(0, len(envs) - 1, 16).astype(int)))
    vh, lh = v.double().cpu().numpy(), lam.double().cpu().numpy()
    sample = [(envs[e], vh[3 * batch.env_node_off[e]:3 * batch.env_node_off[e + 1]],
               lh[3 * batch.env_con_off[e]:3 * batch.env_con_off[e + 1]]) for e in pick]
    s.close()
    kavg = sum(kms) / len(kms)
    per_sweep = sum(sweep_bytes(e.n_nodes, e.nnzb, e.n_contacts, 4) for e in envs)
    achieved = per_sweep * L / (kavg * 1e-3) / 1e9
    return {"value": batch.n_env / (ms * 1e-3), "unit": "env-step/s", "ms_per_step": ms, "n_env": batch.n_env,
            "n_nodes": p.n_nodes, "nnzb": p.nnzb, "n_contacts": p.n_contacts, "sweeps_per_step": L,
            "dtype": "f32 (f64 residual)", "graph": True, "variant": variant, "kernel_ms": kavg,
            "kernel_ms_median": dist(kms)["median"], "kernel_ms_p90": dist(kms)["p90"], "_sample": sample,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBPS, "traffic": load_traffic("batched2048", L),
                         "kernel": "k_vfpi_batched (persistent, one launch per step)",
                         "bytes_per_launch": per_sweep * L},
            "vs_plain_contact_iters_per_s": p.n_contacts * L / (ms * 1e-3)}


def adjoint_bench(args, torch, vf, scenes):
    """64x64 cloth: one converged step (tol 1e-13) forward with tape and its
    adjoint (kernel times), also with anisotropic friction and with the
    proximal operator, and a 100-step rollout with gradient (checkpoint every
    10 steps) against the same rollout without gradient."""
    from paper_2201_09212_amd.autograd import rollout
    from scenes.cloth_torch import TorchCloth
    dev = torch.device("cuda", 0)
    sc, x0, v0 = scenes.cloth_cfg5_scene(args.seed)
    tc = TorchCloth(sc, dev)
    s = vf.Solver(sc.n_nodes, tc.nnzb, sc.n_nodes)
    # single landed step: kernel times of forward and backward
    import numpy as np
    xl = x0.copy()
    xl[:, 2] = np.random.default_rng(args.seed).uniform(-5e-4, 4e-3, size=xl.shape[0])
    vl = v0.copy()
    vl[:, 2] -= 0.6
    p = sc.assemble(xl, vl)
    A = vf.bsr_from_arrays(p.n_nodes, p.row_ptr, p.col_idx, p.val, device=dev)
    crp, ccol, cval = p.jc_bsr()
    Jc = vf.contacts_from_arrays(crp, ccol, cval, p.phi, p.mu, device=dev)
    b = torch.as_tensor(p.b, device=dev)
    gv = torch.as_tensor(np.random.default_rng(1).normal(size=p.n), device=dev)
    tape = s.tape(p.n_nodes, p.n_contacts)
    vf.vfpi_timing_enable(s.ctx, True)
    fwd, bwd, fit, bit = [], [], 0, 0
    for _ in range(5):
        v = torch.as_tensor(p.v0, device=dev).clone()
        lam, st = s.step(A, b, Jc, v, tape=tape, max_iters=100000, tol=1e-13)
        fwd.append(vf.vfpi_timing_read(s.ctx)[1])
        g = s.step_backward(A, Jc, tape, gv, max_iters=100000, tol=1e-13, want_A=True)
        bwd.append(vf.vfpi_timing_read(s.ctx)[1])
        fit, bit = vf.read_stats(st)[0]["iters"], vf.read_stats(g["stats"])[0]["iters"]

    def variant_step(Jc_, **opt):
        """The same landed step with another contact model: kernel times and
        sweep counts of the converged forward and of its adjoint."""
        fw, bw = [], []
        for _ in range(3):
            v = torch.as_tensor(p.v0, device=dev).clone()
            _, st_ = s.step(A, b, Jc_, v, tape=tape, max_iters=100000, tol=1e-13, **opt)
            fw.append(vf.vfpi_timing_read(s.ctx)[1])
            g_ = s.step_backward(A, Jc_, tape, gv, max_iters=100000, tol=1e-13, want_A=True, **opt)
            bw.append(vf.vfpi_timing_read(s.ctx)[1])
        f_, b_ = vf.read_stats(st_)[0], vf.read_stats(g_["stats"])[0]
        return {"step_fwd_ms": sorted(fw)[1], "step_bwd_ms": sorted(bw)[1], "fwd_sweeps": f_["iters"],
                "bwd_sweeps": b_["iters"], "n_slip": f_["n_slip"],
                "converged": bool(f_["status"] == 0 and b_["status"] == 0)}

    Jc_aniso = vf.contacts_from_arrays(crp, ccol, cval, p.phi, p.mu, device=dev, mu2=0.5 * np.asarray(p.mu))
    variants = {"anisotropic, mu2 = mu/2 (f4)": variant_step(Jc_aniso),
                "proximal operator (f3)": variant_step(Jc, projection="proximal")}
    vf.vfpi_timing_enable(s.ctx, False)
    # rollout
    x0t = torch.as_tensor(x0, device=dev)
    v0t = torch.as_tensor(v0, device=dev)
    target = x0t.clone()
    kk = torch.tensor(1e3, device=dev, dtype=torch.float64, requires_grad=True)
    mu = torch.full((sc.n_nodes,), 0.5, device=dev, dtype=torch.float64, requires_grad=True)
    steps = args.rollout_steps
    # warm-up of both paths (first-call costs of the assembly ops and autograd)
    with torch.no_grad():
        rollout(tc, s, x0t, v0t, (kk, mu), 10)
    xw, _ = rollout(tc, s, x0t, v0t, (kk, mu), 10, checkpoint_every=10)
    ((xw - target) ** 2).sum().backward()
    kk.grad = None
    mu.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.no_grad():
        rollout(tc, s, x0t, v0t, (kk, mu), steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    xN, _ = rollout(tc, s, x0t, v0t, (kk, mu), steps, checkpoint_every=10)
    ((xN - target) ** 2).sum().backward()
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    s.close()
    fm, bm = sorted(fwd)[len(fwd) // 2], sorted(bwd)[len(bwd) // 2]
    return {"_cpu": (p, gv.cpu().numpy()),
            "step_fwd_ms": fm, "step_bwd_ms": bm, "bwd_over_fwd_step": bm / fm, "fwd_sweeps": fit,
            "bwd_sweeps": bit, "n_contacts": p.n_contacts, "rollout_steps": steps,
            "rollout_fwd_s": t_fwd, "rollout_fwd_bwd_s": t_fb,
            "bwd_over_fwd_rollout": (t_fb - t_fwd) / t_fwd, "contact_models": variants,
            "workload": "cloth64x64 on plane, FP64, converged to 1e-13, checkpoint every 10 steps"}


def extensions_bench(args, torch, vf, scenes, p):
    """Per-sweep cost of the paper's extensions at a fixed 100 sweeps, each
    next to the plain strict sweep of the same run: on the 128x128 cloth the
    proximal operator, the invertible contact (omega), anisotropic friction
    (mu2 = mu / 2), Chebyshev acceleration and BB1 step sizes; node-node
    contacts on two colliding 64x64 cloths; virtual nodes (eq. vnode) for
    particles on the 10x10 cloth, with the system build timed as well."""
    import numpy as np
    dev = torch.device("cuda", 0)
    L = 100

    def timed(prob_or_dev, opt, Jc_override=None, reps=5):
        A, b, Jc, vv, lam, stats = prob_or_dev
        Jc = Jc_override or Jc
        s = vf.Solver(A.n_nodes, A.nnzb, Jc.n_contacts)
        v0 = vv.clone()
        vf.vfpi_timing_enable(s.ctx, True)
        ms = []
        for _ in range(reps + 1):
            vv.copy_(v0)
            s.step(A, b, Jc, vv, lam, stats=stats, max_iters=L, fixed_iters=True, **opt)
            ms.append(vf.vfpi_timing_read(s.ctx)[1])
        vf.vfpi_timing_enable(s.ctx, False)
        st = vf.read_stats(stats)[0]
        assert st["iters"] == L and st["status"] == 1, st
        s.close()
        vv.copy_(v0)
        return dist(ms[1:])["median"] * 1e3 / L

    out = {}
    cl = upload(torch, vf, p)
    crp, ccol, cval = p.jc_bsr()
    Jc_aniso = vf.contacts_from_arrays(crp, ccol, cval, p.phi, p.mu, device=dev, mu2=0.5 * np.asarray(p.mu))
    base = timed(cl, {})
    rows = {"strict": base,
            "proximal (f3)": timed(cl, dict(projection="proximal")),
            "invertible, omega 1e-3 (f3)": timed(cl, dict(omega=1e-3)),
            "anisotropic, mu2 = mu/2 (f4)": timed(cl, {}, Jc_override=Jc_aniso),
            "Chebyshev l_s 10 (f1)": timed(cl, dict(cheby_ls=10)),
            "BB1 step sizes": timed(cl, dict(w_mode="bb1"))}
    out["cloth128"] = {k: {"sweep_us": v, "contact_iters_per_s": p.n_contacts / (v * 1e-6), "vs_strict": v / base}
                       for k, v in rows.items()}
    q = scenes.cloth_pair_collision(args.seed, side=64)
    t = timed(upload(torch, vf, q), {})
    out["d_contacts_pair64 (f2)"] = {"n_nodes": q.n_nodes, "nnzb": q.nnzb, "n_contacts": q.n_contacts,
                                    "sweep_us": t, "contact_iters_per_s": q.n_contacts / (t * 1e-6)}
    vs = scenes.particles_on_cloth(args.seed)
    A_o = vf.bsr_from_arrays(vs.n_o, vs.row_ptr, vs.col_idx, vs.val, device=dev)
    b_o = torch.as_tensor(vs.b, device=dev)
    v_o = torch.as_tensor(vs.v0, device=dev)
    jp, jc, jv = (torch.as_tensor(a) for a in (vs.jv_ptr, vs.jv_col, vs.jv_val))
    build = []
    for _ in range(6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A, b, v = vf.vnode_augment(A_o, b_o, v_o, jp, jc, jv, 1e4)
        torch.cuda.synchronize()
        build.append((time.perf_counter() - t0) * 1e3)
    pj = scenes.Problem(n_nodes=A.n_nodes, row_ptr=np.zeros(A.n_nodes + 1), col_idx=np.zeros(0),
                        val=np.zeros((0, 3, 3)), b=np.zeros(3 * A.n_nodes), v0=np.zeros(3 * A.n_nodes),
                        c_node=vs.c_node, c_node_j=vs.c_node_j, R=vs.R, phi=vs.phi, mu=vs.mu)
    crp, ccol, cval = pj.jc_bsr()
    Jv = vf.contacts_from_arrays(crp, ccol, cval, vs.phi, vs.mu, device=dev)
    lam = torch.empty(3 * Jv.n_contacts, dtype=torch.float64, device=dev)
    t = timed((A, b, Jv, v, lam, vf.new_stats(1, dev)), {})
    out["virtual_nodes_particles_on_cloth10 (f2)"] = {
        "n_nodes": A.n_nodes, "n_virtual": vs.n_v, "n_contacts": Jv.n_contacts, "k_v": 1e4,
        "system_build_ms_host_incl": dist(build[1:])["median"], "sweep_us": t}
    return out


def context_bench(args, torch, vf, scenes):
    """Convergence to theta < 1e-4 / 1e-6 (plain and Chebyshev) on the 128x128
    cloth and on the paper-size FEM block (16x16x4 cells, 4,335 DOF), the
    latter also at fixed 50 / 100 sweeps, next to the paper's soft-mat
    timings (other scene and hardware: context only)."""
    sc, x, v = scenes.fem_ctx(args.seed)
    q = sc.assemble(x, v)
    return {
        "cloth128_converge": converge_runs(torch, vf, args._cloth128, fixed=(50, 200)),
        "fem16x16x4": {"n_nodes": q.n_nodes, "dof": q.n, "nnzb": q.nnzb, "n_contacts": q.n_contacts,
                       "runs": converge_runs(torch, vf, q, tols=(1e-4, 1e-5, 1e-6), fixed=(50, 100)),
                       "paper_context": "soft mat, 4438 DOF, i5-7500 4C CPU: 8.65 ms and 39.72 iterations at "
                                        "1e-4 with Chebyshev; 10.85 / 20.90 ms at fixed 50 / 100 iterations"},
    }


# ---------------------------------------------------------------------------
# CPU baseline leg: the only part of the bench that runs the FP64 oracle
# (on the host cores, bounded samples of the same inputs).

_MC = {}


def _oracle_worker(budget_s):
    """Forked worker: the single-thread oracle on the parent's cloth input."""
    from threadpoolctl import threadpool_limits
    import oracle
    p, L = _MC["p"], _MC["L"]
    n = 0
    t0 = time.perf_counter()
    with threadpool_limits(1):
        while True:
            oracle.vfpi(p, max_iters=L, fixed_iters=True)
            n += 1
            if time.perf_counter() - t0 >= budget_s:
                break
    return n


def cpu_multicore(args, p, budget_s):
    """The oracle on every host core at once (one forked process per core,
    each a single-thread oracle on the same input): aggregate throughput.
    Runs before the process touches the GPU."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    P = max(1, min(16, len(os.sched_getaffinity(0))))
    _MC.update(p=p, L=args.sweeps)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(P, mp_context=mp.get_context("fork")) as ex:
        n = sum(ex.map(_oracle_worker, [budget_s] * P))
    el = time.perf_counter() - t0
    return {"value": p.n_contacts * args.sweeps * n / el, "unit": "contact-iter/s", "cores": P, "kind": "oracle",
            "sample": f"{n} steps x {args.sweeps} sweeps over {P} single-thread oracle processes on the "
                      f"128x128 cloth input, {el:.1f} s"}


def cpu_baseline(args, p, budget_s):
    import oracle
    L = args.sweeps
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.vfpi(p, max_iters=L, fixed_iters=True)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": p.n_contacts * L * n / el, "unit": "contact-iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} steps x {L} sweeps of the FP64 oracle (NumPy/SciPy, single thread) on the same "
                      f"128x128 cloth input, {el:.1f} s"}


def cpu_context(args, scenes, batched_sample=None, adjoint_step=None):
    """Oracle timings the paper's comparisons call for: V-FPI (plain and
    Chebyshev) against PGS on the Delassus operator on the 10x10 cloth and
    the paper-size FEM block; the oracle forward and adjoint of one converged
    64x64 cloth step; a sample of the batched environments in FP64 with the
    GPU FP32 result's relative error."""
    import numpy as np
    import oracle
    from oracle.adjoint import adjoint as oracle_adjoint
    from oracle.chebyshev import vfpi_chebyshev
    from oracle.delassus import delassus, pgs

    def rel(x, y):
        ny = np.linalg.norm(y)
        return float(np.linalg.norm(np.asarray(x) - y) / ny) if ny > 0 else float(np.abs(x).max(initial=0.0))

    out = {}
    for key, make in (("cloth10", lambda: scenes.cloth_cfg1(args.seed)),
                      ("fem16x16x4", lambda: scenes.fem_ctx(args.seed))):
        sc, x, v = make()
        q = sc.assemble(x, v)
        rows = []
        for tol in (1e-4, 1e-6):
            t0 = time.perf_counter()
            f = oracle.vfpi(q, max_iters=100000, tol=tol)
            t1 = time.perf_counter()
            g = vfpi_chebyshev(q, max_iters=100000, tol=tol, l_s=10)
            t2 = time.perf_counter()
            rows.append({"tol": tol, "vfpi_iters": f["iters"], "vfpi_s": t1 - t0,
                         "vfpi_cheby_iters": g["iters"], "vfpi_cheby_s": t2 - t1})
        t0 = time.perf_counter()
        dl = delassus(q)
        t_d = time.perf_counter() - t0
        for r in rows:
            t0 = time.perf_counter()
            h = pgs(q, tol=r["tol"], max_sweeps=5000, dl=dl)
            r.update(pgs_sweeps=h["sweeps"], pgs_s=time.perf_counter() - t0 + t_d)
        out[key] = {"n_nodes": q.n_nodes, "n_contacts": q.n_contacts, "delassus_s": t_d, "runs": rows}
    if adjoint_step is not None:
        q, gv = adjoint_step
        t0 = time.perf_counter()
        f = oracle.vfpi(q, max_iters=100000, tol=1e-13)
        t1 = time.perf_counter()
        a = oracle_adjoint(q, f, gv, None, tol=1e-13)
        t2 = time.perf_counter()
        out["adjoint_step_cloth64"] = {"fwd_s": t1 - t0, "bwd_s": t2 - t1, "bwd_over_fwd": (t2 - t1) / (t1 - t0),
                                       "fwd_sweeps": f["iters"], "bwd_sweeps": a.get("iters")}
    if batched_sample:
        errs, t = [], 0.0
        for e, vg, lg in batched_sample:
            t0 = time.perf_counter()
            f = oracle.vfpi(e, max_iters=args.sweeps, fixed_iters=True)
            t += time.perf_counter() - t0
            errs.append({"n_nodes": e.n_nodes, "n_contacts": e.n_contacts, "rel_err_v": rel(vg, f["v"]),
                         "rel_err_lambda": rel(lg, f["lam"].ravel()) if e.n_contacts else 0.0})
        out["batched_sample"] = {"envs": len(batched_sample), "oracle_env_steps_per_s": len(batched_sample) / t,
                                 "cores": 1, "max_rel_err": max(max(r["rel_err_v"], r["rel_err_lambda"])
                                                                for r in errs),
                                 "per_env": errs}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sweeps", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-soft", action="store_true", help="skip the FEM and 10x10 cloth legs")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-context", action="store_true",
                    help="skip the convergence runs (tolerances, Chebyshev, paper-size FEM block)")
    ap.add_argument("--batched-variant", type=int, default=0)
    ap.add_argument("--rollout-steps", type=int, default=100)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs are not part of it", file=sys.stderr)
        sys.exit(2)

    import torch

    import scenes

    sc, x, v = scenes.cloth_cfg2(args.seed)
    p = sc.assemble(x, v)
    args._cloth128 = p
    multicore = None
    if not args.no_cpu:
        multicore = cpu_multicore(args, p, args.cpu_seconds)

    import paper_2201_09212_amd as vf

    torch.cuda.set_device(0)
    p, r = plain_bench(args, torch, vf, scenes, p=p)
    out = {
        "metric": METRIC, "value": r["value"], "unit": "contact-iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "cloth128x128_16spheres_fp64", "n_nodes": p.n_nodes, "dof": p.n, "nnzb": p.nnzb,
                   "n_contacts": p.n_contacts, "sweeps_per_step": args.sweeps, "parallelism": "single GPU"},
        "hbm_gbps": r["roofline"]["achieved"], "hbm_frac": r["roofline"]["frac"],
        "sweep_us": r["sweep_us"], "setup_ms": r["setup_ms"], "solve_ms": r["solve_ms"], "variant": r["variant"],
        "dof_iters_per_s": p.n * args.sweeps * args.steps / (r["ms_per_step"] * args.steps * 1e-3),
        "solve_ms_median": r["solve_ms_median"], "solve_ms_p90": r["solve_ms_p90"],
        "roofline": r["roofline"],
    }
    out["roofline"]["measured_copy_gbps"] = copy_peak(torch)
    if not args.no_soft:
        # the other single-instance workloads: the FEM soft block and the 10x10 cloth
        for key, make, var, tn in (("fem", lambda: scenes.fem_cfg3(args.seed), 5 | (5 << 8), "fem"),
                                   ("cloth10", lambda: scenes.cloth_cfg1(args.seed), 5 | (2 << 8), None)):
            sc_, x_, v_ = make()
            q = sc_.assemble(x_, v_)
            _, rq = plain_bench(args, torch, vf, scenes, p=q, variant=var, traffic_name=tn)
            out[key] = {"workload": {"fem": "FEM block 64x64x16 cells, 5 tets/cell, FP64",
                                     "cloth10": "10x10 cloth landing on a plane, FP64"}[key],
                        "n_nodes": q.n_nodes, "nnzb": q.nnzb, "n_contacts": q.n_contacts,
                        "contact_iters_per_s": rq["value"], "sweep_us": rq["sweep_us"], "variant": var,
                        "hbm_gbps": rq["roofline"]["achieved"], "hbm_frac": rq["roofline"]["frac"],
                        "traffic": rq["roofline"]["traffic"], "dram_gbps": rq["roofline"]["dram_gbps"],
                        "kernel": rq["roofline"]["kernel"]}
    if not args.no_context:
        out["context"] = context_bench(args, torch, vf, scenes)
        out["extensions"] = extensions_bench(args, torch, vf, scenes, p)
    if not args.no_batched:
        out["batched"] = batched_bench(args, torch, vf, scenes)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_bench(args, torch, vf, scenes)
    sample = out["batched"].pop("_sample") if "batched" in out else None
    adj = out["adjoint"].pop("_cpu") if "adjoint" in out else None
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args, p, args.cpu_seconds)
        out["cpu_baseline_multicore"] = multicore
        out["cpu_context"] = cpu_context(args, scenes, sample, adj)
    if args.copy_calibration:
        x = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read_per_copy": 1 << 30, "bytes_written_per_copy": 1 << 30, "copies": 3}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
