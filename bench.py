#!/usr/bin/env python3
"""Benchmark of the V-FPI contact solve on one MI355X.

Headline: one step = one vfpi_step call (setup + the whole V-FPI loop, every
row of the hot path) on the co-rotated FEM soft block of 64x64x16 cells
(71,825 nodes, 215,475 DOF, 895,409 blocks, 12,675 contacts, FP64) with a
fixed number of sweeps per step and the inputs already resident in HBM.
Prints one JSON line:

  value        contact-iterations per second (sum of n_c * sweeps / solver time)
  roofline     the persistent sweep kernel: algorithmic bytes per launch over
               its average duration (HIP events the library records on the
               launch stream), against the 8 TB/s HBM peak
  cpu_baseline the CPU FP64 oracle on the same FEM input, one single-thread
               oracle process per host core allotted to the job, bounded
               sample, CPU model stated
  legs         the other workloads, each with its own numbers: the 128x128
               cloth over spheres and the 10x10 cloth (plain FP64), the
               2048-environment batched FP32 step (error against the oracle
               for every environment, and the free-running rollout
               divergence of a 16-environment sub-batch), the adjoint of the
               64x64 cloth, and the size sweep (time against size, Sec. V-D)

``--detail PATH`` also writes everything measured (convergence runs,
extensions, per-size rows, per-step divergence, CPU context) as JSON.

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

SCALING_CLOTH = (32, 64, 128, 256, 512, 768, 1024)
SCALING_FEM = ((16, 16, 4), (32, 32, 8), (48, 48, 12), (64, 64, 16), (128, 64, 16))


def sweep_bytes(n_nodes, nnzb, n_contacts, w):
    """Algorithmic bytes of one sweep: A read once (values + column index),
    row offsets, v / b / W read and v written once per DOF, the node->contact
    map, and per contact its packed record (R, phi, mu, gamma) read and lambda
    written."""
    return (nnzb * (9 * w + 4) + 4 * (n_nodes + 1) + 3 * n_nodes * 4 * w + 4 * n_nodes
            + n_contacts * (12 * w + 3 * w))


def kernel_name(variant, n_nodes=None):
    """The persistent sweep kernel a vfpi_step variant runs."""
    kind = variant & 0xff
    if kind == 0 and n_nodes is not None:
        kind = 5 if (n_nodes + 63) // 64 <= 8 * 256 else 1
    return {1: "k_vfpi_grid<1,NW> (lane per node, streamed A, grid)", 2: "k_vfpi_grid<3,NW> (lane per row, grid)",
            3: "k_vfpi_grid<1,NW> (one workgroup)", 4: "k_vfpi_grid<3,5> (one workgroup)",
            5: "k_vfpi_regs (A's first levels in registers, grid)"}.get(kind, f"kind {kind}")


def kernel_sources_hash():
    """Hash of the HIP sources of the forward and batched kernels with
    comments and whitespace removed, so that the stored byte counters stay
    valid across documentation edits but not across code changes.  The
    backward (adjoint.hip) and the virtual-node builder (vnode.hip) are
    included after those kernels in the one translation unit and define
    nothing they use, so they are left out; so is the allocation-free entry
    point (noalloc.hip, last in that unit), which only calls vfpi_step, and
    the host-side context and error-string code (api.hip), which holds no
    device code."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2201_09212_amd", "csrc")
    skip = ("adjoint.hip", "vnode.hip", "noalloc.hip", "api.hip")
    for f in sorted(os.listdir(csrc)):
        if f in skip:
            continue
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        if f == "vfpi_lib.hip":
            src = src.replace('#include "noalloc.hip"', " ")
        h.update(f.encode() + " ".join(src.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(name):
    """HBM traffic per launch from the committed rocprofv3 --pmc summary
    (profiles/traffic.json, one entry per workload), or None when the
    kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f).get(name)
    if not t or t.get("sources_hash") != kernel_sources_hash():
        return None
    return t.get("bytes_per_launch")


def dist(xs):
    """Mean, median and 90th percentile of a list of timings."""
    s = sorted(xs)
    return {"mean": sum(s) / len(s), "median": s[len(s) // 2], "p90": s[min(len(s) - 1, int(0.9 * len(s)))]}


def r3(x, n=4):
    """Round for the compact line."""
    if isinstance(x, float):
        return float(f"{x:.{n}g}")
    return x


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


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


def converge_runs(torch, vf, p, tols=(1e-4, 1e-6), cheby=(0, 10), reps=3, fixed=(), dev_data=None):
    """Iterations and solver time to reach theta < tol from the step's warm
    start, plain and with Chebyshev acceleration (l_s = 10, u = 1), with the
    library's default launch; optionally also fixed sweep counts."""
    A, b, Jc, vv, lam, stats = dev_data or upload(torch, vf, p)
    v0 = vv.clone()
    runs = [dict(tol=t, cheby_ls=c) for c in cheby for t in tols] + [dict(fixed=L) for L in fixed]
    out = []
    with vf.Solver(p.n_nodes, p.nnzb, p.n_contacts) as s:
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
    vv.copy_(v0)
    return out


def plain_bench(args, torch, vf, p, variant=0, traffic_name=None, tune=False):
    """The timed loop of one single-instance workload: W warm-up steps, then
    K steps between two events; then K steps again with the library's own
    events around the setup and the persistent kernel (the roofline's
    duration)."""
    A, b, Jc, vv, lam, stats = upload(torch, vf, p)
    L = args.sweeps
    with vf.Solver(p.n_nodes, p.nnzb, p.n_contacts) as s:
        if tune and variant == 0:
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
        vf.vfpi_timing_enable(s.ctx, True)
        setup_ms, solve_ms = [], []
        for _ in range(args.steps):
            s.step(A, b, Jc, vv, lam, stats=stats, **opt)
            a, c = vf.vfpi_timing_read(s.ctx)
            setup_ms.append(a)
            solve_ms.append(c)
        vf.vfpi_timing_enable(s.ctx, False)
    solve_avg = sum(solve_ms) / len(solve_ms)
    per_sweep = sweep_bytes(p.n_nodes, p.nnzb, p.n_contacts, 8)
    achieved = per_sweep * L / (solve_avg * 1e-3) / 1e9
    traffic = load_traffic(traffic_name) if traffic_name else None
    sd = dist(solve_ms)
    return {
        "ms_per_step": ms_total / args.steps, "wall_s": wall,
        "value": p.n_contacts * L * args.steps / (ms_total * 1e-3), "stats": st,
        "setup_ms": sum(setup_ms) / len(setup_ms), "solve_ms": solve_avg, "solve_ms_median": sd["median"],
        "solve_ms_p90": sd["p90"], "sweep_us": solve_avg * 1e3 / L, "variant": variant,
        "dof_iters_per_s": p.n * L * args.steps / (ms_total * 1e-3),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": kernel_name(variant, p.n_nodes), "bytes_per_launch": per_sweep * L,
                     "bytes_per_sweep": per_sweep, "sweeps_per_launch": L,
                     "dram_gbps": None if traffic is None else traffic / (solve_avg * 1e-3) / 1e9},
    }


def batched_bench(args, torch, vf, envs, batch):
    """2048 cloth environments (side 8..48), FP32 with FP64 residual, one
    persistent launch per step captured in a HIP graph, largest-first queue.
    Also returns one fresh step's result for every environment (compared
    with the oracle on the host cores)."""
    import numpy as np
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
    L = args.sweeps
    with vf.Solver(p.n_nodes, p.nnzb, p.n_contacts, batch.n_env) as s:
        variant = args.batched_variant
        if variant == 0:
            from paper_2201_09212_amd import autotune
            variant = autotune.best_batched_variant(s, batch, A, b, Jc, v, lam, stats, no, co, order, L)
        opt = dict(max_iters=L, fixed_iters=True, variant=variant)
        run = lambda: s.step_batched(batch.n_env, no, co, A, b, Jc, v, lam, env_order=order, stats=stats, **opt)
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        vf.vfpi_timing_enable(s.ctx, True)
        kms = []
        for _ in range(max(3, args.steps // 4)):
            run()
            kms.append(vf.vfpi_timing_read(s.ctx)[1])
        vf.vfpi_timing_enable(s.ctx, False)
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
        # one fresh step from the warm start, for the oracle comparison
        v.copy_(torch.as_tensor(p.v0, device=dev).float())
        run()
        torch.cuda.synchronize()
        vh, lh = v.double().cpu().numpy(), lam.double().cpu().numpy()
        del g
    kavg = sum(kms) / len(kms)
    per_sweep = sum(sweep_bytes(e.n_nodes, e.nnzb, e.n_contacts, 4) for e in envs)
    achieved = per_sweep * L / (kavg * 1e-3) / 1e9
    traffic = load_traffic("batched2048")
    return {"value": batch.n_env / (ms * 1e-3), "unit": "env-step/s", "ms_per_step": ms, "n_env": batch.n_env,
            "n_nodes": p.n_nodes, "nnzb": p.nnzb, "n_contacts": p.n_contacts, "sweeps_per_step": L,
            "dtype": "f32 (f64 residual)", "graph": True, "variant": variant, "kernel_ms": kavg,
            "kernel_ms_median": dist(kms)["median"], "kernel_ms_p90": dist(kms)["p90"], "_result": (vh, lh),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                         "kernel": "k_vfpi_batched (persistent, one launch per step)",
                         "bytes_per_launch": per_sweep * L,
                         "dram_gbps": None if traffic is None else traffic / (kavg * 1e-3) / 1e9},
            "vs_plain_contact_iters_per_s": p.n_contacts * L / (ms * 1e-3)}


def rollout_envs(envs_all, k=16):
    """Indices of a sub-batch spread over the size range, half of them with
    contacts at the first step."""
    import numpy as np
    sizes = np.array([sc.n_nodes for sc, _, _ in envs_all])
    order = np.argsort(sizes, kind="stable")
    pick = [int(order[q]) for q in np.linspace(0, len(order) - 1, k).astype(int)]
    return sorted(set(pick))


def batched_rollout_gpu(args, torch, vf, scenes, envs_sub, steps):
    """Free-running FP32 batched rollout of a sub-batch: each step assembles
    every environment at the GPU's own state (host), solves the batch in one
    vfpi_step_batched launch (fixed sweeps) and advances x += h v.  Returns
    per-step positions and velocities of every environment."""
    import numpy as np
    dev = torch.device("cuda", 0)
    state = [(sc, x.copy(), v.copy()) for sc, x, v in envs_sub]
    n_nodes = sum(sc.n_nodes for sc, _, _ in state)
    nnzb = sum(int(sc.row_ptr[-1]) for sc, _, _ in state)
    xs, vs = [], []
    with vf.Solver(n_nodes, nnzb, n_nodes, len(state)) as s:
        for _ in range(steps):
            probs = [sc.assemble(x, v) for sc, x, v in state]
            batch = scenes.concat_problems(probs)
            p = batch.problem
            A = vf.bsr_from_arrays(p.n_nodes, p.row_ptr, p.col_idx, p.val, dtype=torch.float32, device=dev)
            crp, ccol, cval = p.jc_bsr()
            Jc = vf.contacts_from_arrays(crp, ccol, cval, p.phi, p.mu, dtype=torch.float32, device=dev)
            b = torch.as_tensor(p.b, device=dev).float()
            vd = torch.as_tensor(p.v0, device=dev).float()
            no = torch.as_tensor(batch.env_node_off, device=dev)
            co = torch.as_tensor(batch.env_con_off, device=dev)
            s.step_batched(batch.n_env, no, co, A, b, Jc, vd, max_iters=args.sweeps, fixed_iters=True)
            vh = vd.double().cpu().numpy()
            new = []
            for e, (sc, x, v) in enumerate(state):
                ve = vh[3 * batch.env_node_off[e]:3 * batch.env_node_off[e + 1]].reshape(-1, 3)
                new.append((sc, sc.advance(x, ve), ve))
            state = new
            xs.append([x.copy() for _, x, _ in state])
            vs.append([v.copy() for _, _, v in state])
    return xs, vs


def rollout_bench(args, torch, vf, scenes):
    """The 10x10 cloth dropped 2 cm onto the plane (100 steps) and the 128x128
    cloth dropped onto its 16 spheres (200 steps, mass damping 5/s) as the
    rollouts those workloads name: every step assembles A, b and the contacts on the host at the GPU's
    own state, solves to theta < tol on the GPU and advances x += h v, so the
    contact set evolves.  Run with W recomputed every step, and with the row
    sums of W reused (reuse_w) for nine steps in ten.  A step that does not
    converge (status other than converged) or returns a non-finite iterate
    ends its rollout, which reports where.  Per rollout: GPU setup and solve
    time, sweeps, contact counts, host time (assembly and transfers)."""
    import numpy as np
    cases = (("cloth10_drop_100_steps", lambda: scenes.cloth_cfg1(args.seed, landing=False), 100),
             ("cloth128_drop_onto_spheres_200_steps", lambda: scenes.cloth_cfg2_drop(args.seed), 200))
    out = {}
    for name, make, steps in cases:
        res = {}
        for reuse in (False, True):
            sc, x, v = make()
            solve, setup, sweeps, ncs = [], [], [], []
            host = 0.0
            failed = None
            t0 = time.perf_counter()
            with vf.Solver(sc.n_nodes, int(sc.row_ptr[-1]), sc.n_nodes) as s:
                vf.vfpi_timing_enable(s.ctx, True)
                for k in range(steps):
                    th = time.perf_counter()
                    p = sc.assemble(x, v)
                    A, b, Jc, vv, lam, stats = upload(torch, vf, p)
                    host += time.perf_counter() - th
                    s.step(A, b, Jc, vv, lam, stats=stats, max_iters=args.rollout_max_iters, tol=args.rollout_tol,
                           reuse_w=reuse and k % 10 != 0)
                    a_, c_ = vf.vfpi_timing_read(s.ctx)
                    st = vf.read_stats(stats)[0]
                    setup.append(a_)
                    solve.append(c_)
                    sweeps.append(st["iters"])
                    ncs.append(p.n_contacts)
                    th = time.perf_counter()
                    v = vv.cpu().numpy().reshape(-1, 3)
                    host += time.perf_counter() - th
                    if st["status"] != 0 or not np.all(np.isfinite(v)):
                        failed = {"step": k, "status": st["status"], "iters": st["iters"], "theta": st["theta"]}
                        break
                    th = time.perf_counter()
                    x = sc.advance(x, v)
                    host += time.perf_counter() - th
            res["reuse_w" if reuse else "w_every_step"] = {
                "gpu_solve_ms": sum(solve), "gpu_setup_ms": sum(setup), "sweeps_total": sum(sweeps),
                "sweeps_mean": sum(sweeps) / len(sweeps), "sweeps_max": max(sweeps),
                "contacts_first_last_max": [ncs[0], ncs[-1], max(ncs)], "host_ms": host * 1e3,
                "wall_ms": (time.perf_counter() - t0) * 1e3, "final_x": x.copy(),
                "steps_done": len(sweeps), "stopped": failed}
        out[name] = {"steps": steps, "tol": args.rollout_tol, **res}
    return out


def adjoint_bench(args, torch, vf, scenes):
    """64x64 cloth: one converged step (tol 1e-13) forward with tape and its
    adjoint (kernel times), also with anisotropic friction and with the
    proximal operator, and a 100-step rollout with gradient (checkpoint every
    10 steps) against the same rollout without gradient."""
    import numpy as np
    from paper_2201_09212_amd.autograd import rollout
    from scenes.cloth_torch import TorchCloth
    dev = torch.device("cuda", 0)
    sc, x0, v0 = scenes.cloth_cfg5_scene(args.seed)
    tc = TorchCloth(sc, dev)
    s = vf.Solver(sc.n_nodes, tc.nnzb, sc.n_nodes)
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

    def variant_step(Jc_, s_=s, A_=A, b_=b, tape_=tape, gv_=gv, v0_=p.v0, **opt):
        fw, bw = [], []
        for _ in range(3):
            v = torch.as_tensor(v0_, device=dev).clone()
            _, st_ = s_.step(A_, b_, Jc_, v, tape=tape_, max_iters=100000, tol=1e-13, **opt)
            fw.append(vf.vfpi_timing_read(s_.ctx)[1])
            g_ = s_.step_backward(A_, Jc_, tape_, gv_, max_iters=100000, tol=1e-13, want_A=True, **opt)
            bw.append(vf.vfpi_timing_read(s_.ctx)[1])
        f_, bs = vf.read_stats(st_)[0], vf.read_stats(g_["stats"])[0]
        return {"step_fwd_ms": sorted(fw)[1], "step_bwd_ms": sorted(bw)[1], "fwd_sweeps": f_["iters"],
                "bwd_sweeps": bs["iters"], "n_slip": f_["n_slip"],
                "bwd_over_fwd": sorted(bw)[1] / sorted(fw)[1],
                "converged": bool(f_["status"] == 0 and bs["status"] == 0)}

    Jc_aniso = vf.contacts_from_arrays(crp, ccol, cval, p.phi, p.mu, device=dev, mu2=0.5 * np.asarray(p.mu))
    variants = {"anisotropic, mu2 = mu/2 (f4)": variant_step(Jc_aniso),
                "proximal operator (f3)": variant_step(Jc, projection="proximal")}
    vf.vfpi_timing_enable(s.ctx, False)
    # D-contacts (J_m = [R, -R] on two nodes): two 64x64 cloths meeting in free fall
    q = scenes.cloth_pair_collision(args.seed, side=64)
    sq = vf.Solver(q.n_nodes, q.nnzb, q.n_contacts)
    Aq, bq, Jq, _, _, _ = upload(torch, vf, q)
    vf.vfpi_timing_enable(sq.ctx, True)
    variants["D-contacts, two 64x64 cloths (f2)"] = variant_step(
        Jq, s_=sq, A_=Aq, b_=bq, tape_=sq.tape(q.n_nodes, q.n_contacts),
        gv_=torch.as_tensor(np.random.default_rng(2).normal(size=q.n), device=dev), v0_=q.v0)
    variants["D-contacts, two 64x64 cloths (f2)"]["n_contacts"] = q.n_contacts
    sq.close()
    x0t = torch.as_tensor(x0, device=dev)
    v0t = torch.as_tensor(v0, device=dev)
    target = x0t.clone()
    kk = torch.tensor(1e3, device=dev, dtype=torch.float64, requires_grad=True)
    mu = torch.full((sc.n_nodes,), 0.5, device=dev, dtype=torch.float64, requires_grad=True)
    steps = args.rollout_steps
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
        v0 = vv.clone()
        with vf.Solver(A.n_nodes, A.nnzb, Jc.n_contacts) as s:
            vf.vfpi_timing_enable(s.ctx, True)
            ms = []
            for _ in range(reps + 1):
                vv.copy_(v0)
                s.step(A, b, Jc, vv, lam, stats=stats, max_iters=L, fixed_iters=True, **opt)
                ms.append(vf.vfpi_timing_read(s.ctx)[1])
            st = vf.read_stats(stats)[0]
            assert st["iters"] == L and st["status"] == 1, st
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


def context_bench(args, torch, vf, scenes, cloth128):
    """Convergence to theta < 1e-4 / 1e-6 (plain and Chebyshev) on the 128x128
    cloth and on the paper-size FEM block (16x16x4 cells, 4,335 DOF), the
    latter also at fixed 50 / 100 sweeps, next to the paper's soft-mat
    timings (other scene and hardware: context only)."""
    sc, x, v = scenes.fem_ctx(args.seed)
    q = sc.assemble(x, v)
    return {
        "cloth128_converge": converge_runs(torch, vf, cloth128, fixed=(50, 200)),
        "fem16x16x4": {"n_nodes": q.n_nodes, "dof": q.n, "nnzb": q.nnzb, "n_contacts": q.n_contacts,
                       "runs": converge_runs(torch, vf, q, tols=(1e-4, 1e-5, 1e-6), fixed=(50, 100)),
                       "paper_context": "soft mat, 4438 DOF, i5-7500 4C CPU: 8.65 ms and 39.72 iterations at "
                                        "1e-4 with Chebyshev; 10.85 / 20.90 ms at fixed 50 / 100 iterations"},
    }


def linfit_r2(xs, ys):
    """Least-squares line y = a x + c and its coefficient of determination."""
    import numpy as np
    x, y = np.asarray(xs, float), np.asarray(ys, float)
    a, c = np.polyfit(x, y, 1)
    res = y - (a * x + c)
    ss = ((y - y.mean()) ** 2).sum()
    return {"slope": float(a), "intercept": float(c), "r2": float(1.0 - (res ** 2).sum() / ss) if ss > 0 else 1.0}


def scaling_bench(args, torch, vf, scenes, cloth_sides=SCALING_CLOTH, fem_cells=SCALING_FEM):
    """Solver time against problem size (the paper's scalability experiment,
    Sec. V-D, on FEM blocks; here also on cloth): per size the library's
    default launch at a fixed 100 sweeps (per-sweep time, algorithmic GB/s,
    counter traffic when committed) and the sweeps and time to theta < 1e-4,
    plain and with Chebyshev (l_s = 10).  R^2 of a straight-line fit of the
    time to 1e-4 and of the fixed-sweep time against the DOF count."""
    rows = []
    cases = [("cloth", s, lambda s=s: scenes.cloth_drape(s, args.seed)) for s in cloth_sides]
    cases += [("fem", c, lambda c=c: scenes.fem_block(c, args.seed)) for c in fem_cells]
    for fam, size, make in cases:
        t0 = time.perf_counter()
        sc, x, v = make()
        p = sc.assemble(x, v)
        host_s = time.perf_counter() - t0
        name = f"{fam}{'x'.join(map(str, size)) if fam == 'fem' else f'{size}x{size}'}"
        dd = upload(torch, vf, p)
        runs = converge_runs(torch, vf, p, tols=(1e-4,), cheby=(0, 10), reps=2, fixed=(100,), dev_data=dd)
        fx = runs[-1]
        per_sweep = sweep_bytes(p.n_nodes, p.nnzb, p.n_contacts, 8)
        traffic = load_traffic(f"scaling_{name}")
        rows.append({"workload": name, "n_nodes": p.n_nodes, "dof": p.n, "nnzb": p.nnzb, "n_contacts": p.n_contacts,
                     "a_mb": p.nnzb * 76 / 1e6, "kernel": kernel_name(0, p.n_nodes),
                     "sweep_us": fx["solve_ms"] * 1e3 / 100, "setup_ms": fx["setup_ms"],
                     "gbps": per_sweep * 100 / (fx["solve_ms"] * 1e-3) / 1e9,
                     "dram_gbps": None if traffic is None else traffic / (fx["solve_ms"] * 1e-3) / 1e9,
                     "tol1e-4_iters": runs[0]["iters"], "tol1e-4_ms": runs[0]["solve_ms"],
                     "tol1e-4_cheby_iters": runs[1]["iters"], "tol1e-4_cheby_ms": runs[1]["solve_ms"],
                     "host_build_s": host_s})
        del dd
        torch.cuda.empty_cache()
    fits = {}
    for fam in ("cloth", "fem"):
        rr = [r for r in rows if r["workload"].startswith(fam)]
        if len(rr) >= 3:
            dof = [r["dof"] for r in rr]
            fits[fam] = {"tol1e-4_ms_vs_dof": linfit_r2(dof, [r["tol1e-4_ms"] for r in rr]),
                         "tol1e-4_cheby_ms_vs_dof": linfit_r2(dof, [r["tol1e-4_cheby_ms"] for r in rr]),
                         "fixed100_ms_vs_dof": linfit_r2(dof, [r["sweep_us"] * 0.1 for r in rr])}
    return {"rows": rows, "fits": fits}


# ---------------------------------------------------------------------------
# CPU leg: the only part of the bench that runs the FP64 oracle (on the host
# cores, bounded samples of the same inputs), in processes forked before the
# parent touches the GPU.

_MC = {}


def _oracle_worker(budget_s):
    """Single-thread oracle on the headline input until the budget is spent."""
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
    return n, time.perf_counter() - t0


def _env_oracle(e):
    """FP64 oracle step of batched environment e (same sweeps as the GPU)."""
    from threadpoolctl import threadpool_limits
    import oracle
    with threadpool_limits(1):
        f = oracle.vfpi(_MC["envs"][e], max_iters=_MC["L"], fixed_iters=True)
    return f["v"], f["lam"].ravel()


def _env_rollout_oracle(e):
    """FP64 oracle rollout of one environment of the divergence sub-batch."""
    from threadpoolctl import threadpool_limits
    import oracle
    sc, x, v = _MC["roll_envs"][e]
    x, v = x.copy(), v.copy()
    xs, vs = [], []
    with threadpool_limits(1):
        for _ in range(_MC["roll_steps"]):
            f = oracle.vfpi(sc.assemble(x, v), max_iters=_MC["L"], fixed_iters=True)
            v = f["v"].reshape(-1, 3)
            x = sc.advance(x, v)
            xs.append(x.copy())
            vs.append(v.copy())
    return xs, vs


def _cloth10_rollout_oracle(args_t):
    """FP64 oracle rollout of the 10x10 cloth drop (the same steps as the
    GPU's, W recomputed every step)."""
    from threadpoolctl import threadpool_limits
    import oracle
    import scenes
    seed, steps, tol, max_iters = args_t
    sc, x, v = scenes.cloth_cfg1(seed, landing=False)
    sw = []
    with threadpool_limits(1):
        for _ in range(steps):
            f = oracle.vfpi(sc.assemble(x, v), max_iters=max_iters, tol=tol)
            sw.append(f["iters"])
            v = f["v"].reshape(-1, 3)
            x = sc.advance(x, v)
    return x, sw


def cpu_baseline(pool, P, p, args, what):
    """The oracle on every allotted host core at once (one single-thread
    process per core, same input): aggregate and per-process throughput."""
    _MC.update(p=p, L=args.sweeps)
    t0 = time.perf_counter()
    res = pool.map(_oracle_worker, [args.cpu_seconds] * P, chunksize=1)
    el = time.perf_counter() - t0
    n = sum(r[0] for r in res)
    single = sum(p.n_contacts * args.sweeps * r[0] / r[1] for r in res) / len(res)
    return {"value": p.n_contacts * args.sweeps * n / el, "unit": "contact-iter/s", "cores": P, "kind": "oracle",
            "cpu_model": cpu_model(), "single_thread_value": single,
            "sample": f"{n} steps x {args.sweeps} sweeps of the FP64 oracle (NumPy/SciPy, one single-thread "
                      f"process per core, {P} cores allotted to the job) on the same {what} input, {el:.1f} s"}


def batched_errors(envs, batch, vh, lh, oracle_res):
    """Per-environment error of the FP32 batched step against the FP64 oracle:
    norm-wise relative error and element-wise error max_i |x_i - y_i| /
    max_j |y_j| (all-zero reference: max |x_i|), for v and lambda; maximum
    over all environments and per size class."""
    import numpy as np

    def ew(x, y):
        if y.size == 0:
            return 0.0
        s = np.abs(y).max()
        return float(np.abs(x - y).max() / s) if s > 0 else float(np.abs(x).max())

    def rn(x, y):
        ny = np.linalg.norm(y)
        return float(np.linalg.norm(x - y) / ny) if ny > 0 else float(np.abs(x).max(initial=0.0))

    rows = []
    for e, (vo, lo) in enumerate(oracle_res):
        n0, n1 = batch.env_node_off[e], batch.env_node_off[e + 1]
        m0, m1 = batch.env_con_off[e], batch.env_con_off[e + 1]
        vg, lg = vh[3 * n0:3 * n1], lh[3 * m0:3 * m1]
        side = int(round(np.sqrt(envs[e].n_nodes)))
        rows.append((side, envs[e].n_contacts, ew(vg, vo), ew(lg, lo), rn(vg, vo), rn(lg, lo)))
    classes = {"8-14": (8, 14), "15-22": (15, 22), "23-34": (23, 34), "35-48": (35, 48)}
    out = {"envs": len(rows), "envs_with_contacts": sum(1 for r in rows if r[1] > 0),
           "max_elementwise_v": max(r[2] for r in rows), "max_elementwise_lambda": max(r[3] for r in rows),
           "max_rel_v": max(r[4] for r in rows), "max_rel_lambda": max(r[5] for r in rows), "by_side": {}}
    for k, (a, b) in classes.items():
        rr = [r for r in rows if a <= r[0] <= b]
        if rr:
            out["by_side"][k] = {"envs": len(rr), "max_elementwise": max(max(r[2], r[3]) for r in rr),
                                 "max_rel": max(max(r[4], r[5]) for r in rr)}
    return out


def rollout_divergence(gpu_xs, gpu_vs, orc):
    """Per step, over the sub-batch, between the free-running FP32 GPU rollout
    and the FP64 oracle rollout: the largest position difference (m), the
    largest velocity difference (m/s), and the largest velocity difference
    relative to the environment's largest oracle speed over the whole rollout
    (a cloth that has come to rest has v near zero, so a per-step norm would
    divide FP32 rounding by nothing)."""
    import numpy as np
    steps = len(gpu_xs)
    scale = [max(float(np.abs(v).max()) for v in ovs) for _, ovs in orc]
    dx, dv, dr = [], [], []
    for k in range(steps):
        mx, mv, mr = 0.0, 0.0, 0.0
        for e, (oxs, ovs) in enumerate(orc):
            mx = max(mx, float(np.abs(gpu_xs[k][e] - oxs[k]).max()))
            d = float(np.abs(gpu_vs[k][e] - ovs[k]).max())
            mv = max(mv, d)
            mr = max(mr, d / scale[e] if scale[e] > 0 else d)
        dx.append(mx)
        dv.append(mv)
        dr.append(mr)
    return dx, dv, dr


def cpu_context(args, scenes, adjoint_step=None):
    """Oracle timings the paper's comparisons call for: V-FPI (plain and
    Chebyshev) against PGS on the Delassus operator on the 10x10 cloth and
    the paper-size FEM block; the oracle forward and adjoint of one converged
    64x64 cloth step."""
    import oracle
    from oracle.adjoint import adjoint as oracle_adjoint
    from oracle.chebyshev import vfpi_chebyshev
    from oracle.delassus import delassus, pgs

    out = {}
    for key, make in (("cloth10", lambda: scenes.cloth_cfg1(args.seed)),
                      ("fem16x16x4", lambda: scenes.fem_ctx(args.seed))):
        print(f"bench: cpu context {key}", file=sys.stderr, flush=True)
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
        print("bench: cpu context adjoint", file=sys.stderr, flush=True)
        q, gv = adjoint_step
        t0 = time.perf_counter()
        f = oracle.vfpi(q, max_iters=100000, tol=1e-13)
        t1 = time.perf_counter()
        a = oracle_adjoint(q, f, gv, None, tol=1e-13)
        t2 = time.perf_counter()
        out["adjoint_step_cloth64"] = {"fwd_s": t1 - t0, "bwd_s": t2 - t1, "bwd_over_fwd": (t2 - t1) / (t1 - t0),
                                       "fwd_sweeps": f["iters"], "bwd_sweeps": a.get("iters")}
    return out


def leg_summary(r, p, workload):
    """Compact form of a single-instance leg for the JSON line."""
    rf = r["roofline"]
    return {"workload": workload, "n_nodes": p.n_nodes, "nnzb": p.nnzb, "n_contacts": p.n_contacts,
            "value": r3(r["value"]), "unit": "contact-iter/s", "sweep_us": r3(r["sweep_us"]),
            "setup_ms": r3(r["setup_ms"]), "variant": r["variant"],
            "roofline": {"bound": rf["bound"], "achieved": r3(rf["achieved"]), "peak": rf["peak"], "unit": "GB/s",
                         "frac": r3(rf["frac"]), "traffic": rf["traffic"],
                         "dram_gbps": r3(rf["dram_gbps"]) if rf["dram_gbps"] else None,
                         "dram_frac": r3(rf["dram_gbps"] / HBM_PEAK_GBPS) if rf["dram_gbps"] else None,
                         "kernel": rf["kernel"]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sweeps", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--variant", type=lambda x: int(x, 0), default=0, help="launch variant of the FEM headline (0: library default)")
    ap.add_argument("--cloth-variant", type=lambda x: int(x, 0), default=0, help="launch variant of the cloth128 leg (0: autotuned)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-cores", type=int, default=0, help="0: every core allotted to the job, at most 16")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-soft", action="store_true", help="skip the cloth128 and 10x10 cloth legs")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-context", action="store_true",
                    help="skip the convergence runs (tolerances, Chebyshev, paper-size FEM block) and extensions")
    ap.add_argument("--no-scaling", action="store_true", help="skip the size sweep")
    ap.add_argument("--no-rollout", action="store_true", help="skip the batched rollout divergence")
    ap.add_argument("--scaling-only", action="store_true", help="only the size sweep (for counter runs)")
    ap.add_argument("--batched-variant", type=lambda x: int(x, 0), default=0)
    ap.add_argument("--rollout-steps", type=int, default=100)
    ap.add_argument("--rollout-tol", type=float, default=1e-6, help="tolerance of the cloth rollouts' steps")
    ap.add_argument("--rollout-max-iters", type=int, default=2000)
    ap.add_argument("--no-cloth-rollouts", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--detail", default="", help="also write every measurement to this JSON file")
    ap.add_argument("--maps-out", default="",
                    help="write the process's memory map (/proc/self/maps) to this file at exit, to resolve the "
                         "addresses of a native stack trace printed after the program ends")
    args = ap.parse_args()
    if args.maps_out:
        import atexit

        def _dump_maps(path=args.maps_out):
            os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
            with open("/proc/self/maps") as src, open(path, "w") as dst:
                dst.write(src.read())
        atexit.register(_dump_maps)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on one GPU; --gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)
    if args.scaling_only:
        args.no_cpu = args.no_batched = args.no_soft = args.no_adjoint = args.no_context = True

    import numpy as np
    import torch

    import scenes

    def say(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    sc, x, v = scenes.fem_cfg3(args.seed)
    p_fem = sc.assemble(x, v)
    sc, x, v = scenes.cloth_cfg2(args.seed)
    p_cl = sc.assemble(x, v)
    envs_all = envs = batch = None
    if not args.no_batched:
        envs_all = scenes.cloth_cfg4_envs(args.seed)
        envs = [sc_.assemble(x_, v_) for sc_, x_, v_ in envs_all]
        batch = scenes.concat_problems(envs)
    pool, P = None, 0
    cpu_base = None
    if not args.no_cpu:
        import multiprocessing as mp
        P = args.cpu_cores or max(1, min(16, len(os.sched_getaffinity(0))))
        sub = [envs_all[e] for e in rollout_envs(envs_all)] if envs_all else []
        _MC.update(p=p_fem, L=args.sweeps, envs=envs, roll_envs=sub, roll_steps=args.rollout_steps)
        pool = mp.get_context("fork").Pool(P)  # forked before anything touches the GPU
        say(f"cpu baseline: FEM oracle on {P} cores")
        cpu_base = cpu_baseline(pool, P, p_fem, args, "FEM block 64x64x16")

    import paper_2201_09212_amd as vf

    torch.cuda.set_device(0)
    detail = {}
    legs = {}
    out = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    if not args.scaling_only:
        say("FEM block (headline)")
        r = plain_bench(args, torch, vf, p_fem, variant=args.variant, traffic_name="fem")
        r["roofline"]["measured_copy_gbps"] = copy_peak(torch)
        rf = r["roofline"]
        out.update({
            "value": r["value"], "unit": "contact-iter/s", "ms_per_step": r["ms_per_step"],
            "config": {"workload": "fem_block_64x64x16_cells_5tets_fp64", "n_nodes": p_fem.n_nodes, "dof": p_fem.n,
                       "nnzb": p_fem.nnzb, "n_contacts": p_fem.n_contacts, "sweeps_per_step": args.sweeps,
                       "parallelism": "single GPU"},
            "roofline": {k: rf[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        })
        out["roofline"].update(kernel=rf["kernel"], bytes_per_launch=rf["bytes_per_launch"],
                               dram_gbps=rf["dram_gbps"], measured_copy_gbps=rf["measured_copy_gbps"],
                               dram_frac=(rf["dram_gbps"] / HBM_PEAK_GBPS) if rf["dram_gbps"] else None,
                               residency="A (68 MB FP64) barely leaves the chip between sweeps: its first eleven "
                                         "block levels stay in VGPRs and LDS, the streamed rest in the 256 MB "
                                         "Infinity Cache; the algorithmic bytes (every block, gather and store "
                                         "once per sweep) are the 8 TB/s roofline's convention, so frac can "
                                         "exceed 1; dram_frac is what reaches HBM")
        out.update({"sweep_us": r["sweep_us"], "setup_ms": r["setup_ms"], "solve_ms_median": r["solve_ms_median"],
                    "solve_ms_p90": r["solve_ms_p90"], "dof_iters_per_s": r["dof_iters_per_s"],
                    "variant": r["variant"]})
        if cpu_base:
            out["cpu_baseline"] = cpu_base
        detail["fem"] = r
    if not args.no_soft:
        say("cloth128 / cloth10")
        r = plain_bench(args, torch, vf, p_cl, variant=args.cloth_variant, traffic_name="cloth128", tune=True)
        legs["cloth128"] = leg_summary(r, p_cl, "cloth 128x128 over 16 spheres, FP64")
        legs["cloth128"]["roofline"]["residency"] = ("A in VGPRs/LDS for the whole step; DRAM traffic is the "
                                                     "neighbour gathers and v stores")
        detail["cloth128"] = r
        sc, x, v = scenes.cloth_cfg1(args.seed)
        q = sc.assemble(x, v)
        r = plain_bench(args, torch, vf, q, variant=5 | (2 << 8))
        legs["cloth10"] = leg_summary(r, q, "cloth 10x10 landing on a plane, FP64")
        detail["cloth10"] = r
    if not args.no_soft and not args.no_cloth_rollouts:
        say("cloth rollouts (10x10 drop, 128x128 drop onto spheres)")
        orc10 = None
        if pool is not None:
            orc10 = pool.apply_async(_cloth10_rollout_oracle,
                                     ((args.seed, 100, args.rollout_tol, args.rollout_max_iters),))
        rr = rollout_bench(args, torch, vf, scenes)
        legs["cloth_rollouts"] = {}
        for k, r in rr.items():
            legs["cloth_rollouts"][k] = {"steps": r["steps"], "tol": r["tol"]}
            for mode in ("w_every_step", "reuse_w"):
                m = dict(r[mode])
                m.pop("final_x")
                legs["cloth_rollouts"][k][mode] = {a: (r3(b_) if isinstance(b_, float) else b_) for a, b_ in m.items()}
        if orc10 is not None:
            ox, osw = orc10.get()
            gx = rr["cloth10_drop_100_steps"]["w_every_step"]["final_x"]
            legs["cloth_rollouts"]["cloth10_drop_100_steps"]["vs_oracle_rollout"] = {
                "max_final_position_diff_m": r3(float(np.abs(gx - ox).max()), 3),
                "oracle_sweeps_total": int(sum(osw))}
        detail["cloth_rollouts"] = {k: {m: {a: b_ for a, b_ in r[m].items() if a != "final_x"}
                                        for m in ("w_every_step", "reuse_w")} for k, r in rr.items()}
    if not args.no_context:
        say("convergence runs and extensions")
        detail["context"] = context_bench(args, torch, vf, scenes, p_cl)
        detail["extensions"] = extensions_bench(args, torch, vf, scenes, p_cl)
        fc = detail["context"]["fem16x16x4"]["runs"]
        legs["convergence_fem16x16x4_tol1e-4"] = {
            "plain": {"iters": fc[0]["iters"], "solve_ms": r3(fc[0]["solve_ms"])},
            "chebyshev_ls10": {"iters": fc[3]["iters"], "solve_ms": r3(fc[3]["solve_ms"])},
            "paper_context": "soft mat 4438 DOF, i5-7500: 39.72 iterations, 8.65 ms (Chebyshev)"}
    if not args.no_batched:
        say("batched 2048 environments")
        rb = batched_bench(args, torch, vf, envs, batch)
        vh, lh = rb.pop("_result")
        roll = None
        orc_async = None
        if pool is not None and not args.no_rollout:
            orc_async = pool.map_async(_env_rollout_oracle, range(len(_MC["roll_envs"])), chunksize=1)
        if not args.no_rollout:
            say("batched rollout (16 environments)")
            sub = [envs_all[e] for e in rollout_envs(envs_all)]
            gx, gv_ = batched_rollout_gpu(args, torch, vf, scenes, sub, args.rollout_steps)
            if orc_async is not None:
                dx, dv, dr = rollout_divergence(gx, gv_, orc_async.get())
                ks = [k for k in (1, 10, 25, 50, 100) if k <= len(dx)]
                roll = {"envs": len(sub), "steps": args.rollout_steps, "sweeps_per_step": args.sweeps,
                        "max_pos_diff_m": {str(k): r3(dx[k - 1], 3) for k in ks},
                        "max_v_diff_mps": {str(k): r3(dv[k - 1], 3) for k in ks},
                        "max_v_diff_over_max_speed": {str(k): r3(dr[k - 1], 3) for k in ks},
                        "gated": False}
                detail["batched_rollout"] = {"max_pos_diff_m": dx, "max_v_diff_mps": dv,
                                             "max_v_diff_over_max_speed": dr}
        errs = None
        if pool is not None:
            say("batched: oracle on every environment")
            t0 = time.perf_counter()
            res = pool.map(_env_oracle, range(batch.n_env), chunksize=8)
            t_orc = time.perf_counter() - t0
            errs = batched_errors(envs, batch, vh, lh, res)
            errs["oracle_env_steps_per_s"] = batch.n_env / t_orc
            errs["oracle_cores"] = P
        rbf = rb["roofline"]
        legs["batched"] = {"workload": "2048 cloth envs side 8..48, FP32 + FP64 residual, graph-captured",
                           "value": r3(rb["value"]), "unit": "env-step/s", "ms_per_step": r3(rb["ms_per_step"]),
                           "variant": rb["variant"],
                           "vs_plain_contact_iters_per_s": r3(rb["vs_plain_contact_iters_per_s"]),
                           "roofline": {"bound": "hbm", "achieved": r3(rbf["achieved"]), "peak": HBM_PEAK_GBPS,
                                        "unit": "GB/s", "frac": r3(rbf["frac"]), "traffic": rbf["traffic"],
                                        "dram_gbps": r3(rbf["dram_gbps"]) if rbf["dram_gbps"] else None,
                                        "dram_frac": r3(rbf["dram_gbps"] / HBM_PEAK_GBPS) if rbf["dram_gbps"] else None,
                                        "residency": "each environment's iterate in LDS and the first 512 nodes' first "
                                                     "9 levels of A in registers for the whole step, so the "
                                                     "algorithmic bytes exceed what DRAM serves (frac > 1 is that, "
                                                     "not a rate above the peak); dram_frac is the counted traffic"}}
        if errs:
            legs["batched"]["error_vs_oracle_all_envs"] = {
                k: (r3(v_, 3) if isinstance(v_, float) else v_) for k, v_ in errs.items() if k != "by_side"}
            legs["batched"]["error_vs_oracle_all_envs"]["by_side"] = {
                k: {"envs": c["envs"], "max_elementwise": r3(c["max_elementwise"], 3)}
                for k, c in errs["by_side"].items()}
        if roll:
            legs["batched"]["rollout_divergence"] = roll
        detail["batched"] = {**rb, "errors": errs}
    adj = None
    if not args.no_adjoint:
        say("adjoint")
        ra = adjoint_bench(args, torch, vf, scenes)
        adj = ra.pop("_cpu")
        legs["adjoint"] = {"workload": ra["workload"], "bwd_over_fwd_step": r3(ra["bwd_over_fwd_step"]),
                           "step_fwd_ms": r3(ra["step_fwd_ms"]), "step_bwd_ms": r3(ra["step_bwd_ms"]),
                           "fwd_sweeps": ra["fwd_sweeps"], "bwd_sweeps": ra["bwd_sweeps"],
                           "bwd_over_fwd_rollout": r3(ra["bwd_over_fwd_rollout"]),
                           "rollout_fwd_s": r3(ra["rollout_fwd_s"]), "rollout_fwd_bwd_s": r3(ra["rollout_fwd_bwd_s"]),
                           "aniso_bwd_over_fwd": r3(ra["contact_models"]["anisotropic, mu2 = mu/2 (f4)"]
                                                    ["bwd_over_fwd"]),
                           "d_contact_bwd_over_fwd": r3(ra["contact_models"]["D-contacts, two 64x64 cloths (f2)"]
                                                        ["bwd_over_fwd"])}
        detail["adjoint"] = ra
    if not args.no_scaling:
        say("size sweep")
        rs = scaling_bench(args, torch, vf, scenes)
        legs["scaling"] = {
            "rows": [[r["workload"], r["dof"], r3(r["a_mb"], 3), r3(r["sweep_us"]), r3(r["gbps"]),
                      r["tol1e-4_iters"], r3(r["tol1e-4_ms"]), r["tol1e-4_cheby_iters"], r3(r["tol1e-4_cheby_ms"])]
                     for r in rs["rows"]],
            "columns": ["workload", "dof", "A_MB", "sweep_us", "alg_GBps", "iters_1e-4", "ms_1e-4",
                        "cheby_iters_1e-4", "cheby_ms_1e-4"],
            "r2_ms_1e-4_vs_dof": {f: r3(v_["tol1e-4_ms_vs_dof"]["r2"]) for f, v_ in rs["fits"].items()},
            "r2_fixed100_vs_dof": {f: r3(v_["fixed100_ms_vs_dof"]["r2"]) for f, v_ in rs["fits"].items()}}
        detail["scaling"] = rs
        if args.scaling_only:
            out.update({"value": None, "unit": "contact-iter/s", "config": {"workload": "size sweep only"}})
    if pool is not None:
        say("cpu context")
        detail["cpu_context"] = cpu_context(args, scenes, adj)
        pool.close()
        pool.join()
    if args.copy_calibration:
        xx = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        yy = torch.empty_like(xx)
        for _ in range(3):
            yy.copy_(xx)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read_per_copy": 1 << 30, "bytes_written_per_copy": 1 << 30, "copies": 3}
        del xx, yy
    out["legs"] = legs
    if args.detail:
        def plain(o):
            if isinstance(o, dict):
                return {str(k): plain(v_) for k, v_ in o.items()}
            if isinstance(o, (list, tuple)):
                return [plain(v_) for v_ in o]
            if hasattr(o, "tolist"):
                return o.tolist()
            return o if isinstance(o, (int, float, str, bool)) or o is None else str(o)
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as f:
            json.dump(plain({"line": out, "detail": detail}), f, indent=1)
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
