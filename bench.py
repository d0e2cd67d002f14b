#!/usr/bin/env python3
"""Benchmark of the V-FPI contact solve on one MI355X.

One step = one vfpi_step call (setup + the whole V-FPI loop, every row of the
hot path) on the 128x128 cloth draped over 16 spheres (49,152 DOF, ~5.2k
contacts, FP64), with a fixed number of sweeps per step and the inputs already
resident in HBM.  Prints one JSON line:

  value        contact-iterations per second (sum of n_c * sweeps / solver time)
  roofline     the persistent sweep kernel: algorithmic bytes per launch over
               its average duration (HIP events on the launch stream)
  cpu_baseline the CPU FP64 oracle on the same input, bounded sample
  batched      batched FP32 environments (env-steps/s), when enabled
  adjoint      backward/forward time ratio, when enabled

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


def kernel_sources_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2201_09212_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
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


def plain_bench(args, torch, vf, scenes):
    sc, x, v = scenes.cloth_cfg2(args.seed)
    p = sc.assemble(x, v)
    dev = torch.device("cuda", 0)
    A = vf.bsr_from_arrays(p.n_nodes, p.row_ptr, p.col_idx, p.val, device=dev)
    crp, ccol, cval = p.jc_bsr()
    Jc = vf.contacts_from_arrays(crp, ccol, cval, p.phi, p.mu, device=dev)
    b = torch.as_tensor(p.b, device=dev)
    vv = torch.as_tensor(p.v0, device=dev).clone()
    lam = torch.empty(3 * p.n_contacts, dtype=torch.float64, device=dev)
    stats = vf.new_stats(1, dev)
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)
    L = args.sweeps
    opt = dict(max_iters=L, fixed_iters=True, variant=args.variant)
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
    traffic = load_traffic("cloth128", L)
    return p, {
        "ms_per_step": ms_total / args.steps,
        "wall_s": wall,
        "value": p.n_contacts * L * args.steps / (ms_total * 1e-3),
        "stats": st,
        "setup_ms": setup_avg,
        "solve_ms": solve_avg,
        "sweep_us": solve_avg * 1e3 / L,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic,
                     "kernel": "k_vfpi_grid (persistent sweep loop)",
                     "bytes_per_launch": per_sweep * L},
    }


def cpu_baseline(args, p, oracle_mod, budget_s):
    L = args.sweeps
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle_mod.vfpi(p, max_iters=L, fixed_iters=True)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": p.n_contacts * L * n / el, "unit": "contact-iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} steps x {L} sweeps of the FP64 oracle (NumPy/SciPy, single thread) on the same "
                      f"128x128 cloth input, {el:.1f} s"}


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
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs are not part of it", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2201_09212_amd as vf
    import scenes

    torch.cuda.set_device(0)
    p, r = plain_bench(args, torch, vf, scenes)
    out = {
        "metric": METRIC, "value": r["value"], "unit": "contact-iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "cloth128x128_16spheres_fp64", "n_nodes": p.n_nodes, "dof": p.n, "nnzb": p.nnzb,
                   "n_contacts": p.n_contacts, "sweeps_per_step": args.sweeps, "parallelism": "single GPU"},
        "hbm_gbps": r["roofline"]["achieved"], "hbm_frac": r["roofline"]["frac"],
        "sweep_us": r["sweep_us"], "setup_ms": r["setup_ms"], "solve_ms": r["solve_ms"],
        "dof_iters_per_s": p.n * args.sweeps * args.steps / (r["ms_per_step"] * args.steps * 1e-3),
        "roofline": r["roofline"],
    }
    if not args.no_cpu:
        import oracle
        out["cpu_baseline"] = cpu_baseline(args, p, oracle, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
