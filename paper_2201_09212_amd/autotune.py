"""Launch-variant autotuner for the plain and batched V-FPI kernels.

A variant is the ``vfpi_opts.variant`` word: ``kind | slots << 8 | cap << 16``
where kind 1 = one lane per node, 2 = three lanes (rows) per node, 3/4 = the
same on a single workgroup, 5 = one lane per node with A's row kept in
registers for the whole step (one chunk pass per workgroup); ``slots`` = 64-node chunks per workgroup pass;
``cap`` = workgroup limit (0 = library default).  The tuner times each
candidate on the caller's own problem with the library's HIP events (a short
fixed number of sweeps), keeps the fastest, and caches the choice in a JSON
file keyed by the problem's shape, the candidate list and a hash of the built
library, so later runs of the same build skip the search and a rebuilt
library searches again.  The cache lives in the user's cache directory
(``$XDG_CACHE_HOME/vfpi`` or ``~/.cache/vfpi``), or at ``$VFPI_TUNE_CACHE``.
"""
from __future__ import annotations

import functools
import hashlib
import json
import os
import zlib

import torch

from . import _abi



def cache_path():
    env = os.environ.get("VFPI_TUNE_CACHE")
    if env:
        return env
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "vfpi", "tuned_variants.json")


@functools.lru_cache(maxsize=None)
def library_hash(path=_abi.LIB_PATH):
    """Short content hash of the built library: tuned choices are only valid
    for the kernels they were timed with."""
    h = hashlib.sha256()
    with open(path, "rb") as f:
        for blk in iter(lambda: f.read(1 << 20), b""):
            h.update(blk)
    return h.hexdigest()[:12]

PLAIN_CANDIDATES = [1 | (1 << 8), 1 | (2 << 8), 1 | (4 << 8), 2 | (1 << 8), 2 | (2 << 8),
                    1 | (2 << 8) | (128 << 16), 1 | (4 << 8) | (128 << 16), 3 | (16 << 8), 3 | (4 << 8),
                    5 | (1 << 8), 5 | (2 << 8), 5 | (4 << 8), 5 | (5 << 8), 5 | (6 << 8), 5 | (8 << 8)]
BATCHED_CANDIDATES = [1 | (1 << 8), 1 | (2 << 8), 1 | (4 << 8), 1 | (8 << 8), 2 | (1 << 8), 2 | (2 << 8),
                      3 | (4 << 8), 3 | (8 << 8), 4 | (16 << 8), 4 | (8 << 8), 4 | (8 << 8) | (1 << 26)]


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _time(solver, call, reps=3):
    _abi.vfpi_timing_enable(solver.ctx, True)
    try:
        call()  # warm-up
        best = None
        for _ in range(reps):
            call()
            ms = _abi.vfpi_timing_read(solver.ctx)[1]
            best = ms if best is None else min(best, ms)
        return best
    finally:
        _abi.vfpi_timing_enable(solver.ctx, False)


def cache_key(key, candidates):
    return f"{key}/cand{zlib.crc32(repr(candidates).encode()) & 0xffff:04x}/lib{library_hash()}"


def _search(key, candidates, call_for, log):
    key = cache_key(key, candidates)
    cache = _load()
    if key in cache:
        return int(cache[key]["variant"])
    results = {}
    for var in candidates:
        try:
            results[var] = _time(call_for.solver, lambda: call_for(var))
        except _abi.VfpiError:
            continue
        if log:
            log(f"autotune {key}: variant {var:#x} {results[var]:.3f} ms")
    best = min(results, key=results.get)
    cache[key] = {"variant": best, "ms": results[best], "candidates": {hex(k): v for k, v in results.items()}}
    _store(cache)
    return best


def best_step_variant(solver, A, b, Jc, v, lam, stats, sweeps=20, log=None):
    """Fastest vfpi_step variant for this problem shape (FP64)."""
    key = f"step/N{A.n_nodes}/nnzb{A.nnzb}/nc{Jc.n_contacts}"
    v0 = v.clone()

    def call(var):
        v.copy_(v0)
        solver.step(A, b, Jc, v, lam, stats=stats, max_iters=sweeps, fixed_iters=True, variant=var)

    call.solver = solver
    best = _search(key, PLAIN_CANDIDATES, call, log)
    v.copy_(v0)
    torch.cuda.synchronize()
    return best


def best_batched_variant(solver, batch, A, b, Jc, v, lam, stats, env_node_off, env_con_off, env_order, sweeps,
                         log=None):
    """Fastest vfpi_step_batched variant for this batch shape (FP32)."""
    key = f"batched/E{batch.n_env}/N{A.n_nodes}/nnzb{A.nnzb}/nc{Jc.n_contacts}"
    v0 = v.clone()
    short = max(5, min(sweeps, 20))

    def call(var):
        v.copy_(v0)
        solver.step_batched(batch.n_env, env_node_off, env_con_off, A, b, Jc, v, lam, env_order=env_order,
                            stats=stats, max_iters=short, fixed_iters=True, variant=var)

    call.solver = solver
    best = _search(key, BATCHED_CANDIDATES, call, log)
    v.copy_(v0)
    torch.cuda.synchronize()
    return best
