"""The launch-variant autotuner: its cache lives outside the package and is
keyed by the built library's hash (CPU); on the GPU it picks a candidate that
solves the problem to the oracle's result, and a second call is served from
the cache without timing anything."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2201_09212_amd import autotune


def test_cache_outside_package_and_keyed_by_library(tmp_path, monkeypatch):
    monkeypatch.delenv("VFPI_TUNE_CACHE", raising=False)
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    p = autotune.cache_path()
    assert p.startswith(str(tmp_path)) and "paper_2201_09212_amd" not in p
    monkeypatch.setenv("VFPI_TUNE_CACHE", str(tmp_path / "x.json"))
    assert autotune.cache_path() == str(tmp_path / "x.json")
    lib = tmp_path / "lib.so"
    lib.write_bytes(b"one build")
    h1 = autotune.library_hash(str(lib))
    lib.write_bytes(b"another build")
    assert autotune.library_hash.__wrapped__(str(lib)) != h1
    k = autotune.cache_key("step/N5", autotune.PLAIN_CANDIDATES)
    assert k.startswith("step/N5/cand") and f"/lib{autotune.library_hash()}" in k


@pytest.mark.gpu
def test_search_picks_a_correct_variant_and_caches_it(tmp_path, monkeypatch):
    import oracle
    import paper_2201_09212_amd as vf
    import scenes
    from tests.gpu_util import gate, upload

    monkeypatch.setenv("VFPI_TUNE_CACHE", str(tmp_path / "tune.json"))
    p = scenes.random_problem(900, 300, 21, degree=5.0, phi_scale=0.5)
    s = vf.Solver(p.n_nodes, p.nnzb, p.n_contacts)
    A, Jc, b, v = upload(p)
    lam = torch.empty(3 * p.n_contacts, dtype=torch.float64, device="cuda")
    stats = vf.new_stats(1)
    lines = []
    var = autotune.best_step_variant(s, A, b, Jc, v, lam, stats, log=lines.append)
    assert var in autotune.PLAIN_CANDIDATES and len(lines) >= 5
    cache = json.load(open(os.environ["VFPI_TUNE_CACHE"]))
    (key, entry), = cache.items()
    assert entry["variant"] == var and key.endswith(f"/lib{autotune.library_hash()}")
    lines2 = []
    assert autotune.best_step_variant(s, A, b, Jc, v, lam, stats, log=lines2.append) == var and not lines2
    assert np.array_equal(v.cpu().numpy(), p.v0)  # the search leaves the warm start as it was
    s.step(A, b, Jc, v, lam, stats=stats, max_iters=20, fixed_iters=True, variant=var)
    ref = oracle.vfpi(p, max_iters=20, fixed_iters=True)
    gate(v.cpu().numpy(), ref["v"], 1e-9, "tuned variant v")
    gate(lam.cpu().numpy(), ref["lam"], 1e-9, "tuned variant lambda")
    s.close()
