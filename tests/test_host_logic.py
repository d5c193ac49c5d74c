"""Host-side logic that needs no GPU: scene generators, serving accounting,
autotuner helpers."""
import math

import numpy as np

from paper_1810_01054_amd import scenes as S


def test_config_sizes_match_the_stated_workloads():
    assert S.config_1a().n_particles == 1024
    assert S.config_1b().n_particles == 4096
    c2 = S.config_2()
    assert c2.n_particles == 98304 and c2.n_act == 48 and c2.amp.shape == (48, 4)
    c3 = S.config_3()
    assert c3.n_particles == 504064 and c3.n_act == 16 and c3.n_grid == 64
    # every particle's stencil base is inside [0, n-3]
    for sc in (S.config_1a(), c2, c3):
        base = np.floor(sc.x.astype(np.float64) * sc.n_grid - 0.5)
        assert base.min() >= 0 and base.max() <= sc.n_grid - 3
    c4 = S.config_4()
    assert len(c4) == 64
    for sc in c4:
        assert sc.n_grid in (64, 128, 256)
        assert 1800 <= sc.n_particles <= 66000
        base = np.floor(sc.x.astype(np.float64) * sc.n_grid - 0.5)
        assert base.min() >= 0 and base.max() <= sc.n_grid - 3


def test_config5_request_mix():
    reqs = S.config_5(n_requests=40, rate=10.0)
    arr = [r.arrival for r in reqs]
    assert arr == sorted(arr) and arr[0] > 0
    dims = [r.scene.dim for r in reqs]
    assert 0 < dims.count(3) < 40
    for r in reqs:
        assert 100 <= r.T <= 500
        sc = r.scene
        base = np.floor(sc.x.astype(np.float64) * sc.n_grid - 0.5)
        assert base.min() >= 0 and base.max() <= sc.n_grid - 3


def test_serving_footprint_grows_with_work():
    from paper_1810_01054_amd.serve import footprint_bytes
    small = S.floor_block(np.random.default_rng(1), 2, 64, 2000)
    big = S.floor_block(np.random.default_rng(1), 2, 256, 50000)
    assert footprint_bytes(small, 100, 32) < footprint_bytes(big, 100, 32)
    assert footprint_bytes(big, 100, 32) < footprint_bytes(big, 400, 32)
    # the per-substep grids dominate a long 3D tape: T * (1 + d) * n^3 * 4 bytes
    q = S.floor_block(np.random.default_rng(2), 3, 64, 200000)
    assert footprint_bytes(q, 500, 32) > 500 * 4 * 64 ** 3 * 4


def test_serving_summary_percentiles():
    from paper_1810_01054_amd.serve import Result, summarize
    res = [Result(i, arrival=0.0, start=0.0, done=0.01 * (i + 1), particles=10, substeps=5)
           for i in range(100)]
    res[7].error = -3
    s = summarize(res, wall=1.0)
    assert s["failed"] == 1 and s["requests"] == 100
    assert abs(s["latency_s"]["p50"] - 0.505) < 0.011
    assert s["latency_s"]["p99"] <= 1.0 and s["particle_substeps_per_s"] == 99 * 50


def test_autotune_helpers():
    from paper_1810_01054_amd import autotune
    assert autotune.best_k(512) == 23 and autotune.best_k(1) == 1
    c2 = autotune.candidates(2)
    assert {"scatter": 3, "tile": 8, "graphs": True} in c2
    c3 = autotune.candidates(3)
    assert all(c["tile"] in (4, 8) for c in c3)
