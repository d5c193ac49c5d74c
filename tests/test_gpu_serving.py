"""Serving loop on the GPU: requests batched into one multi-scene context per
lane (one launch per kernel per substep for the whole batch, each scene held
fixed past its own T).  In deterministic mode each request's result in the
mix equals its result served alone bit for bit (final positions, the
velocity adjoint and dL/ds under a loss that depends on the actuation); a
poisoned request fails alone while the rest of its batch is served; admission
respects the memory budget while batches overlap."""
import zlib

import numpy as np
import pytest
import torch

from paper_1810_01054_amd import scenes as S
from paper_1810_01054_amd.serve import Server, footprint_bytes, summarize
from tests.gpu_helpers import require_gpu, say

pytestmark = pytest.mark.gpu


def _requests(burst=True, n=8):
    rng = np.random.default_rng(1816)
    reqs = []
    for i in range(n):
        if i % 2 == 0:
            m = int(rng.choice([32, 64]))
            sc = S.floor_block(rng, 2, m, int(rng.integers(800, 3000)), name=f"r{i}")
        else:
            sc = S.floor_block(rng, 3, 24, int(rng.integers(1500, 6000)), name=f"r{i}")
        T = int(rng.integers(20, 41))
        reqs.append(S.Request(arrival=0.0 if burst else 5e-4 * i, scene=sc, T=T))
    return reqs


def _seed(sc):
    # L = centroid x + a seeded linear form of the final positions (the
    # centroid alone barely depends on the actuation over a few dozen
    # substeps in free flight)
    rng = np.random.default_rng(zlib.crc32(sc.name.encode()))
    d, N = sc.dim, sc.n_particles
    gx = np.zeros((d, N))
    gx[0] += 1.0 / N
    gx += rng.normal(size=(d, N)) / N
    return [gx.astype(np.float32), np.zeros((d, N), np.float32),
            np.zeros((d * d, N), np.float32), np.zeros((d * d, N), np.float32)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _bits(t):
    return t.detach().cpu().numpy().view(np.uint32)


def test_mix_equals_alone_and_poisoned_request_fails_alone():
    reqs = _requests()
    bad = S.floor_block(np.random.default_rng(7), 2, 32, 900, name="bad")
    bad.x[0, 5] = 0.1 / 32          # stencil base below 0: MPM_ERR_DOMAIN
    reqs.insert(3, S.Request(arrival=0.0, scene=bad, T=25))
    say("serving mix", len(reqs))
    mix_srv = Server(max_batch=8, lanes=2, ckpt_k=8, keep_results=True, deterministic=True,
                     seed_of=_seed)
    mix = mix_srv.run(reqs)
    alone = Server(ckpt_k=8, keep_results=True, deterministic=True,
                   seed_of=_seed).run(reqs, fifo=True)
    assert mix[3].error == -3 and alone[3].error == -3
    assert max(len(b) for b in mix_srv.batches) > 1      # requests shared launches
    for i, (a, b) in enumerate(zip(mix, alone)):
        if i == 3:
            continue
        assert a.error is None and b.error is None, (i, a.error, b.error)
        assert np.array_equal(_bits(a.xT), _bits(b.xT)), i
        assert np.array_equal(_bits(a.g_v0), _bits(b.g_v0)), i
        assert np.array_equal(_bits(a.g_act), _bits(b.g_act)), i
        assert np.abs(b.g_act.cpu().numpy()).max() > 0.0
    s = summarize(mix)
    assert s["failed"] == 1 and s["latency_s"]["p99"] is not None


def test_admission_respects_the_budget():
    reqs = _requests(burst=False, n=12)
    fps = [footprint_bytes(r.scene, r.T, 8) for r in reqs]
    budget = int(2.5 * max(fps))
    say("serving budget", budget)
    srv = Server(max_batch=8, lanes=2, hbm_budget=budget, ckpt_k=8)
    res = srv.run(reqs)
    assert all(r.error is None for r in res)
    assert srv.peak_bytes <= budget
    # requests started while others were still running (continuous
    # admission), and the requests of every batch fit the budget
    overlap = sum(1 for a in res for b in res
                  if a.index < b.index and b.start < a.done)
    assert overlap > 0
    for b in srv.batches:
        assert len(b) == 1 or sum(fps[i] for i in b) <= budget
