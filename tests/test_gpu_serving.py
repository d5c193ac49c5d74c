"""Serving loop on the GPU: each request's result in the mix equals its result
served alone (within the GPU parity tolerance), a poisoned request fails on
its own, and admission respects the memory budget."""
import numpy as np
import pytest
import torch

from paper_1810_01054_amd import scenes as S
from paper_1810_01054_amd.serve import Server, footprint_bytes, summarize
from tests.gpu_helpers import require_gpu, say
from tests.helpers import err

pytestmark = pytest.mark.gpu


def _requests(burst=True):
    rng = np.random.default_rng(1816)
    reqs = []
    for i in range(8):
        if i % 2 == 0:
            n = int(rng.choice([32, 64]))
            sc = S.floor_block(rng, 2, n, int(rng.integers(800, 3000)), name=f"r{i}")
        else:
            sc = S.floor_block(rng, 3, 24, int(rng.integers(1500, 6000)), name=f"r{i}")
        T = int(rng.integers(20, 41))
        reqs.append(S.Request(arrival=0.0 if burst else 5e-4 * i, scene=sc, T=T))
    return reqs


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_mix_equals_alone_and_poisoned_request_fails_alone():
    reqs = _requests()
    bad = S.floor_block(np.random.default_rng(7), 2, 32, 900, name="bad")
    bad.x[0, 5] = 0.1 / 32          # stencil base below 0: MPM_ERR_DOMAIN
    reqs.insert(3, S.Request(arrival=0.0, scene=bad, T=25))
    say("serving mix", len(reqs))
    mix = Server(max_slots=4, ckpt_k=8, keep_results=True).run(reqs)
    alone = Server(max_slots=1, ckpt_k=8, keep_results=True).run(reqs, fifo=True)
    assert mix[3].error == -3 and alone[3].error == -3
    for i, (a, b) in enumerate(zip(mix, alone)):
        if i == 3:
            continue
        assert a.error is None and b.error is None, (i, a.error, b.error)
        assert err(a.xT.cpu().numpy(), b.xT.cpu().numpy()) < 1e-6
        assert err(a.g_v0.cpu().numpy(), b.g_v0.cpu().numpy()) < 1e-5
        # the centroid loss barely depends on actuation over a few dozen
        # substeps (|dL/ds| ~ 1e-16, rounding level): compare absolutely
        assert np.allclose(a.g_act.cpu().numpy(), b.g_act.cpu().numpy(),
                           rtol=1e-4, atol=1e-10)
    s = summarize(mix)
    assert s["failed"] == 1 and s["latency_s"]["p99"] is not None


def test_admission_respects_the_budget():
    reqs = _requests(burst=False)
    fps = [footprint_bytes(r.scene, r.T, 8) for r in reqs]
    budget = int(2.5 * max(fps))
    say("serving budget", budget)
    srv = Server(max_slots=8, hbm_budget=budget, ckpt_k=8)
    res = srv.run(reqs)
    assert all(r.error is None for r in res)
    assert srv.peak_bytes <= budget
    # requests started while others were still running (continuous admission),
    # never more at once than the budget holds
    overlap = sum(1 for a in res for b in res
                  if a.index < b.index and b.start < a.done)
    assert overlap > 0
    most = max(sum(1 for b in res if b.start <= a.start < b.done) for a in res)
    assert most * min(fps) <= budget
