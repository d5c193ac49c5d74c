"""Request loop for forward + gradient rollout requests.

Each request is one scene (2D or 3D), a number of substeps T and its
actuation parameters; serving it means a forward rollout and the reverse
pass (final state, adjoint of the initial state, actuation gradient).

Scheduling: requests are admitted in arrival order as soon as a slot is free
and their device-memory footprint fits the budget.  Every admitted request
gets its own libmpm context on its own HIP stream, so the rollouts of all
admitted requests are in flight on the device at once and overlap there; a
request that arrives while others are running starts without waiting for
them.  Completion is detected with a stream event; latency is measured from
arrival to completion.  ``fifo=True`` replays the plain one-at-a-time loop.

Marshalling and scheduling only: the simulation runs in the library.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import scenes as S
from ._lib import MPMError
from .sim import Simulator, act_bank_forward


@dataclass
class Result:
    index: int
    arrival: float
    start: float = math.nan
    done: float = math.nan
    error: Optional[int] = None
    particles: int = 0
    substeps: int = 0
    xT: Optional[torch.Tensor] = None
    g_v0: Optional[torch.Tensor] = None
    g_act: Optional[torch.Tensor] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def footprint_bytes(scene: S.Scene, T: int, ckpt_k: int, tile: Optional[int] = None) -> int:
    """Upper estimate of the device memory one request holds: the context's
    grids, tile boxes and binning arrays, the tape (checkpoints, segment
    states, per-substep grids), and the request's own tensors."""
    d, n, N = scene.dim, scene.n_grid, scene.n_particles
    B = tile or (8 if d == 2 else 4)
    G = n ** d
    nt = (n - 2 + B - 1) // B
    tiles = nt ** d
    S_ = B + 4
    state = (2 * d + 2 * d * d) * N * 4
    ctx = ((2 + 4 * d) * G * 4            # m, p, v, vbar, pbar, mbar
           + state                         # scratch state
           + 8 * N * 4                     # binning per particle
           + tiles * (B ** d + 6) * 4      # per-cell / per-tile counts
           + tiles * (d + 1) * S_ ** d * 4)  # tile boxes
    k = max(1, min(ckpt_k, T)) if ckpt_k > 0 else 1
    ncp = (T + k - 1) // k + 1 if ckpt_k > 0 else T + 1
    tape = ((ncp + (2 * k if ckpt_k > 0 else 0) + 4) * state
            + T * (1 + d) * G * 4
            + T * max(scene.n_act, 1) * 12)
    own = 5 * state + T * max(scene.n_act, 1) * 8
    return int(1.1 * (ctx + tape + own)) + (8 << 20)


class _Slot:
    def __init__(self, res: Result, sim: Simulator, stream, event, keep, nbytes):
        self.res, self.sim, self.stream, self.event = res, sim, stream, event
        self.keep, self.nbytes = keep, nbytes


class Server:
    """Continuous admission of rollout requests onto concurrent streams."""

    def __init__(self, max_slots: int = 8, hbm_budget: Optional[int] = None,
                 ckpt_k: int = 32, keep_results: bool = False, poll_s: float = 2e-4):
        self.max_slots = max_slots
        if hbm_budget is None:
            free, total = torch.cuda.mem_get_info()
            hbm_budget = int(0.6 * free)
        self.budget = hbm_budget
        self.ckpt_k = ckpt_k
        self.keep_results = keep_results
        self.poll_s = poll_s
        self.streams = [torch.cuda.Stream() for _ in range(max_slots)]
        self.peak_bytes = 0

    def _launch(self, i, req, res: Result, stream) -> _Slot:
        sc = req.scene
        nbytes = footprint_bytes(sc, req.T, self.ckpt_k)
        dev = torch.device("cuda")
        with torch.cuda.stream(stream):
            t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(
                dev, non_blocking=False)
            sim = Simulator([sc.params()], act_id=sc.act_id, stream=stream)
            s0 = tuple(t(a) for a in sc.state)
            act = act_bank_forward(req.T, sc.dt, t(sc.freq), t(sc.amp), t(sc.phase),
                                   stream=stream)
            gT = [torch.zeros_like(a) for a in s0]
            gT[0][0].fill_(1.0 / sc.n_particles)   # L = centroid x of the final state
            sT, g0, g_act = sim.rollout(s0, act, req.T, self.ckpt_k, tuple(gT))
            ev = torch.cuda.Event()
            ev.record(stream)
        keep = (sT, g0, g_act, s0, act, gT)
        return _Slot(res, sim, stream, ev, keep, nbytes)

    def _finish(self, sl: _Slot, t0: float):
        res = sl.res
        res.done = time.perf_counter() - t0
        try:
            sl.sim.sync_errors()
            if self.keep_results:
                res.xT = sl.keep[0][0].clone()
                res.g_v0 = sl.keep[1][1].clone()
                res.g_act = None if sl.keep[2] is None else sl.keep[2].clone()
        except MPMError as e:
            res.error = e.code
        sl.sim.close()

    def run(self, requests: List[S.Request], fifo: bool = False) -> List[Result]:
        """Serve `requests` (arrival times in seconds from the start) in real
        time; returns one Result per request, in request order."""
        results = [Result(i, r.arrival, particles=r.scene.n_particles, substeps=r.T)
                   for i, r in enumerate(requests)]
        pending = collections.deque(sorted(range(len(requests)),
                                           key=lambda i: requests[i].arrival))
        active: List[_Slot] = []
        free_streams = list(self.streams)
        used = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        slots = 1 if fifo else self.max_slots
        while pending or active:
            now = time.perf_counter() - t0
            progressed = False
            for sl in list(active):
                if sl.event.query():
                    self._finish(sl, t0)
                    active.remove(sl)
                    free_streams.append(sl.stream)
                    used -= sl.nbytes
                    progressed = True
            while pending and requests[pending[0]].arrival <= now and len(active) < slots:
                i = pending[0]
                nb = footprint_bytes(requests[i].scene, requests[i].T, self.ckpt_k)
                if active and used + nb > self.budget:
                    break
                pending.popleft()
                res = results[i]
                res.start = time.perf_counter() - t0
                stream = free_streams.pop()
                try:
                    sl = self._launch(i, requests[i], res, stream)
                except MPMError as e:
                    res.error = e.code
                    res.done = time.perf_counter() - t0
                    free_streams.append(stream)
                    continue
                active.append(sl)
                used += sl.nbytes
                self.peak_bytes = max(self.peak_bytes, used)
                progressed = True
            if not progressed:
                nxt = requests[pending[0]].arrival - now if pending else self.poll_s
                time.sleep(max(0.0, min(self.poll_s, nxt)))
        return results


def summarize(results: List[Result], wall: Optional[float] = None) -> dict:
    ok = [r for r in results if r.error is None]
    lat = sorted(r.latency for r in ok)
    span = wall if wall is not None else (max(r.done for r in results) -
                                          min(r.arrival for r in results))

    def pct(q):
        if not lat:
            return None
        k = (len(lat) - 1) * q
        lo = int(k)
        hi = min(lo + 1, len(lat) - 1)
        return lat[lo] + (lat[hi] - lat[lo]) * (k - lo)

    pss = sum(r.particles * r.substeps for r in ok)
    return {"requests": len(results), "failed": len(results) - len(ok),
            "requests_per_s": len(ok) / span if span > 0 else None,
            "particle_substeps_per_s": pss / span if span > 0 else None,
            "latency_s": {"p50": pct(0.5), "p99": pct(0.99), "max": lat[-1] if lat else None},
            "span_s": span}
