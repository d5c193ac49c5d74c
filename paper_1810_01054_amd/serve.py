"""Request loop for forward + gradient rollout requests, with continuous
batching.

Each request is one scene (2D or 3D), a number of substeps T and its
actuation parameters; serving it means a forward rollout and the reverse
pass (final state, adjoint of the initial state, actuation gradient).

Scheduling: `lanes` batch lanes, each with its own HIP stream and host
thread.  Whenever a lane is free it admits the requests that have arrived
and are waiting: the oldest one and, in arrival order, every other waiting
request of the same dimension, up to `max_batch` requests and the
device-memory budget.  The admitted requests become ONE multi-scene libmpm
context: every kernel of a substep covers all of them in one launch, each
scene held fixed past its own T (per-scene horizons), in one rollout of the
largest T with its reverse pass.  A request that arrives while batches are
running joins the next batch a lane admits, and the lanes' batches overlap on
the device.  Completion is detected with a stream event; latency is measured
from arrival to completion.  If a batch fails (a request left the grid or
inverted), its requests are served again one by one, so a poisoned request
fails alone.  ``fifo=True`` replays the plain one-at-a-time loop (one lane,
batches of one).

Marshalling and scheduling only: the simulation runs in the library.
"""
from __future__ import annotations

import math
import threading
import time
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence

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
    batch: int = 0          # requests in the batch that served it
    xT: Optional[torch.Tensor] = None
    g_v0: Optional[torch.Tensor] = None
    g_act: Optional[torch.Tensor] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def footprint_bytes(scene: S.Scene, T: int, ckpt_k: int, tile: Optional[int] = None) -> int:
    """Upper estimate of the device memory one request holds: its share of a
    context's grids, tile boxes and binning arrays, of the tape
    (checkpoints, segment states, per-substep grids), and its own tensors."""
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
    tape = ((ncp + (3 * k if ckpt_k > 0 else 0) + 4) * state
            + T * (1 + d) * G * 4
            + T * max(scene.n_act, 1) * 12)
    own = 5 * state + T * max(scene.n_act, 1) * 8
    return int(1.1 * (ctx + tape + own)) + (8 << 20)


def centroid_seed(sc: S.Scene) -> List[np.ndarray]:
    """dL/dS^T of L = mean_p x_{p,0}^T (centroid x of the final state)."""
    d, N = sc.dim, sc.n_particles
    g = [np.zeros((d, N), np.float32), np.zeros((d, N), np.float32),
         np.zeros((d * d, N), np.float32), np.zeros((d * d, N), np.float32)]
    g[0][0] = 1.0 / N
    return g


class Server:
    """Continuous batching of rollout requests over `lanes` concurrent
    batch lanes (see the module docstring)."""

    def __init__(self, max_batch: int = 16, lanes: int = 2, hbm_budget: Optional[int] = None,
                 ckpt_k: int = 32, keep_results: bool = False, poll_s: float = 2e-4,
                 deterministic: bool = False,
                 seed_of: Callable[[S.Scene], Sequence[np.ndarray]] = centroid_seed):
        self.max_batch = max_batch
        self.lanes = lanes
        if hbm_budget is None:
            free, total = torch.cuda.mem_get_info()
            hbm_budget = int(0.6 * free)
        self.budget = hbm_budget
        self.ckpt_k = ckpt_k
        self.keep_results = keep_results
        self.poll_s = poll_s
        self.deterministic = deterministic
        self.seed_of = seed_of
        self.peak_bytes = 0
        self.batches: List[List[int]] = []

    # -- one batch on one lane -----------------------------------------------
    def _serve(self, reqs: List[S.Request], idx: List[int], results: List[Result],
               stream, t0: float):
        """One multi-scene rollout (forward + reverse) of requests `idx`;
        raises MPMError if the batch fails."""
        scs = [reqs[i].scene for i in idx]
        Ts = [reqs[i].T for i in idx]
        T = max(Ts)
        dev = torch.device("cuda")
        with torch.cuda.stream(stream):
            t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(dev)
            sim = Simulator([sc.params() for sc in scs],
                            act_id=np.concatenate([sc.act_id for sc in scs]),
                            stream=stream, deterministic=self.deterministic)
            try:
                sim.set_horizons(Ts)
                s0 = tuple(t(np.concatenate([sc.state[c] for sc in scs], axis=1))
                           for c in range(4))
                acts = [act_bank_forward(T, sc.dt, t(sc.freq), t(sc.amp), t(sc.phase),
                                         stream=stream) for sc in scs if sc.n_act > 0]
                act = torch.cat(acts, dim=1).contiguous() if acts else None
                seeds = [self.seed_of(sc) for sc in scs]
                gT = tuple(t(np.concatenate([np.asarray(g[c], np.float32) for g in seeds],
                                            axis=1)) for c in range(4))
                sT, g0, g_act = sim.rollout(s0, act, T, self.ckpt_k, gT)
                ev = torch.cuda.Event()
                ev.record(stream)
                ev.synchronize()
                sim.sync_errors()
                done = time.perf_counter() - t0
                off = aoff = 0
                for i, sc in zip(idx, scs):
                    r = results[i]
                    r.done = done
                    r.batch = len(idx)
                    N, na = sc.n_particles, sc.n_act
                    if self.keep_results:
                        r.xT = sT[0][:, off:off + N].clone()
                        r.g_v0 = g0[1][:, off:off + N].clone()
                        r.g_act = (None if g_act is None else
                                   g_act[:reqs[i].T, aoff:aoff + na].clone())
                    off += N
                    aoff += na
            finally:
                sim.close()

    def _lane(self, reqs, results, pending, lock, stream, t0, fifo, state):
        while True:
            with lock:
                if not pending:
                    return
                now = time.perf_counter() - t0
                head = pending[0]
                if reqs[head].arrival > now:
                    wait = reqs[head].arrival - now
                    idx = None
                else:
                    # the oldest waiting request, then in arrival order the
                    # waiting requests of its dimension that fit the budget
                    dim = reqs[head].scene.dim
                    idx, nb = [], 0
                    for i in list(pending):
                        if reqs[i].arrival > now or len(idx) >= (1 if fifo else self.max_batch):
                            break
                        if reqs[i].scene.dim != dim:
                            continue
                        fb = footprint_bytes(reqs[i].scene, reqs[i].T, self.ckpt_k)
                        # a request larger than the whole budget still runs,
                        # alone, once nothing else holds memory
                        if state["used"] + nb + fb > self.budget and (idx or state["used"] > 0):
                            break
                        idx.append(i)
                        nb += fb
                    if not idx:
                        # the oldest request waits for memory to free up
                        idx, wait = None, self.poll_s
                    else:
                        for i in idx:
                            pending.remove(i)
                        state["used"] += nb
                        state["active"] += 1
                        self.peak_bytes = max(self.peak_bytes, state["used"])
                        self.batches.append(list(idx))
            if idx is None:
                time.sleep(max(0.0, min(self.poll_s, wait)))
                continue
            start = time.perf_counter() - t0
            for i in idx:
                results[i].start = start
            try:
                self._serve(reqs, idx, results, stream, t0)
            except MPMError:
                # isolate the failing request(s): serve the batch one by one
                for i in idx:
                    try:
                        self._serve(reqs, [i], results, stream, t0)
                    except MPMError as e:
                        results[i].error = e.code
                        results[i].done = time.perf_counter() - t0
            with lock:
                state["used"] -= nb
                state["active"] -= 1

    def run(self, requests: List[S.Request], fifo: bool = False) -> List[Result]:
        """Serve `requests` (arrival times in seconds from the start) in real
        time; returns one Result per request, in request order."""
        results = [Result(i, r.arrival, particles=r.scene.n_particles, substeps=r.T)
                   for i, r in enumerate(requests)]
        pending = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
        lock = threading.Lock()
        state = {"used": 0, "active": 0}
        lanes = 1 if fifo else self.lanes
        streams = [torch.cuda.Stream() for _ in range(lanes)]
        self.batches = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        threads = [threading.Thread(target=self._lane,
                                    args=(requests, results, pending, lock, streams[k], t0,
                                          fifo, state))
                   for k in range(lanes)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        torch.cuda.synchronize()
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
    sizes = [r.batch for r in ok if r.batch]
    return {"requests": len(results), "failed": len(results) - len(ok),
            "requests_per_s": len(ok) / span if span > 0 else None,
            "particle_substeps_per_s": pss / span if span > 0 else None,
            "latency_s": {"p50": pct(0.5), "p99": pct(0.99), "max": lat[-1] if lat else None},
            "mean_batch": float(np.mean(sizes)) if sizes else None,
            "span_s": span}
