"""Autotuner for libmpm's launch and tape options.

For a batch of scenes, `tune` times short forward + reverse rollouts under
each candidate launch configuration (binned scatter mode and tile edge,
persistent grid kernels, G2P fused with the next P2G or not in 3D, hipGraph
replay) and keeps the one
with the smallest median time over the repeats; `tune_checkpoint` then times
the candidate checkpoint intervals k on a longer probe with those options,
and `tune_rebin` whether re-binning at every checkpoint pays at that k.
Results are cached on disk, keyed by GPU architecture, dimension, grid sizes,
scene count and a particle-count bucket (and, for k, the rollout length), so
a configuration is measured once per shape class.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from .sim import Simulator

CACHE_PATH = os.environ.get(
    "MPM_AUTOTUNE_CACHE",
    os.path.join(os.path.expanduser("~"), ".cache", "mpm_mi355x", "autotune.json"))


def candidates(dim: int) -> List[dict]:
    """Binned-scatter variants (mode, tile edge; the sorted scatter also with
    persistent grid kernels and, in 3D, without the fused G2P + P2G kernel)
    x hipGraph replay."""
    base = ([{"scatter": 3, "tile": 8}, {"scatter": 3, "tile": 8, "persistent": True},
             {"scatter": 1, "tile": 8}, {"scatter": 1, "tile": 16}]
            if dim == 2 else
            [{"scatter": 3, "tile": 4}, {"scatter": 3, "tile": 4, "persistent": True},
             {"scatter": 3, "tile": 4, "fusion": 1},
             {"scatter": 1, "tile": 4}, {"scatter": 1, "tile": 8}])
    return [dict(c, graphs=g) for c in base for g in (False, True)]


def shape_key(scenes: Sequence[dict]) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] \
        if torch.cuda.is_available() else "cpu"
    dim = scenes[0]["dim"]
    grids = sorted({s["n_grid"] for s in scenes})
    N = sum(s["n_particles"] for s in scenes)
    bucket = int(round(math.log2(max(N, 1)) * 2))  # half-octave buckets
    return f"{arch}/d{dim}/n{'-'.join(map(str, grids))}/s{len(scenes)}/N{bucket}"


def _load() -> Dict[str, dict]:
    try:
        with open(CACHE_PATH) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache: Dict[str, dict]):
    os.makedirs(os.path.dirname(CACHE_PATH), exist_ok=True)
    tmp = CACHE_PATH + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE_PATH)


def best_k(T: int) -> int:
    """Checkpoint interval minimising the tape's state slots (T/k + k)."""
    return max(1, int(round(math.sqrt(max(T, 1)))))


def _median_time(sim, state, act, T, k, gT, repeats):
    sim.rollout(state, act, T, k, gT)          # warm-up / capture
    torch.cuda.synchronize()
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        sim.rollout(state, act, T, k, gT)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    sim.sync_errors()
    return float(np.median(ts))


def tune(scenes: Sequence[dict], act_id: np.ndarray, state, act: Optional[torch.Tensor],
         T_probe: int = 16, repeats: int = 3, use_cache: bool = True) -> dict:
    """Fastest option set (Simulator keyword arguments) for this batch: the
    smallest median time of `repeats` fwd + bwd rollouts of T_probe substeps."""
    key = shape_key(scenes)
    cache = _load() if use_cache else {}
    if key in cache:
        return dict(cache[key]["opts"])
    dim = scenes[0]["dim"]
    act_p = None if act is None else act[:T_probe].contiguous()
    timings = []
    for opts in candidates(dim):
        try:
            sim = Simulator(scenes, act_id=act_id, **opts)
        except Exception:
            continue
        gT = tuple(torch.zeros_like(s) for s in state)
        timings.append((_median_time(sim, state, act_p, T_probe, 8, gT, repeats), opts))
        sim.close()
    timings.sort(key=lambda t: t[0])
    best = timings[0][1]
    if use_cache:
        cache[key] = {"opts": best, "ms": [round(t * 1e3, 3) for t, _ in timings],
                      "candidates": [o for _, o in timings]}
        _store(cache)
    return dict(best)


def tune_checkpoint(scenes: Sequence[dict], act_id: np.ndarray, state,
                    act: Optional[torch.Tensor], T: int, opts: dict,
                    ks: Sequence[int] = (8, 16, 32, 64), T_probe: int = 128,
                    repeats: int = 3, use_cache: bool = True) -> int:
    """Checkpoint interval for rollouts of T substeps: the candidate k
    (k <= T) with the smallest median time of fwd + bwd rollouts of
    min(T, T_probe) substeps under the options `opts`."""
    key = f"{shape_key(scenes)}/T{T}/k"
    cache = _load() if use_cache else {}
    if key in cache:
        return int(cache[key]["k"])
    Tp = min(T, T_probe)
    act_p = None if act is None else act[:Tp].contiguous()
    sim = Simulator(scenes, act_id=act_id, **opts)
    gT = tuple(torch.zeros_like(s) for s in state)
    timings = [(_median_time(sim, state, act_p, Tp, k, gT, repeats), k)
               for k in ks if k <= Tp] or [(0.0, best_k(T))]
    sim.close()
    timings.sort()
    k = int(timings[0][1])
    if use_cache:
        cache[key] = {"k": k, "ms": [round(t * 1e3, 3) for t, _ in timings],
                      "candidates": [kk for _, kk in timings]}
        _store(cache)
    return k


def tune_rebin(scenes: Sequence[dict], act_id: np.ndarray, state,
               act: Optional[torch.Tensor], T: int, k: int, opts: dict,
               T_probe: int = 512, repeats: int = 3, use_cache: bool = True) -> bool:
    """Whether to sort the particles into tiles again at every checkpoint
    (pays when they travel more than a cell per segment, which shows only
    late in a rollout: the probe is min(T, T_probe) substeps long)."""
    if k <= 0 or k >= T:
        return False
    key = f"{shape_key(scenes)}/T{T}/k{k}/rebin"
    cache = _load() if use_cache else {}
    if key in cache:
        return bool(cache[key]["rebin"])
    Tp = min(T, T_probe)
    act_p = None if act is None else act[:Tp].contiguous()
    gT = tuple(torch.zeros_like(s) for s in state)
    timings = []
    for rebin in (False, True):
        sim = Simulator(scenes, act_id=act_id, **dict(opts, rebin=rebin))
        timings.append((_median_time(sim, state, act_p, Tp, k, gT, repeats), rebin))
        sim.close()
    best = min(timings)[1]
    if use_cache:
        cache[key] = {"rebin": best, "ms": [round(t * 1e3, 3) for t, _ in timings]}
        _store(cache)
    return best
