"""Autotuner for libmpm's launch and tape options.

For a batch of scenes it times short forward + reverse rollouts under each
candidate configuration (binned scatter mode, tile edge, hipGraph replay,
checkpoint interval) and keeps the fastest.  Results are cached on disk,
keyed by GPU architecture, dimension, grid sizes and a particle-count
bucket, so a configuration is measured once per shape class.
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
    """Binned-scatter variants (mode, tile edge) x hipGraph replay."""
    base = ([{"scatter": 3, "tile": 8}, {"scatter": 1, "tile": 8}, {"scatter": 1, "tile": 16}]
            if dim == 2 else
            [{"scatter": 3, "tile": 4}, {"scatter": 1, "tile": 4}, {"scatter": 1, "tile": 8}])
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


def tune(scenes: Sequence[dict], act_id: np.ndarray, state, act: Optional[torch.Tensor],
         T_probe: int = 16, repeats: int = 2, use_cache: bool = True) -> dict:
    """Fastest option set (Simulator keyword arguments) for this batch."""
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
        sim.rollout(state, act_p, T_probe, 8, gT)          # warm-up / capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            sim.rollout(state, act_p, T_probe, 8, gT)
        torch.cuda.synchronize()
        timings.append(((time.perf_counter() - t0) / repeats, opts))
        sim.sync_errors()
        sim.close()
    timings.sort(key=lambda t: t[0])
    best = timings[0][1]
    if use_cache:
        cache[key] = {"opts": best, "ms": [round(t * 1e3, 3) for t, _ in timings],
                      "candidates": [o for _, o in timings]}
        _store(cache)
    return dict(best)
