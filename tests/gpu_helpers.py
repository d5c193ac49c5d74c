"""Shared glue for the GPU tests (marshalling and comparisons only)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_1810_01054_amd import scenes as S
from tests.helpers import oscene, f64, rel_err


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")


def say(*a):
    """Name the case before each GPU step (flushed, so a fault still shows it)."""
    print("[gpu]", *a, file=sys.stderr, flush=True)


def to_gpu(state):
    return tuple(torch.tensor(np.ascontiguousarray(a, np.float32), device="cuda")
                 for a in state)


def to_np(state):
    return tuple(t.detach().cpu().numpy().astype(np.float64) for t in state)


def sim_for(scs, **kw):
    from paper_1810_01054_amd.sim import Simulator
    if not isinstance(scs, (list, tuple)):
        scs = [scs]
    ids = np.concatenate([s.act_id for s in scs]) if scs else None
    return Simulator([s.params() for s in scs], act_id=ids, **kw)


def concat_state(scs):
    return tuple(np.concatenate([s.state[k] for s in scs], axis=1) for k in range(4))


def gpu_act_bank(sc, T):
    """Per-step actuation from the library's own bank kernel."""
    from paper_1810_01054_amd.sim import act_bank_forward
    t = lambda a: torch.tensor(np.ascontiguousarray(a, np.float32), device="cuda")
    return act_bank_forward(T, sc.dt, t(sc.freq), t(sc.amp), t(sc.phase))


def seeds(shape_state, seed):
    rng = np.random.default_rng(seed)
    return tuple(rng.normal(size=a.shape) for a in shape_state)
