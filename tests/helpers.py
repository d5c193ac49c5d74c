"""Test glue: converts generator scenes to oracle scenes and compares arrays.

Holds no simulation arithmetic."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1810_01054_amd import scenes as S


def oscene(sc: S.Scene, **over) -> oracle.Scene:
    p = sc.params()
    p.update(over)
    return oracle.Scene(**p)


def f64(state):
    return tuple(np.asarray(a, dtype=np.float64) for a in state)


def act_schedule_oracle(sc: S.Scene, T: int) -> np.ndarray:
    """Per-step actuation s[T][n_act] evaluated by the oracle's bank."""
    return oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase)


def rel_err(a, b) -> float:
    """Normwise relative error ||a - b|| / ||b|| (b is the reference)."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)
