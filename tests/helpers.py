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


def max_err(a, b, scale=None) -> float:
    """Largest per-element error max_i |a_i - b_i| / scale.  The scale
    defaults to the reference's largest magnitude max_i |b_i| (the field's own
    size), so one wrong element shows at its own size instead of being
    averaged over the array as in the normwise error; absolute error when the
    reference is zero."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    if a.shape != b.shape:
        raise ValueError(f"shape mismatch {a.shape} vs {b.shape}")
    if a.size == 0:
        return 0.0
    if not np.isfinite(a).all():
        return float("inf")
    if scale is None:
        scale = float(np.abs(b).max())
    if scale == 0.0:
        return float(np.abs(a - b).max())
    return float(np.abs(a - b).max() / scale)


def err(a, b) -> float:
    """The larger of the normwise relative error and the per-element error
    relative to the field's largest magnitude: a parity bound on err holds
    for the array as a whole and for every element of it."""
    return max(rel_err(a, b), max_err(a, b))


def dx_err(x, ref, dx: float) -> float:
    """Largest position error of any particle component in grid cells."""
    return max_err(x, ref, scale=dx)
