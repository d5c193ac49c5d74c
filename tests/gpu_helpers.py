"""Shared glue for the GPU tests (marshalling and comparisons only)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_1810_01054_amd import scenes as S
from tests.helpers import oscene, f64, err, max_err


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


# Final state of a rollout (up to ~100 substeps) against the oracle: bound on
# err() per field (normwise and per element, relative to the field's largest
# magnitude) and on the largest position error in grid cells.  Positions
# follow the required bound (1e-5 after 100 substeps).  The FP32 velocity
# and affine matrix come out of 3^d-node weighted sums of grid velocities
# (v_i = p_i / m_i with cancellation in p_i), and C' = (4/dx^2) sum N v_i
# (x_i - x_p) differences node velocities across a cell: each substep's
# rounding of v and C is ~1e-6 and ~1e-5 of their size, and it is not
# damped from one substep to the next; F' = (I + dt C') F carries dt times
# C's error into F every substep: over T dt = 0.01 (100 substeps) with |C|
# up to tens per second in contact and C within 1e-3 of its largest
# magnitude per element, F's per-element error can reach
# 0.01 * 1e-3 * 10 = 1e-4 of |F| (normwise it stays near 1e-6).
STATE_TOL = {"x": 1e-5, "v": 1e-4, "C": 1e-3, "F": 1e-4}
X_DX_TOL = 1e-3


def state_errs(got, ref, dx):
    e = {k: err(a, b) for k, a, b in zip("xvCF", got, ref)}
    e["x_dx"] = max_err(got[0], ref[0], scale=dx)
    return e


def check_state(got, ref, dx, label="", tol=None, x_dx=None):
    """Assert the final state `got` (x, v, C, F) against the oracle's."""
    tol = dict(STATE_TOL, **(tol or {}))
    x_dx = X_DX_TOL if x_dx is None else x_dx
    e = state_errs(got, ref, dx)
    say("state", label, {k: f"{v:.2e}" for k, v in e.items()})
    for k in "xvCF":
        assert e[k] < tol[k], (label, k, e[k], tol[k])
    assert e["x_dx"] < x_dx, (label, "x in cells", e["x_dx"], x_dx)
    return e
