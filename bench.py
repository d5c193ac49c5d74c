#!/usr/bin/env python3
"""Throughput of differentiable MLS-MPM rollouts on one MI355X.

A step is one whole forward + backward rollout of the 3D quadruped scene
(64^3 grid, 504,064 particles, 16 actuators driven by a sinusoid bank,
512 substeps, checkpoint every 32 substeps with recompute) through
torch.autograd: actuation bank (HIP) -> MPM rollout (HIP, C ABI) ->
loss = centroid x of the final state -> backward (HIP, C ABI).  Inputs are
resident in HBM before the timed region.

Prints one JSON line.  Besides the throughput it reports the roofline of the
dominant kernel (HIP events on the library's stream, algorithmic bytes per
particle) and the FP64 oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def kernel_bytes_per_particle(kernel: str, d: int) -> int:
    """Algorithmic HBM bytes per particle of one launch (FP32 state streams
    read and written once; grid, bins and checkpoints excluded)."""
    v, m = 4 * d, 4 * d * d          # one vector / one matrix per particle
    state = 2 * v + 2 * m            # x, v, C, F
    return {
        "p2g": state + 4,                          # state + act id
        "g2p": (v + m) + state,                    # x, F in; state out
        "adj_scatter": (v + m) + state,            # x, F, adjoint in
        "adj_gather": state + m + state + 4 + state,  # S^n, C^{n+1}, adj in, id; adj out
    }[kernel]


def kernel_bytes_per_node(kernel: str, d: int) -> int:
    """Algorithmic bytes per grid node of the grid kernels."""
    return {"grid": 4 + 4 * d + 4 * d,                  # m, p in; v out
            "adj_grid": 4 + 4 * d + 4 * d + 4 * d + 4 + 4 * d}[kernel]  # m, p, vbar in; pbar, mbar, v out


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(sc, T_sample: int):
    """The FP64 oracle (single-threaded C) on the first T_sample substeps of
    the same scene, forward + memo reverse pass."""
    import numpy as np
    import oracle
    p = sc.params()
    os_ = oracle.Scene(**p)
    acts = oracle.act_bank_fwd(T_sample, sc.dt, sc.freq, sc.amp, sc.phase)
    st = tuple(np.asarray(a, np.float64) for a in sc.state)
    gT = [np.zeros_like(a) for a in st]
    gT[0][0] = 1.0 / sc.n_particles
    t0 = time.perf_counter()
    oracle.rollout(os_, st, T_sample, sc.act_id, acts, gT)
    dt = time.perf_counter() - t0
    return {"value": sc.n_particles * T_sample / dt, "unit": "particle-substeps/s",
            "cores": 1, "kind": "oracle",
            "sample": f"{sc.name}: {sc.n_particles} particles, first {T_sample} "
                      f"substeps forward + reverse (memo), FP64, one thread, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--T", type=int, default=512, help="substeps per rollout")
    ap.add_argument("--ckpt", type=int, default=32,
                    help="checkpoint interval (0 = store every state)")
    ap.add_argument("--cpu-sample", type=int, default=2,
                    help="substeps of the oracle sample (0 = skip)")
    ap.add_argument("--scatter", type=int, default=0,
                    help="binned scatter mode: 0 default, 1 per-particle LDS atomics, "
                         "2 per-cell in bin order, 3 per-cell after an LDS sort")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the HIP-event kernel timing")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one MI355X only (one GPU per box); "
              "multi-GPU runs are not part of it", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1810_01054_amd import scenes as S
    from paper_1810_01054_amd.autograd import act_bank, rollout
    from paper_1810_01054_amd.sim import Simulator

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = "cuda:0"
    torch.cuda.set_device(0)

    sc = S.config_3()
    T, k = args.T, args.ckpt
    N, d = sc.n_particles, sc.dim
    sim = Simulator([sc.params()], act_id=sc.act_id, scatter=args.scatter)
    t = lambda a: torch.tensor(np.ascontiguousarray(a, np.float32), device=dev)
    x0, v0, C0, F0 = (t(a) for a in sc.state)
    v0.requires_grad_(True)
    freq = t(sc.freq)
    amp = t(sc.amp).requires_grad_(True)
    phase = t(sc.phase).requires_grad_(True)

    def one_step():
        act = act_bank(T, sc.dt, freq, amp, phase)
        xT, vT, CT, FT = rollout(sim, (x0, v0, C0, F0), act, T, k)
        loss = xT[0].mean()              # centroid x of the final state
        loss.backward()
        return loss

    # warm-up; the first warm-up step also finds the dominant kernel
    dominant = "adj_gather"
    warm_prof = None
    for w in range(max(args.warmup, 1)):
        if w == 0 and not args.no_profile:
            sim.profile(["p2g", "grid", "g2p", "adj_scatter", "adj_grid", "adj_gather"])
        one_step()
        if w == 0 and not args.no_profile:
            prof = sim.profile_read()
            sim.profile([])
            dominant = max(prof, key=lambda kk: prof[kk][1])
            warm_prof = {kk: round(ms * 1e3 / max(n, 1), 2)
                         for kk, (n, ms) in prof.items() if n}
    sim.sync_errors()
    torch.cuda.synchronize()

    if not args.no_profile:
        sim.profile([dominant])
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record()
        one_step()
        ev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync_errors()
    lat = [a.elapsed_time(b) for a, b in ev]
    roof = None
    if not args.no_profile:
        prof = sim.profile_read()
        sim.profile([])
        n_launch, ms = prof[dominant]
        avg_s = ms / max(n_launch, 1) / 1e3
        if dominant in ("grid", "adj_grid"):
            bpu, units = kernel_bytes_per_node(dominant, d), sim.G
        else:
            bpu, units = kernel_bytes_per_particle(dominant, d), N
        achieved = bpu * units / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "kernel": dominant,
                "avg_launch_us": round(avg_s * 1e6, 2), "launches": n_launch,
                "bytes_per_unit": bpu, "units_per_launch": units}

    ms_per_step = wall / args.steps * 1e3
    value = N * T * args.steps / wall
    out = {
        "metric": "particle-substeps/s fwd+bwd, 3D 64³/500k; % HBM peak; p99 rollout latency",
        "value": round(value, 1),
        "unit": "particle-substeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{sc.name}: 3D quadruped, 64^3 grid, {N} particles, "
                               f"16 actuators, T={T} substeps fwd+bwd, checkpoint k={k} "
                               f"with recompute, torch.autograd.Function",
                   "particles": N, "grid": "64^3", "substeps": T, "ckpt_k": k,
                   "scatter_mode": args.scatter,
                   "global_batch": 1, "parallelism": "single GPU"},
        "pct_hbm_peak_672B_per_pss": round(672.0 * value / (HBM_PEAK_GBS * 1e9), 4),
        "rollout_latency_ms": {"p50": round(percentile(lat, 0.5), 3),
                               "p99": round(percentile(lat, 0.99), 3)},
        "roofline": roof,
        "kernel_avg_us": warm_prof,
        "cpu_baseline": None,
    }
    if args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
