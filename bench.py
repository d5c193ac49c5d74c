#!/usr/bin/env python3
"""Throughput of differentiable MLS-MPM rollouts on one MI355X.

A step is one whole forward + backward rollout of the 3D quadruped scene
(64^3 grid, 504,064 particles, 16 actuators driven by a sinusoid bank,
512 substeps, checkpoint every 32 substeps with recompute) through
torch.autograd: actuation bank (HIP) -> MPM rollout (HIP, C ABI) ->
loss = centroid x of the final state -> backward (HIP, C ABI).  Inputs are
resident in HBM before the timed region.

``--workload c3ctrl`` runs the same scene with its actuation from a
closed-loop controller (mpm_rollout_ctrl); c4, c5 and copy are the batched,
serving and byte-counter calibration workloads.

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
        "adj_gather": state + state + 4 + state,   # S^n, adj in, id; adj out
        # x, F, id in; x, F out (v and C too on checkpoint substeps)
        "g2p_p2g": (v + m) + 4 + (v + m),
        # state n, adjoint of n+1, id, x and F of n-1 in; adjoint of n out
        "adj_fused": state + state + 4 + (v + m) + state,
    }[kernel]


def stage_bytes_per_particle(kernel: str, d: int):
    """Algorithmic bytes per particle of the method stage a kernel carries
    out, as the hot-path byte model counts them (each stage reads and writes
    its particle streams once): a forward substep S^n -> S^{n+1} reads and
    writes the state (2 x 48 B in 3D), the recompute does the same, and a
    reverse substep reads S^n and the adjoint of S^{n+1} and writes the
    adjoint of S^n (3 x 48 B); 672 B per particle-substep in 3D.  None for
    kernels that carry only part of a stage (their realised bytes are
    reported instead)."""
    state = 4 * (2 * d + 2 * d * d)
    return {"g2p_p2g": 2 * state,           # forward substep (fused G2P + P2G)
            "g2p": 2 * state,               # recompute of one substep
            "adj_gather": 3 * state,        # reverse substep's particle streams
            "adj_fused": 3 * state}.get(kernel)


def kernel_bytes_per_node(kernel: str, d: int) -> int:
    """Algorithmic bytes per grid node of the grid kernels."""
    return {"grid": 4 + 4 * d + 4 * d,                  # m, p in; v out
            "adj_grid": 4 + 4 * d + 4 * d + 4 * d + 4 + 4 * d}[kernel]  # m, p, vbar in; pbar, mbar, v out


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "c3_hbm_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1810_01054_amd", "csrc", f)
                  for f in ("mpm_kernels.hip", "mpm_internal.h")]


def kernels_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel: str):
    """Measured HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE
    counters, scaled by the same counters' reading on a plain copy of known
    size) from the committed counter summary; None when there is none or the
    kernel sources changed since the counters were taken."""
    import re
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"kernel sources sha256: `([0-9a-f]{64})`", text)
    if not m or m.group(1) != kernels_sha256():
        return None
    m = re.search(r"^\| k_%s\S* \|(?:[^|]*\|){3} *([0-9.]+) *\|" % re.escape(kernel), text, re.M)
    return float(m.group(1)) if m else None


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def _oracle_sample(sc, T_sample: int) -> float:
    """One oracle run: the first T_sample substeps of the scene forward, then
    the memo reverse pass; returns its wall time in seconds."""
    import numpy as np
    import oracle
    os_ = oracle.Scene(**sc.params())
    acts = oracle.act_bank_fwd(T_sample, sc.dt, sc.freq, sc.amp, sc.phase)
    st = tuple(np.asarray(a, np.float64) for a in sc.state)
    gT = [np.zeros_like(a) for a in st]
    gT[0][0] = 1.0 / sc.n_particles
    t0 = time.perf_counter()
    oracle.rollout(os_, st, T_sample, sc.act_id, acts, gT)
    return time.perf_counter() - t0


def _oracle_worker(core, sc, T_sample, start, q):
    os.sched_setaffinity(0, {core})
    start.wait()
    q.put(_oracle_sample(sc, T_sample))


def cpu_baseline(sc, T_one: int, T_all: int):
    """The FP64 oracle (single-threaded C, as it stands) on a bounded sample
    of the same scene: first on one pinned core (T_one substeps forward +
    memo reverse), then one copy per available host core, each pinned to its
    own core and running the first T_all substeps (aggregate throughput of
    all cores).  Runs before the GPU is touched (forked workers)."""
    import multiprocessing as mp
    import oracle
    oracle.lib()
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    affinity = sorted(os.sched_getaffinity(0))
    try:
        os.sched_setaffinity(0, {affinity[0]})
        dt1 = _oracle_sample(sc, T_one)
    finally:
        os.sched_setaffinity(0, set(affinity))
    one = sc.n_particles * T_one / dt1
    ctx = mp.get_context("fork")
    q, start = ctx.Queue(), ctx.Event()
    procs = [ctx.Process(target=_oracle_worker, args=(c, sc, T_all, start, q))
             for c in affinity]
    for pr in procs:
        pr.start()
    t0 = time.perf_counter()
    start.set()
    times = [q.get() for _ in procs]
    wall = time.perf_counter() - t0
    for pr in procs:
        pr.join()
    allc = len(procs) * sc.n_particles * T_all / wall
    return {"value": round(allc, 1), "unit": "particle-substeps/s",
            "cores": len(procs), "kind": "oracle",
            "sample": f"{sc.name}: {sc.n_particles} particles, first {T_all} substeps "
                      f"forward + reverse (memo), FP64; one copy per host core "
                      f"({len(procs)} single-threaded processes, each pinned to its "
                      f"own core), {wall:.1f} s wall (slowest copy {max(times):.1f} s)",
            "one_core": {"value": round(one, 1), "cores": 1,
                         "sample": f"first {T_one} substeps forward + reverse (memo), "
                                   f"one thread pinned to one core, {dt1:.1f} s"},
            "cpu_model": model, "host_cores_available": len(affinity)}


def run_copy(args):
    """Calibration workload for the HBM byte counters: an elementwise copy
    (x 1.0) of --copy-mib MiB, device to device; reads and writes exactly
    that many bytes per launch."""
    import torch
    n = args.copy_mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(max(args.warmup, 1)):
        torch.mul(src, 1.0, out=dst)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(args.steps):
        torch.mul(src, 1.0, out=dst)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) / 1e3 / args.steps
    nbytes = 2 * n * 4
    print(json.dumps({"metric": "device copy bandwidth (read + write)",
                      "value": round(nbytes / sec / 1e9, 1), "unit": "GB/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f32",
                      "data": "synthetic",
                      "config": {"workload": f"elementwise copy of {args.copy_mib} MiB",
                                 "bytes_read": n * 4, "bytes_written": n * 4}}), flush=True)


def run_batched(args):
    """64 uneven 2D scenes (N log-uniform in [2k, 60k], grids 64^2..256^2) in
    one context: every kernel of a substep covers all scenes in one launch.
    Compared with the same kernels run one scene at a time."""
    import numpy as np
    import torch

    from paper_1810_01054_amd import scenes as S
    from paper_1810_01054_amd.autograd import rollout
    from paper_1810_01054_amd.sim import Simulator, act_bank_forward

    dev = "cuda:0"
    scs = S.config_4()
    T, k = args.T if args.T != 512 else 200, args.ckpt
    t = lambda a: torch.tensor(np.ascontiguousarray(a, np.float32), device=dev)

    def acts_of(group):
        return torch.cat([act_bank_forward(T, s.dt, t(s.freq), t(s.amp), t(s.phase))
                          for s in group], dim=1).contiguous()

    def state_of(group):
        return tuple(t(np.concatenate([s.state[c] for s in group], axis=1)) for c in range(4))

    def seed_of(group):
        # L = sum over scenes of the centroid x of the final state
        g = [np.zeros((2, sum(s.n_particles for s in group)), np.float32),
             None, None, None]
        off = 0
        for s in group:
            g[0][0, off:off + s.n_particles] = 1.0 / s.n_particles
            off += s.n_particles
        n = g[0].shape[1]
        return (t(g[0]), torch.zeros(2, n, device=dev), torch.zeros(4, n, device=dev),
                torch.zeros(4, n, device=dev))

    def make(group, **opts):
        ids = np.concatenate([s.act_id for s in group])
        sim = Simulator([s.params() for s in group], act_id=ids, **opts)
        return sim, state_of(group), acts_of(group), seed_of(group)

    def run(setups, steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for sim, s0, act, gT in setups:
                sim.rollout(s0, act, T, k, gT)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    from paper_1810_01054_amd.autotune import tune, tune_checkpoint, tune_rebin
    N = sum(s.n_particles for s in scs)
    ids = np.concatenate([s.act_id for s in scs])
    tuned = tune([s.params() for s in scs], ids, state_of(scs), acts_of(scs), use_cache=False)
    # the checkpoint interval too, unless one was given
    if args.ckpt_given is None:
        k = tune_checkpoint([s.params() for s in scs], ids, state_of(scs), acts_of(scs), T,
                            tuned, use_cache=False)
    tuned["rebin"] = tune_rebin([s.params() for s in scs], ids, state_of(scs), acts_of(scs),
                                T, k, tuned, use_cache=False)
    batched = [make(scs, **tuned)]
    run(batched, 1)
    wb = run(batched, args.steps)
    batched[0][0].sync_errors()
    eager = [make(scs, **dict(tuned, graphs=False))]
    run(eager, 1)
    we = run(eager, args.steps)
    eager[0][0].sync_errors()
    del eager
    loop = [make([s]) for s in scs]
    run(loop, 1)
    wl = run(loop, args.steps)
    for sim, *_ in loop:
        sim.sync_errors()
    vb = N * T * args.steps / wb
    ve = N * T * args.steps / we
    vl = N * T * args.steps / wl
    out = {"metric": "particle-substeps/s fwd+bwd, 64 batched 2D scenes",
           "value": round(vb, 1), "unit": "particle-substeps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": round(wb / args.steps * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"64 2D scenes, {N} particles in total, grids "
                                  f"{sorted(set(s.n_grid for s in scs))}, T={T} fwd+bwd, "
                                  f"checkpoint k={k}, one launch per kernel per substep, "
                                  f"autotuned options",
                      "scenes": len(scs), "particles": N, "substeps": T, "ckpt_k": k,
                      "autotuned": tuned},
           "batched_without_graphs": {"value": round(ve, 1),
                                      "ms_per_step": round(we / args.steps * 1e3, 3)},
           "per_scene_loop": {"value": round(vl, 1), "ms_per_step": round(wl / args.steps * 1e3, 3)},
           "speedup_vs_per_scene_loop": round(vb / vl, 3)}
    print(json.dumps(out), flush=True)


def run_c2(args):
    """C2: 2D 256^2, six soft-robot blocks (98,304 particles, 48 actuators
    with sinusoid banks), T = 1,000 substeps forward + reverse with a
    checkpoint every 64; loss = centroid x of the final state.  Its blocks
    travel several cells, so most particles leave their tile box's slack in
    the second half of the rollout; by default the particles are sorted into
    tiles again at every checkpoint (``--rebin 0``: once per rollout)."""
    import numpy as np
    import torch

    from paper_1810_01054_amd import scenes as S
    from paper_1810_01054_amd.sim import Simulator, act_bank_forward

    sc = S.config_2()
    rebin = int(args.rebin if args.rebin is not None else 1)
    T = args.T if args.T != 512 else 1000
    k = args.ckpt_given if args.ckpt_given is not None else 64
    dev = "cuda:0"
    t = lambda a: torch.tensor(np.ascontiguousarray(a, np.float32), device=dev)
    sim = Simulator([sc.params()], act_id=sc.act_id, fusion=args.fusion, rebin=rebin)
    s0 = tuple(t(a) for a in sc.state)
    act = act_bank_forward(T, sc.dt, t(sc.freq), t(sc.amp), t(sc.phase))
    N = sc.n_particles
    gT = [torch.zeros_like(a) for a in s0]
    gT[0][0].fill_(1.0 / N)
    gT = tuple(gT)
    for _ in range(max(args.warmup, 1)):
        sim.rollout(s0, act, T, k, gT)
    sim.sync_errors()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sim.rollout(s0, act, T, k, gT)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync_errors()
    value = N * T * args.steps / wall
    print(json.dumps({"metric": "particle-substeps/s fwd+bwd, 2D 256^2/98k", "value": round(value, 1),
                      "unit": "particle-substeps/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 3),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": "f32", "data": "synthetic",
                      "config": {"workload": f"c2_2d256_98k: 6 blocks, {N} particles, "
                                             f"T={T} fwd+bwd, checkpoint k={k}"
                                             + (", re-binned at every checkpoint"
                                                if rebin else ""),
                                 "particles": N, "substeps": T, "ckpt_k": k,
                                 "rebin": rebin}}), flush=True)


def run_serving(args):
    """Poisson arrivals of forward+gradient rollout requests (half 2D, half
    3D) served with continuous batching (waiting requests of one dimension
    share one multi-scene context per lane, each held fixed past its own T)
    and, on the same trace, by the plain one-at-a-time loop.  The arrival
    rate is swept at fractions of the plain loop's measured capacity plus one
    overload point."""
    import torch

    from paper_1810_01054_amd import scenes as S
    from paper_1810_01054_amd.serve import Server, summarize

    n_req = args.requests
    base = S.config_5(n_requests=n_req, rate=1.0, seed=1815)
    # warm-up: a burst of two full batches per lane through the batched
    # server (its multi-scene contexts grow the device memory pool to the
    # steady state), then a few requests through the plain loop
    warm = S.config_5(n_requests=2 * args.max_batch * args.lanes, rate=1.0, seed=1816)
    Server(max_batch=args.max_batch, lanes=args.lanes, ckpt_k=args.ckpt).run(
        [S.Request(0.0, r.scene, r.T) for r in warm])
    Server(ckpt_k=args.ckpt).run([S.Request(0.0, r.scene, r.T) for r in warm[:6]], fifo=True)
    burst = [S.Request(0.0, r.scene, r.T) for r in base]
    cap_res = Server(ckpt_k=args.ckpt).run(burst, fifo=True)
    cap = summarize(cap_res)["requests_per_s"]
    print(f"c5: plain-loop capacity {cap:.2f} requests/s", file=sys.stderr, flush=True)
    points = []
    for frac in (0.5, 0.8, 0.95, 1.5):
        rate = frac * cap
        reqs = [S.Request(r.arrival / rate, r.scene, r.T) for r in base]
        mix = summarize(Server(max_batch=args.max_batch, lanes=args.lanes,
                               ckpt_k=args.ckpt).run(reqs))
        print(f"c5: load {frac} batched p50 {mix['latency_s']['p50']:.3f} p99 "
              f"{mix['latency_s']['p99']:.3f} req/s {mix['requests_per_s']:.2f} "
              f"mean batch {mix['mean_batch']:.2f}", file=sys.stderr, flush=True)
        fifo = summarize(Server(ckpt_k=args.ckpt).run(reqs, fifo=True))
        print(f"c5: load {frac} fifo p50 {fifo['latency_s']['p50']:.3f} p99 "
              f"{fifo['latency_s']['p99']:.3f} req/s {fifo['requests_per_s']:.2f}",
              file=sys.stderr, flush=True)
        points.append({"load": frac, "rate_per_s": round(rate, 3), "batched": mix,
                       "fifo": fifo})
    top = points[2]["batched"]
    out = {"metric": "p99 rollout latency (serving, Poisson mix of 2D/3D fwd+grad requests)",
           "value": top["latency_s"]["p99"], "unit": "s", "n_gpus": 1, "steps": n_req,
           "warmup": len(warm), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{n_req} requests, half 2D (4k-100k particles, 64-256^2) "
                                  f"half 3D (50k-500k, 32-64^3), T 100-500, load 0.95 of "
                                  f"the plain loop's capacity", "max_batch": args.max_batch,
                      "lanes": args.lanes, "ckpt_k": args.ckpt},
           "plain_loop_capacity_req_per_s": round(cap, 3),
           "points": points}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--T", type=int, default=512, help="substeps per rollout")
    ap.add_argument("--ckpt", type=int, default=None,
                    help="checkpoint interval (0 = store every state; default 32, "
                         "autotuned for c4)")
    ap.add_argument("--cpu-sample", type=int, default=10,
                    help="substeps of the oracle sample (0 = skip)")
    ap.add_argument("--scatter", type=int, default=0,
                    help="binned scatter mode: 0 default, 1 per-particle LDS atomics, "
                         "2 per-cell in bin order, 3 per-cell after an LDS sort")
    ap.add_argument("--workload", default="c3",
                    choices=["c3", "c3ctrl", "c2", "c4", "c5", "copy"],
                    help="c3: 3D quadruped (headline); c2: 2D 256^2, 98k particles, "
                         "1,000 substeps; c3ctrl: the same quadruped, closed-loop "
                         "controller; c4: 64 batched 2D scenes; "
                         "c5: serving a Poisson request mix; copy: plain device copy "
                         "(calibrates the HBM byte counters)")
    ap.add_argument("--copy-mib", type=int, default=1024, help="copy: MiB per launch")
    ap.add_argument("--requests", type=int, default=60, help="c5: requests per load point")
    ap.add_argument("--max-batch", type=int, default=16,
                    help="c5: requests per batch (one multi-scene context)")
    ap.add_argument("--lanes", type=int, default=2, help="c5: concurrent batches")
    ap.add_argument("--friction", type=float, default=None,
                    help="c3/c3ctrl: walls with the friction projection and this "
                         "coefficient instead of sticky walls")
    ap.add_argument("--materials", action="store_true",
                    help="c3: a per-particle stiffness and density field (E, rho "
                         "x U[0.5, 1.5) / U[0.7, 1.3)) with their gradients")
    ap.add_argument("--fusion", type=int, default=0,
                    help="c3: 0 = G2P fused with the next P2G (default), 1 = every "
                         "kernel separate, 2 = also the reverse gather fused with the "
                         "previous adjoint scatter")
    ap.add_argument("--drift", type=float, default=0.0,
                    help="c3: add this x-velocity (domain units per second) to every "
                         "particle, so the body travels across cells and tiles during "
                         "the rollout (1.0: 3.3 cells over 512 substeps)")
    ap.add_argument("--rebin", type=int, default=None, choices=(0, 1, 2),
                    help="c2/c3: sort the particles into tiles again at every checkpoint "
                         "(1), or at the checkpoints where more than 0.5%% of the last "
                         "segment's particle-substeps overflowed their tile boxes (2); "
                         "default: 1 for c2, whose blocks travel, 0 for c3")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the HIP-event kernel timing")
    args = ap.parse_args()
    args.ckpt_given = args.ckpt
    if args.ckpt is None:
        args.ckpt = 32

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: measures the single-GPU path on one MI355X; runs on more "
              "than one GPU are not supported (the scenes would shard as described "
              "in the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from paper_1810_01054_amd import scenes as S

    sc = S.config_3()
    ctrl = args.workload == "c3ctrl"
    cpu = None
    if (args.workload == "c3" and args.cpu_sample > 0 and args.friction is None
            and not args.materials and not args.drift):
        # the oracle first, while no process has touched the GPU (its
        # all-cores leg forks one worker per host core)
        cpu = cpu_baseline(sc, args.cpu_sample, max(1, args.cpu_sample // 2))
        print(f"bench: oracle {cpu['one_core']['value']:.3g} pss/s on one core, "
              f"{cpu['value']:.3g} on {cpu['cores']} cores", file=sys.stderr, flush=True)

    import torch

    from paper_1810_01054_amd.autograd import (act_bank, rollout, rollout_ctrl,
                                               rollout_materials)
    from paper_1810_01054_amd.sim import Simulator

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.workload == "c4":
        return run_batched(args)
    if args.workload == "c2":
        return run_c2(args)
    if args.workload == "c5":
        return run_serving(args)
    if args.workload == "copy":
        return run_copy(args)

    if args.friction is not None:
        sc.bc, sc.friction = 1, float(np.float32(args.friction))
    if args.drift:
        sc.v[0, :] += np.float32(args.drift)
    T, k = args.T, args.ckpt
    N, d = sc.n_particles, sc.dim
    sim = Simulator([sc.params()], act_id=sc.act_id, scatter=args.scatter,
                    fusion=args.fusion, rebin=int(args.rebin or 0))
    t = lambda a: torch.tensor(np.ascontiguousarray(a, np.float32), device=dev)
    x0, v0, C0, F0 = (t(a) for a in sc.state)
    v0.requires_grad_(True)
    freq = t(sc.freq)
    amp = t(sc.amp).requires_grad_(True)
    phase = t(sc.phase).requires_grad_(True)

    if ctrl:
        # closed loop: a = tanh(W z + b) over the 16 actuated leg quadrants'
        # mean positions and velocities (z has 3 + 96 entries)
        comp, n_comp, W, b, target = S.controller_params(sc, seed=1816, w_scale=0.1)
        comp_t = torch.tensor(comp, dtype=torch.int32, device=dev)
        W_t, b_t = t(W).requires_grad_(True), t(b).requires_grad_(True)
        target_t = t(target)

    if args.materials:
        E_p, rho_p = S.material_field(sc, 1817)
        E_t, rho_t = t(E_p).requires_grad_(True), t(rho_p).requires_grad_(True)

    def one_step():
        if args.materials:
            act = act_bank(T, sc.dt, freq, amp, phase)
            xT, vT, CT, FT = rollout_materials(sim, (x0, v0, C0, F0), act, T, E_t, rho_t, k)
            loss = xT[0].mean()
            loss.backward()
            return loss
        if ctrl:
            xT, vT, CT, FT, _ = rollout_ctrl(sim, (x0, v0, C0, F0), T, comp_t, n_comp, W_t,
                                             b_t, target_t, k)
        else:
            act = act_bank(T, sc.dt, freq, amp, phase)
            xT, vT, CT, FT = rollout(sim, (x0, v0, C0, F0), act, T, k)
        loss = xT[0].mean()              # centroid x of the final state
        loss.backward()
        return loss

    # warm-up; the first warm-up step also finds the dominant kernel
    dominant = "adj_gather"
    warm_prof = None
    kernel_roof = None
    realised_pss = None
    for w in range(max(args.warmup, 1)):
        if w == 0 and not args.no_profile:
            sim.profile(["p2g", "grid", "g2p", "adj_scatter", "adj_grid", "adj_gather",
                         "g2p_p2g", "adj_fused"])
        one_step()
        if w == 0 and not args.no_profile:
            prof = sim.profile_read()
            sim.profile([])
            dominant = max(prof, key=lambda kk: prof[kk][1])
            warm_prof = {kk: round(ms * 1e3 / max(n, 1), 2)
                         for kk, (n, ms) in prof.items() if n}
            # every kernel against the HBM roofline (algorithmic bytes)
            kernel_roof = {}
            for kk, (n, ms) in prof.items():
                if not n:
                    continue
                if kk in ("grid", "adj_grid"):
                    b = kernel_bytes_per_node(kk, d) * sim.G
                else:
                    b = kernel_bytes_per_particle(kk, d) * N
                gbs = b / (ms / n / 1e3) / 1e9
                kernel_roof[kk] = {"avg_us": round(ms * 1e3 / n, 2), "launches": n,
                                   "algorithmic_GBps": round(gbs, 1),
                                   "frac": round(gbs / HBM_PEAK_GBS, 4),
                                   "share_of_time": None, "_ms": ms}
            tot = sum(v["_ms"] for v in kernel_roof.values())
            for v in kernel_roof.values():
                v["share_of_time"] = round(v.pop("_ms") / tot, 4)
            # the particle-stream bytes the launched kernels move per
            # particle-substep (from the launch counts of this rollout)
            realised_pss = sum(
                n * (kernel_bytes_per_node(kk, d) * sim.G if kk in ("grid", "adj_grid")
                     else kernel_bytes_per_particle(kk, d) * N)
                for kk, (n, ms) in prof.items() if n and kk not in ("grid", "adj_grid")
            ) / (N * T)
    sim.sync_errors()
    torch.cuda.synchronize()

    # the timed region: K whole rollouts, no kernel timing inside
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
        # the dominant kernel's launches timed with HIP events on the
        # library's stream over the same K rollouts, run again right after
        # the timed region (the events add a gap per launch, so they stay
        # out of the headline)
        sim.profile([dominant])
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for i in range(args.steps):
            one_step()
        torch.cuda.synchronize()
        prof_wall = time.perf_counter() - tp
        prof = sim.profile_read()
        sim.profile([])
        n_launch, ms = prof[dominant]
        avg_s = ms / max(n_launch, 1) / 1e3
        realised = (kernel_bytes_per_node(dominant, d) if dominant in ("grid", "adj_grid")
                    else kernel_bytes_per_particle(dominant, d))
        units = sim.G if dominant in ("grid", "adj_grid") else N
        stage = stage_bytes_per_particle(dominant, d)
        bpu = stage if stage is not None else realised
        achieved = bpu * units / avg_s / 1e9
        traffic = recorded_traffic(dominant)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic / avg_s / 1e9, 1),
                "traffic_bytes_per_launch": traffic, "kernel": dominant,
                "avg_launch_us": round(avg_s * 1e6, 2), "launches": n_launch,
                "bytes_per_unit": bpu,
                "bytes_per_unit_source": ("method stage (byte model)" if stage is not None
                                          else "kernel streams"),
                "realised_bytes_per_unit": realised,
                "realised_frac": round(realised * units / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                "units_per_launch": units,
                "timed_over": f"{args.steps} rollouts right after the timed region",
                "profiled_ms_per_step": round(prof_wall / args.steps * 1e3, 3)}

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
                               f"16 actuators "
                               + ("driven by a closed-loop controller tanh(W z + b) over "
                                  "16 component means" if ctrl else "")
                               + f", T={T} substeps fwd+bwd, checkpoint k={k} "
                               f"with recompute, torch.autograd.Function",
                   "controller": "closed loop" if ctrl else "open-loop sinusoid bank",
                   "materials": ("per-particle E, rho field with gradients"
                                 if args.materials else "one per scene"),
                   "walls": ("sticky" if args.friction is None
                             else f"friction projection, c = {args.friction}"),
                   "particles": N, "grid": "64^3", "substeps": T, "ckpt_k": k,
                   "scatter_mode": args.scatter,
                   "fusion": args.fusion,
                   "rebin": int(args.rebin or 0),
                   "drift_vx": args.drift,
                   "binnings_per_rollout": sim.tape_binnings(),
                   "global_batch": 1, "parallelism": "single GPU"},
        "pct_hbm_peak_672B_per_pss": round(672.0 * value / (HBM_PEAK_GBS * 1e9), 4),
        # the particle-stream bytes the launched kernels move (launch counts
        # of the profiled warm-up rollout x each kernel's stream bytes)
        "realised_bytes_per_pss": None if realised_pss is None else round(realised_pss, 1),
        "pct_hbm_peak_realised": (None if realised_pss is None else
                                  round(realised_pss * value / (HBM_PEAK_GBS * 1e9), 4)),
        "rollout_latency_ms": {"p50": round(percentile(lat, 0.5), 3),
                               "p99": round(percentile(lat, 0.99), 3)},
        "roofline": roof,
        "kernel_avg_us": warm_prof,
        "kernel_roofline": kernel_roof,
        "cpu_baseline": None,
    }
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
