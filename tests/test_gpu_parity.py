"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (normwise relative error, ||gpu - oracle|| / ||oracle||):
  * one substep, grid and particle outputs: 2e-5.  FP32 rounding of a 3^d
    stencil sum of O(1) terms is ~1e-7 relative per term; C' and the
    adjoints involve differences of nearly equal node values (x_i - x_p is
    O(dx) while x is O(1), so cancellation costs up to log2(n) bits), which
    the 2e-5 bound covers with a margin of ~10x at n = 256;
  * positions after 100 substeps: 1e-5 (the required bound);
  * gradients (one step or a whole rollout): 1e-3 (the required bound).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_01054_amd import scenes as S
from tests.helpers import oscene, f64, err
from tests.gpu_helpers import (require_gpu, say, to_gpu, to_np, sim_for,
                               concat_state, gpu_act_bank, seeds, check_state)

pytestmark = pytest.mark.gpu

STEP_TOL = 2e-5
POS_TOL = 1e-5
GRAD_TOL = 1e-3


def _cases_small():
    return [
        ("tiny2d", S.tiny_2d(n=16, n_particles=40)),
        ("tiny3d", S.tiny_3d(n=12, n_particles=24)),
        ("c1a_perturbed", S.perturb(S.config_1a(), 5, v_scale=0.3, C_scale=1.0,
                                    F_scale=0.05)),
        ("box3d_ragged", S.perturb(S.box_3d(32, (8, 5, 9), (17, 12, 15)), 6,
                                   v_scale=0.3, C_scale=1.0, F_scale=0.05)),
    ]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("name,sc", _cases_small(), ids=[c[0] for c in _cases_small()])
def test_step_forward_per_kernel(name, sc):
    say("step_forward_per_kernel", name, sc.n_particles)
    os_ = oscene(sc)
    act = np.random.default_rng(3).uniform(-2, 2, sc.n_act).astype(np.float32)
    sim = sim_for(sc)
    out = sim.step_forward(to_gpu(sc.state), torch.tensor(act, device="cuda"))
    m, p, v = [t.cpu().numpy() for t in sim.get_grid()]
    sim.sync_errors()
    om, op = oracle.p2g(os_, f64(sc.state), sc.act_id, act)
    ov = oracle.grid_update(os_, om, op)
    assert err(m, om) < STEP_TOL
    assert err(p, op) < STEP_TOL
    assert err(v, ov) < STEP_TOL
    ref = oracle.step_fwd(os_, f64(sc.state), sc.act_id, act)
    for k, (a, b) in enumerate(zip(to_np(out), ref)):
        assert err(a, b) < STEP_TOL, ("xvCF"[k], err(a, b))


@pytest.mark.parametrize("name,sc", _cases_small(), ids=[c[0] for c in _cases_small()])
def test_step_backward(name, sc):
    say("step_backward", name, sc.n_particles)
    os_ = oscene(sc)
    act = np.random.default_rng(4).uniform(-2, 2, sc.n_act).astype(np.float32)
    gnext = seeds(sc.state, 9)
    gnext32 = tuple(a.astype(np.float32) for a in gnext)
    sim = sim_for(sc)
    g_act = torch.zeros(sc.n_act, device="cuda")
    g = sim.step_backward(to_gpu(sc.state), torch.tensor(act, device="cuda"),
                          to_gpu(gnext32), g_act=g_act)
    sim.sync_errors()
    ref, ref_act = oracle.step_bwd(os_, f64(sc.state), f64(gnext32), sc.act_id, act)
    for k, (a, b) in enumerate(zip(to_np(g), ref)):
        assert err(a, b) < GRAD_TOL, ("xvCF"[k], err(a, b))
        assert err(a, b) < 1e-4, ("xvCF"[k], err(a, b))
    assert err(g_act.cpu().numpy(), ref_act) < 1e-4


def test_step_in_place_and_shuffled_order():
    sc = S.perturb(S.config_1b(), 12, v_scale=0.3, C_scale=1.0, F_scale=0.05)
    say("in_place_shuffled", sc.n_particles)
    os_ = oscene(sc)
    ref = oracle.step_fwd(os_, f64(sc.state), sc.act_id, np.ones(sc.n_act))
    sim = sim_for(sc)
    st = to_gpu(sc.state)
    sim.step_forward(st, torch.ones(sc.n_act, device="cuda"), out=st)  # in place
    sim.sync_errors()
    for a, b in zip(to_np(st), ref):
        assert err(a, b) < STEP_TOL
    # random particle order: chunks are no longer compact, so most take the
    # global-memory path; results must not change beyond rounding
    sh = S.shuffled(sc, 77)
    ref2 = oracle.step_fwd(os_, f64(sh.state), sh.act_id, np.ones(sh.n_act))
    sim2 = sim_for(sh)
    out2 = sim2.step_forward(to_gpu(sh.state), torch.ones(sh.n_act, device="cuda"))
    sim2.sync_errors()
    for a, b in zip(to_np(out2), ref2):
        assert err(a, b) < STEP_TOL


def test_act_bank_matches_oracle():
    sc = S.config_2()
    T = 300
    say("act_bank", T)
    a = gpu_act_bank(sc, T).cpu().numpy()
    ref = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase)
    assert np.abs(a - ref).max() < 1e-6 * max(1.0, np.abs(ref).max())
    from paper_1810_01054_amd.sim import act_bank_backward
    g = np.random.default_rng(1).normal(size=ref.shape).astype(np.float32)
    t = lambda x: torch.tensor(np.ascontiguousarray(x, np.float32), device="cuda")
    ga, gp = act_bank_backward(T, sc.dt, t(sc.freq), t(sc.amp), t(sc.phase), t(g))
    ra, rp = oracle.act_bank_bwd(T, sc.dt, sc.freq, sc.amp, sc.phase, g)
    assert err(ga.cpu().numpy(), ra) < 1e-5
    assert err(gp.cpu().numpy(), rp) < 1e-5


def _rollout_case(sc, T, ks, loss2_seed=21, **sim_kw):
    os_ = oscene(sc)
    acts = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase)
    acts32 = acts.astype(np.float32)
    N = sc.n_particles
    rng = np.random.default_rng(loss2_seed)
    # L = mean_p x_{p,0}^T + sum_p w_p . x_p^T  (the second term makes the
    # actuation gradient non-trivial even in free flight)
    gT = [np.zeros((sc.dim, N)), np.zeros((sc.dim, N)),
          np.zeros((sc.dim ** 2, N)), np.zeros((sc.dim ** 2, N))]
    gT[0][0] += 1.0 / N
    gT[0] += rng.normal(size=(sc.dim, N)) * (1.0 / N)
    gT32 = [a.astype(np.float32) for a in gT]
    refT, ref0, ref_act = oracle.rollout(os_, f64(sc.state), T, sc.act_id,
                                         acts32.astype(np.float64), f64(gT32))
    sim = sim_for(sc, **sim_kw)
    for k in ks:
        say("rollout", sc.name, "T", T, "k", k, sim_kw)
        sT, g0, gact = sim.rollout(to_gpu(sc.state), torch.tensor(acts32, device="cuda"),
                                   T, ckpt_k=k, gT=to_gpu(gT32))
        sim.sync_errors()
        sTn, g0n = to_np(sT), to_np(g0)
        check_state(sTn, refT, 1.0 / sc.n_grid, label=f"{sc.name} k={k}")
        for c in range(4):
            assert err(g0n[c], ref0[c]) < GRAD_TOL, (k, "xvCF"[c], err(g0n[c], ref0[c]))
        assert err(gact.cpu().numpy(), ref_act) < GRAD_TOL, (k, err(gact.cpu().numpy(), ref_act))
    return sim


def test_rollout_c1a_100_steps():
    _rollout_case(S.config_1a(), 100, ks=[0, 1, 8, 100])


def test_rollout_c1b_100_steps():
    _rollout_case(S.config_1b(), 100, ks=[0, 32])


@pytest.mark.parametrize("fusion", [0, 1, 2])
def test_rollout_3d_fused_and_separate_kernels(fusion):
    # 3D binned rollouts: G2P fused with the next P2G (default), every kernel
    # separate, and also each reverse gather fused with the previous
    # substep's adjoint scatter.  k = 1 leaves no substep pair to fuse in a
    # segment, k = 2 one, memo (k = 0) the whole rollout; a ragged last
    # segment (T = 23, k = 8)
    sc = S.perturb(S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=34), 35, v_scale=0.5,
                   C_scale=0.5, F_scale=0.02)
    _rollout_case(sc, 23, ks=[0, 1, 2, 8], fusion=fusion)


@pytest.mark.parametrize("dim", [2, 3])
def test_rollout_persistent_grid_kernels(dim):
    # the node-tile grid kernels as persistent workgroups (a fixed number of
    # one-wave workgroups looping over node tiles): rollouts against the
    # oracle, and a batch of scenes of several grid sizes
    if dim == 2:
        _rollout_case(S.config_1b(), 40, ks=[0, 10], persistent=True)
    else:
        _rollout_case(S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=39), 20, ks=[0, 8],
                      persistent=True)


@pytest.mark.parametrize("scatter", [1, 2, 3])
def test_rollout_scatter_modes(scatter):
    # both binned scatter implementations (per-particle LDS atomics, per-cell
    # register accumulation) in 2D and 3D
    _rollout_case(S.config_1b(), 50, ks=[10], scatter=scatter)
    _rollout_case(S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=32), 30, ks=[0], scatter=scatter)


@pytest.mark.parametrize("case", ["2d_tile16", "3d_tile8"])
def test_rollout_wide_tiles(case):
    # the autotuner's wide-tile candidates (16^2 cells in 2D, 8^3 in 3D): the
    # per-particle LDS-atomic scatters into (tile + 4)^d boxes, and grid nodes
    # summed over one or two boxes per axis, with ragged last tiles
    if case == "2d_tile16":
        _rollout_case(S.config_1b(), 50, ks=[0, 10], tile=16)
    else:
        _rollout_case(S.box_3d(32, (5, 3, 9), (21, 12, 18), seed=33), 30, ks=[0, 10],
                      tile=8)


@pytest.mark.parametrize("recompute_grids", [False, True])
def test_rollout_then_step_then_backward(recompute_grids):
    # the tape survives step calls between a rollout and its reverse pass, for
    # tapes with stored grids and for tapes that recompute them
    sc = S.config_1b()
    T, k = 40, 8
    os_ = oscene(sc)
    acts32 = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
    N = sc.n_particles
    gT = [np.zeros((2, N)), np.zeros((2, N)), np.zeros((4, N)), np.zeros((4, N))]
    gT[0] += np.random.default_rng(3).normal(size=(2, N)) / N
    gT32 = [a.astype(np.float32) for a in gT]
    refT, ref0, ref_act = oracle.rollout(os_, f64(sc.state), T, sc.act_id,
                                         acts32.astype(np.float64), f64(gT32))
    say("rollout_then_step_then_backward", recompute_grids)
    sim = sim_for(sc, recompute_grids=recompute_grids)
    sT = sim.rollout(to_gpu(sc.state), torch.tensor(acts32, device="cuda"), T, ckpt_k=k)
    sim.step_forward(to_gpu(sc.state), torch.ones(sc.n_act, device="cuda"))
    g0, gact = sim.rollout_backward(to_gpu(gT32), T)
    sim.sync_errors()
    check_state(to_np(sT), refT, 1.0 / sc.n_grid, label="rollout_then_step")
    for c in range(4):
        assert err(to_np(g0)[c], ref0[c]) < GRAD_TOL
    assert err(gact.cpu().numpy(), ref_act) < GRAD_TOL
    # the reverse pass can be run again on the same tape
    g0b, _ = sim.rollout_backward(to_gpu(gT32), T)
    sim.sync_errors()
    assert err(to_np(g0b)[0], to_np(g0)[0]) < 1e-6


@pytest.mark.parametrize("dim", [2, 3])
def test_graph_replays_match_eager(dim):
    """Rollouts replayed from captured hipGraphs, several times, with eager
    work and synchronisations between replays, each checked against the
    eager context and the oracle."""
    sc = S.config_1b() if dim == 2 else S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=36)
    T, k = 30, 8
    acts32 = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
    N = sc.n_particles
    d = sc.dim
    gT = [np.random.default_rng(8).normal(size=(d, N)).astype(np.float32) / N,
          np.zeros((d, N), np.float32), np.zeros((d * d, N), np.float32),
          np.zeros((d * d, N), np.float32)]
    refT, ref0, _ = oracle.rollout(oscene(sc), f64(sc.state), T, sc.act_id,
                                   acts32.astype(np.float64), f64(gT))
    eager = sim_for(sc, graphs=False)
    graph = sim_for(sc, graphs=True)
    act = torch.tensor(acts32, device="cuda")
    for rep in range(4):
        say("graph replay", dim, rep)
        e = eager.rollout(to_gpu(sc.state), act, T, ckpt_k=k, gT=to_gpu(gT))
        g = graph.rollout(to_gpu(sc.state), act, T, ckpt_k=k, gT=to_gpu(gT))
        graph.step_forward(to_gpu(sc.state), torch.ones(sc.n_act, device="cuda"))
        torch.cuda.synchronize()
        eager.sync_errors()
        graph.sync_errors()
        # the two contexts add each cell's scatter records in LDS-atomic
        # arrival order, so they agree to FP32 rounding of those sums over
        # 30 substeps, not bit for bit
        for a, b in zip(to_np(g[0]) + to_np(g[1]), to_np(e[0]) + to_np(e[1])):
            assert err(a, b) < 1e-5
        assert err(g[2].cpu().numpy(), e[2].cpu().numpy()) < 1e-5
        check_state(to_np(g[0]), refT, 1.0 / sc.n_grid, label=f"graph {dim} {rep}")
        assert err(to_np(g[1])[1], ref0[1]) < GRAD_TOL


def test_rollout_3d_box_contact():
    # a 3D block dropped onto the floor: wall contact within the rollout
    sc = S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=31)
    _rollout_case(sc, 60, ks=[0, 16])


@pytest.mark.parametrize("scatter", [1, 2, 3])
def test_rollout_fast_drift_uses_overflow_path(scatter):
    # particles binned once per rollout drift ~4 cells here: out of their
    # cell (per-cell mode: LDS atomics into the box) and beyond the one cell
    # of slack of their tile box (global atomics); results must not change
    sc = S.block_2d(64, (0.2, 0.3), (0.35, 0.45), seed=51)
    sc.v[0, :] = 6.0
    sc.v[1, :] = 2.0
    _rollout_case(sc, 100, ks=[0, 25], scatter=scatter)


def test_rollout_c2_100_steps_and_k_invariance():
    """C2 (2D 256^2, 98,304 particles, 48 actuators x 4-sinusoid banks):
    100 substeps fwd + bwd against the oracle; then the full 1,000-substep
    rollout with k = 64 against the same rollout with every state stored.
    The runs differ only in FP32 rounding: the scatter's in-LDS sort orders a
    cell's particles by arrival, and particles that drifted beyond their
    tile box's slack (most of them after ~400 substeps here) add to the grid
    with global atomics, so neither run's sums are bitwise reproducible.
    Over 1,000 substeps the final states agree per field to the bounds the
    rollouts are held to against the oracle, and the adjoints to 1e-4 (an
    order below the gradient tolerance)."""
    sc = S.config_2()
    _rollout_case(sc, 100, ks=[64])
    T = 1000
    say("c2 full", sc.n_particles, T)
    act = gpu_act_bank(sc, T)
    N = sc.n_particles
    gT = [np.zeros((2, N), np.float32), np.zeros((2, N), np.float32),
          np.zeros((4, N), np.float32), np.zeros((4, N), np.float32)]
    gT[0][0] = 1.0 / N                     # centroid x-displacement
    sim = sim_for(sc)
    outs = []
    for k in (64, 0):
        sT, g0, gact = sim.rollout(to_gpu(sc.state), act, T, ckpt_k=k, gT=to_gpu(gT))
        sim.sync_errors()
        outs.append((to_np(sT), to_np(g0), gact.cpu().numpy()))
    (sa, ga, aa), (sb, gb, ab) = outs
    assert all(np.isfinite(x).all() for x in sa + ga) and np.isfinite(aa).all()
    check_state(sa, sb, 1.0 / sc.n_grid, label="c2 T=1000 k=64 vs memo")
    for c in range(4):
        assert err(ga[c], gb[c]) < 1e-4, ("adjoint", c, err(ga[c], gb[c]))
    assert err(aa, ab) < 1e-4, err(aa, ab)


def test_rollout_3d_fast_drift():
    # 3D rollouts fuse each G2P with the next P2G: a block moving ~3 cells
    # over the rollout leaves its tile's staged velocity box (gather from
    # HBM) and its box slack (global atomics) on both passes
    sc = S.box_3d(32, (8, 8, 8), (14, 13, 15), seed=33)
    sc.v[0, :] = 9.0
    sc.v[2, :] = -6.0
    _rollout_case(sc, 100, ks=[0, 25])


def test_batched_3d_scenes_rollout():
    # two 3D scenes of different grids in one context (tiles of both scenes
    # in every launch, fused forward included), each against the oracle
    a = S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=34)
    b = S.box_3d(32, (9, 4, 8), (15, 11, 14), seed=35)
    scs = [a, b]
    T = 30
    say("batched_3d", [s.n_particles for s in scs])
    acts = [oracle.act_bank_fwd(T, s.dt, s.freq, s.amp, s.phase).astype(np.float32) for s in scs]
    act = torch.tensor(np.concatenate(acts, axis=1), device="cuda")
    Ntot = sum(s.n_particles for s in scs)
    rng = np.random.default_rng(6)
    gT = [rng.normal(size=(3, Ntot)).astype(np.float32) / Ntot, np.zeros((3, Ntot), np.float32),
          np.zeros((9, Ntot), np.float32), np.zeros((9, Ntot), np.float32)]
    sim = sim_for(scs)
    sT, g0, gact = sim.rollout(to_gpu(concat_state(scs)), act, T, ckpt_k=8, gT=to_gpu(gT))
    sim.sync_errors()
    sT, g0, gact = to_np(sT), to_np(g0), gact.cpu().numpy()
    offs = np.cumsum([0] + [s.n_particles for s in scs])
    aoffs = np.cumsum([0] + [s.n_act for s in scs])
    for i, s in enumerate(scs):
        sl = slice(offs[i], offs[i + 1])
        refT, ref0, ref_act = oracle.rollout(oscene(s), f64(s.state), T, s.act_id,
                                             acts[i].astype(np.float64),
                                             tuple(np.asarray(x[:, sl], np.float64) for x in gT))
        check_state([a[:, sl] for a in sT], refT, 1.0 / s.n_grid, label=f"batched3d {i}")
        for c in range(4):
            assert err(g0[c][:, sl], ref0[c]) < GRAD_TOL, (i, c)
        assert err(gact[:, aoffs[i]:aoffs[i + 1]], ref_act) < GRAD_TOL


def test_batched_scenes_match_per_scene_oracle():
    a = S.perturb(S.block_2d(64, (0.2, 0.1), (0.5, 0.3), seed=41), 1, 0.2, 0.5, 0.03)
    b = S.perturb(S.block_2d(128, (0.3, 0.05), (0.55, 0.2), seed=42), 2, 0.2, 0.5, 0.03)
    c = S.perturb(S.block_2d(32, (0.3, 0.3), (0.5, 0.5), seed=43), 3, 0.2, 0.5, 0.03)
    scs = [a, b, c]
    say("batched", [s.n_particles for s in scs])
    sim = sim_for(scs)
    acts = [np.random.default_rng(i).uniform(-1, 1, s.n_act) for i, s in enumerate(scs)]
    act = torch.tensor(np.concatenate(acts).astype(np.float32), device="cuda")
    out = to_np(sim.step_forward(to_gpu(concat_state(scs)), act))
    sim.sync_errors()
    off = 0
    for s, ac in zip(scs, acts):
        ref = oracle.step_fwd(oscene(s), f64(s.state), s.act_id, ac.astype(np.float32))
        for k in range(4):
            assert err(out[k][:, off:off + s.n_particles], ref[k]) < STEP_TOL
        off += s.n_particles


def test_batched_config4_spot_check():
    """The 64-scene batched workload in one context; 4 seeded scenes checked
    against the oracle (forward + reverse over 20 substeps)."""
    scs = S.config_4()
    pick = [int(i) for i in np.random.default_rng(1814).choice(len(scs), 4, replace=False)]
    T = 20
    say("batched_c4", sum(s.n_particles for s in scs), pick)
    acts = [oracle.act_bank_fwd(T, s.dt, s.freq, s.amp, s.phase).astype(np.float32) for s in scs]
    act = torch.tensor(np.concatenate(acts, axis=1), device="cuda")
    Ntot = sum(s.n_particles for s in scs)
    rng = np.random.default_rng(5)
    gT = [rng.normal(size=(2, Ntot)).astype(np.float32) / 1000, np.zeros((2, Ntot), np.float32),
          np.zeros((4, Ntot), np.float32), np.zeros((4, Ntot), np.float32)]
    sim = sim_for(scs)
    sT, g0, gact = sim.rollout(to_gpu(concat_state(scs)), act, T, ckpt_k=8, gT=to_gpu(gT))
    sim.sync_errors()
    sT, g0, gact = to_np(sT), to_np(g0), gact.cpu().numpy()
    offs = np.cumsum([0] + [s.n_particles for s in scs])
    aoffs = np.cumsum([0] + [s.n_act for s in scs])
    for i in pick:
        s = scs[i]
        sl = slice(offs[i], offs[i + 1])
        refT, ref0, ref_act = oracle.rollout(oscene(s), f64(s.state), T, s.act_id,
                                             acts[i].astype(np.float64),
                                             tuple(np.asarray(a[:, sl], np.float64) for a in gT))
        check_state([a[:, sl] for a in sT], refT, 1.0 / s.n_grid, label=f"c4 scene {i}")
        for c in range(4):
            assert err(g0[c][:, sl], ref0[c]) < GRAD_TOL, (i, c)
        assert err(gact[:, aoffs[i]:aoffs[i + 1]], ref_act) < GRAD_TOL


def test_empty_scene_in_batch():
    a = S.tiny_2d(n=16, n_particles=40)
    e = S.tiny_2d(n=16, n_particles=0, seed=3)
    say("empty_scene")
    sim = sim_for([a, e])
    act = torch.zeros(a.n_act + e.n_act, device="cuda")
    out = to_np(sim.step_forward(to_gpu(concat_state([a, e])), act))
    sim.sync_errors()
    ref = oracle.step_fwd(oscene(a), f64(a.state), a.act_id, np.zeros(a.n_act))
    for k in range(4):
        assert err(out[k], ref[k]) < STEP_TOL


@pytest.mark.parametrize("kind,code", [("domain", -3), ("inverted", -4), ("nonfinite", -5)])
def test_device_errors_match_oracle(kind, code):
    from paper_1810_01054_amd._lib import MPMError
    sc = S.tiny_2d()
    x, v, C, F = [a.copy() for a in sc.state]
    if kind == "domain":
        x[0, 3] = 0.2 / sc.n_grid
    elif kind == "inverted":
        F[:, 5] = [-1.0, 0.0, 0.0, 1.0]
    else:
        v[1, 2] = np.nan
    say("device_error", kind)
    with pytest.raises(oracle.OracleError) as e:
        oracle.step_fwd(oscene(sc), f64((x, v, C, F)), sc.act_id)
    assert e.value.code == code
    sim = sim_for(sc)
    sim.step_forward(to_gpu((x, v, C, F)), torch.zeros(sc.n_act, device="cuda"))
    with pytest.raises(MPMError) as e2:
        sim.sync_errors()
    assert e2.value.code == code
    # the context stays poisoned
    with pytest.raises(MPMError):
        sim.step_forward(to_gpu(sc.state), torch.zeros(sc.n_act, device="cuda"))


def test_rollout_with_invalid_particle_reports_domain_error():
    """Binning (first step of a rollout) meets a particle outside the domain:
    the call returns MPM_ERR_DOMAIN before anything reads the permutation,
    and the error stays with that context."""
    from paper_1810_01054_amd._lib import MPMError
    sc = S.config_1a()
    x = sc.x.copy()
    x[0, 17] = 0.1 / sc.n_grid
    say("rollout_domain_error")
    sim = sim_for(sc)
    act = torch.zeros(10, sc.n_act, device="cuda")
    with pytest.raises(MPMError) as e:
        sim.rollout(to_gpu((x, sc.v, sc.C, sc.F)), act, 10, ckpt_k=5)
    assert e.value.code == -3
    with pytest.raises(MPMError):
        sim.rollout(to_gpu(sc.state), act, 10, ckpt_k=5)
    other = sim_for(sc)       # a fresh context is unaffected
    other.rollout(to_gpu(sc.state), act, 10, ckpt_k=5)
    other.sync_errors()


def test_full_size_3d_one_step_fwd_bwd():
    """C3 at its real shape (504,064 particles, 64^3) in the launch
    configuration the benchmark uses (sorted rollout), one substep forward and
    backward, compared element by element with the oracle."""
    sc = S.perturb(S.config_3(), 2, v_scale=0.2, C_scale=0.5, F_scale=0.02)
    say("full_size_3d", sc.n_particles)
    os_ = oscene(sc)
    acts = oracle.act_bank_fwd(1, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
    gT = seeds(sc.state, 5)
    gT32 = tuple((a / sc.n_particles).astype(np.float32) for a in gT)
    sim = sim_for(sc)
    sT, g0, gact = sim.rollout(to_gpu(sc.state), torch.tensor(acts, device="cuda"), 1,
                               ckpt_k=1, gT=to_gpu(gT32))
    sim.sync_errors()
    refT, ref0, ref_act = oracle.rollout(os_, f64(sc.state), 1, sc.act_id,
                                         acts.astype(np.float64), f64(gT32))
    for k in range(4):
        assert err(to_np(sT)[k], refT[k]) < STEP_TOL, ("xvCF"[k],)
        assert err(to_np(g0)[k], ref0[k]) < 1e-4, ("g" + "xvCF"[k],)
    assert err(gact.cpu().numpy(), ref_act) < 1e-4


@pytest.mark.parametrize("dim", [2, 3])
def test_stencil_tie_positions(dim):
    """Particles exactly on the stencil tie (x/dx - 0.5 an integer) on one or
    more axes.  The exact floor gives f = 0.5 there, where the third node's
    weight and its derivative are both zero, so the result must not depend
    on the side the floor picks.  One substep forward and backward through
    the step calls (caller order), and rollouts of two substeps (binned
    scatter; in 3D the fused G2P + P2G kernel gathers from the tie
    positions), against the oracle, which takes the same reading."""
    sc = S.config_1b() if dim == 2 else S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=37)
    sc = S.perturb(sc, 62, v_scale=0.3, C_scale=1.0, F_scale=0.05)
    rng = np.random.default_rng(61)
    x = sc.x.copy()
    N = sc.n_particles
    for a in range(dim):
        sel = rng.random(N) < 0.5
        b = np.floor(x[a, sel].astype(np.float64) * sc.n_grid - 0.5)
        x[a, sel] = ((b + 0.5) / sc.n_grid).astype(np.float32)
    sc.x = x
    q = x.astype(np.float64) * sc.n_grid - 0.5
    ties = (q == np.floor(q))
    assert ties.any(axis=0).mean() > 0.4 and ties.all(axis=0).any()
    say("tie positions", dim, int(ties.any(axis=0).sum()), "of", N)
    os_ = oscene(sc)
    act = np.random.default_rng(63).uniform(-2, 2, sc.n_act).astype(np.float32)
    sim = sim_for(sc)
    out = sim.step_forward(to_gpu(sc.state), torch.tensor(act, device="cuda"))
    sim.sync_errors()
    ref = oracle.step_fwd(os_, f64(sc.state), sc.act_id, act)
    for k, (a, b) in enumerate(zip(to_np(out), ref)):
        assert err(a, b) < STEP_TOL, ("xvCF"[k], err(a, b))
    gnext = tuple(a.astype(np.float32) for a in seeds(sc.state, 64))
    g = sim.step_backward(to_gpu(sc.state), torch.tensor(act, device="cuda"), to_gpu(gnext))
    sim.sync_errors()
    gref, _ = oracle.step_bwd(os_, f64(sc.state), f64(gnext), sc.act_id, act)
    for k, (a, b) in enumerate(zip(to_np(g), gref)):
        assert err(a, b) < 1e-4, ("g" + "xvCF"[k], err(a, b))
    _rollout_case(sc, 2, ks=[0, 1])
