"""Full-size parity (C3: the 3D 64^3 quadruped, 504,064 particles) in the
launch configuration the benchmark times (binned rollout, sorted scatter,
checkpoints with recompute): a few substeps forward and backward, compared
element by element with the oracle, for the default path and for each of
the friction walls, the per-particle material field, the closed-loop
controller and binomial checkpointing.  T >= 2 so the fused G2P + P2G
kernel runs.  Tolerances: states 2e-5, adjoints and parameter gradients
1e-4 (a few substeps of FP32 rounding), each on the normwise error and on
the largest per-element error relative to the field's largest magnitude.

The benchmark's own scene (unperturbed C3, checkpoint every 32 substeps with
recompute) is also compared over 100 substeps forward and backward, the
horizon of the required bounds (positions 1e-5, gradients 1e-3)."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1810_01054_amd import scenes as S
from tests.helpers import oscene, f64, err
from tests.gpu_helpers import (require_gpu, say, to_gpu, to_np, sim_for, seeds,
                               check_state)

pytestmark = pytest.mark.gpu

STATE_TOL = 2e-5
ADJ_TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def c3():
    return S.perturb(S.config_3(), 2, v_scale=0.2, C_scale=0.5, F_scale=0.02)


def _seed(sc):
    return tuple((a / sc.n_particles).astype(np.float32) for a in seeds(sc.state, 5))


def _acts(sc, T):
    return oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)


def _cmp(sT, g0, gact, refT, ref0, ref_act):
    for k in range(4):
        assert err(to_np(sT)[k], refT[k]) < STATE_TOL, ("xvCF"[k], err(to_np(sT)[k], refT[k]))
        assert err(to_np(g0)[k], ref0[k]) < ADJ_TOL, ("g" + "xvCF"[k], err(to_np(g0)[k], ref0[k]))
    if gact is not None:
        assert err(gact.cpu().numpy(), ref_act) < ADJ_TOL


@pytest.mark.parametrize("T,k", [(3, 2), (4, -1)], ids=["ckpt2", "binomial1"])
def test_c3_rollout_default_path(c3, T, k):
    sc = c3
    say("full_c3", sc.n_particles, "T", T, "k", k)
    acts, gT = _acts(sc, T), _seed(sc)
    sim = sim_for(sc)
    sT, g0, gact = sim.rollout(to_gpu(sc.state), torch.tensor(acts, device="cuda"), T,
                               ckpt_k=k, gT=to_gpu(gT))
    sim.sync_errors()
    ref = oracle.rollout(oscene(sc), f64(sc.state), T, sc.act_id, acts.astype(np.float64), f64(gT))
    _cmp(sT, g0, gact, *ref)
    sim.close()


def test_c3_friction_walls(c3):
    sc = S.perturb(S.config_3(), 2, v_scale=0.2, C_scale=0.5, F_scale=0.02)
    # lowered by 1.2 cells and pressed into the floor: the feet's stencils
    # reach the floor's wall band, so the projection and its reverse run
    sc.x[1, :] -= np.float32(1.2 / sc.n_grid)
    sc.v[1, :] -= 2.0
    sc.bc, sc.friction = 1, float(np.float32(0.5))
    assert (np.floor(sc.x[1] * sc.n_grid - 0.5) <= sc.wall - 1).any()
    T = 2
    say("full_c3_friction", sc.n_particles)
    acts, gT = _acts(sc, T), _seed(sc)
    sim = sim_for(sc)
    sT, g0, gact = sim.rollout(to_gpu(sc.state), torch.tensor(acts, device="cuda"), T,
                               ckpt_k=2, gT=to_gpu(gT))
    sim.sync_errors()
    ref = oracle.rollout(oscene(sc), f64(sc.state), T, sc.act_id, acts.astype(np.float64), f64(gT))
    _cmp(sT, g0, gact, *ref)
    sim.close()


def test_c3_material_field(c3):
    sc = c3
    T = 2
    E_p, rho_p = S.material_field(sc, 71)
    N = sc.n_particles
    gE, grho = np.zeros(N), np.zeros(N)
    os_ = oscene(sc, E_p=E_p.astype(np.float64), rho_p=rho_p.astype(np.float64),
                 gE_p=gE, grho_p=grho)
    say("full_c3_materials", N)
    acts, gT = _acts(sc, T), _seed(sc)
    sim = sim_for(sc)
    cu = lambda a: torch.tensor(np.ascontiguousarray(a, np.float32), device="cuda")
    sim.set_materials(cu(E_p), cu(rho_p))
    sT, g0, gact = sim.rollout(to_gpu(sc.state), cu(acts), T, ckpt_k=2, gT=to_gpu(gT))
    gEg, grhog = sim.material_grad()
    sim.sync_errors()
    ref = oracle.rollout(os_, f64(sc.state), T, sc.act_id, acts.astype(np.float64), f64(gT))
    _cmp(sT, g0, gact, *ref)
    assert err(gEg.cpu().numpy(), gE) < ADJ_TOL
    assert err(grhog.cpu().numpy(), grho) < ADJ_TOL
    sim.close()


def test_c3_closed_loop_controller(c3):
    sc = c3
    T = 2
    comp, nc, W, b, target = S.controller_params(sc, seed=1816, w_scale=0.1)
    gT = _seed(sc)
    say("full_c3_controller", sc.n_particles)
    refT, racts, r0, rW, rb = oracle.rollout_ctrl(
        oscene(sc), f64(sc.state), T, comp, nc, W.astype(np.float64), b.astype(np.float64),
        target.astype(np.float64), act_id=sc.act_id, gradT=f64(gT))
    cu = lambda a, dt=torch.float32: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    sim = sim_for(sc)
    sT, act, g0, gact, gW, gb = sim.rollout_ctrl(to_gpu(sc.state), T, cu(comp, torch.int32), nc,
                                                 cu(W), cu(b), cu(target), ckpt_k=2,
                                                 gT=to_gpu(gT))
    sim.sync_errors()
    assert err(act.cpu().numpy(), racts) < STATE_TOL
    _cmp(sT, g0, None, refT, r0, None)
    assert err(gW.cpu().numpy(), rW) < ADJ_TOL
    assert err(gb.cpu().numpy(), rb) < ADJ_TOL
    sim.close()


@pytest.mark.timeout(900)
def test_c3_100_substeps_bench_config(capsys):
    """C3 exactly as the benchmark runs it (the unperturbed scene at rest on
    the floor, binned rollout, fused forward kernel, checkpoint every 32
    substeps with G2P-only recompute) for 100 substeps forward and backward,
    against the oracle chained step by step in FP64 (its forward states kept,
    then its reverse substeps from the last to the first).  The loss is the
    centroid's x plus a seeded linear form of the final positions, so every
    adjoint field and dL/ds is non-trivial.  Bounds: final state per field as
    for the other rollouts (positions 1e-5 and 1e-3 cells), adjoint of S^0
    and dL/ds 1e-3, all normwise and per element."""
    sc = S.config_3()
    T, k = 100, 32
    N, d = sc.n_particles, sc.dim
    acts = _acts(sc, T)
    rng = np.random.default_rng(1817)
    gx = np.zeros((d, N))
    gx[0] += 1.0 / N
    gx += rng.normal(size=(d, N)) / N
    gT = (gx.astype(np.float32), np.zeros((d, N), np.float32),
          np.zeros((d * d, N), np.float32), np.zeros((d * d, N), np.float32))
    say("full_c3_T100", N, "k", k)
    sim = sim_for(sc)
    sT, g0, gact = sim.rollout(to_gpu(sc.state), torch.tensor(acts, device="cuda"), T,
                               ckpt_k=k, gT=to_gpu(gT))
    sim.sync_errors()
    sT, g0, gact = to_np(sT), to_np(g0), gact.cpu().numpy()
    sim.close()

    os_ = oscene(sc)
    a64 = acts.astype(np.float64)
    t0 = time.perf_counter()
    states = [f64(sc.state)]
    for n in range(T):
        states.append(oracle.step_fwd(os_, states[-1], sc.act_id, a64[n]))
        if (n + 1) % 10 == 0:
            with capsys.disabled():
                print(f"[oracle] forward {n + 1}/{T} {time.perf_counter() - t0:.0f} s",
                      flush=True)
    refT = states[T]
    check_state(sT, refT, 1.0 / sc.n_grid, label="c3 T=100 k=32")
    g = f64(gT)
    ref_act = np.zeros((T, sc.n_act))
    for n in range(T - 1, -1, -1):
        g, ref_act[n] = oracle.step_bwd(os_, states[n], g, sc.act_id, a64[n])
        states[n + 1] = None
        if n % 10 == 0:
            with capsys.disabled():
                print(f"[oracle] reverse {n}/{T} {time.perf_counter() - t0:.0f} s", flush=True)
    errs = {"g" + c: err(a, b) for c, a, b in zip("xvCF", g0, g)}
    errs["g_act"] = err(gact, ref_act)
    say("c3 T=100 adjoint errors", {kk: f"{v:.2e}" for kk, v in errs.items()})
    for kk, v in errs.items():
        assert v < 1e-3, (kk, v)
