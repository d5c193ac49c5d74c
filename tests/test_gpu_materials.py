"""GPU parity of per-particle materials (E_p, rho_p: mpm_set_materials) and
their gradients (mpm_material_grad) through the C ABI against the oracle,
whose material gradients are pinned by Euler's relation for the joint
scaling of mass, stiffness and actuation and by central differences.
Tolerances: one substep 2e-5 (state) and 1e-4 (adjoints); rollouts 1e-5
(positions) and 1e-3 (every gradient)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_01054_amd import scenes as S
from paper_1810_01054_amd._lib import MPMError
from tests.helpers import oscene, f64, err
from tests.gpu_helpers import require_gpu, say, to_gpu, to_np, sim_for, check_state

pytestmark = pytest.mark.gpu

STEP_TOL = 2e-5
STEP_ADJ_TOL = 1e-4
POS_TOL = 1e-5
GRAD_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _ocase(sc, E_p, rho_p):
    N = sc.n_particles
    gE, grho = np.zeros(N), np.zeros(N)
    os_ = oscene(sc, E_p=E_p.astype(np.float64), rho_p=rho_p.astype(np.float64),
                 gE_p=gE, grho_p=grho)
    return os_, gE, grho


def _cu(a):
    return torch.tensor(np.ascontiguousarray(a, np.float32), device="cuda")


def _cases():
    return [
        ("tiny2d", S.perturb(S.tiny_2d(n=16, n_particles=40), 3, v_scale=0.3, C_scale=1.0,
                             F_scale=0.05)),
        ("box3d_ragged", S.perturb(S.box_3d(32, (8, 5, 9), (17, 12, 15)), 6, v_scale=0.3,
                                   C_scale=1.0, F_scale=0.05)),
    ]


@pytest.mark.parametrize("name,sc", _cases(), ids=[c[0] for c in _cases()])
def test_materials_step_forward_and_backward(name, sc):
    say("materials_step", name, sc.n_particles)
    E_p, rho_p = S.material_field(sc, 61)
    os_, gE, grho = _ocase(sc, E_p, rho_p)
    rng = np.random.default_rng(62)
    act = rng.uniform(-2, 2, sc.n_act).astype(np.float32)
    sim = sim_for(sc)
    sim.set_materials(_cu(E_p), _cu(rho_p))
    out = sim.step_forward(to_gpu(sc.state), _cu(act))
    sim.sync_errors()
    ref = oracle.step_fwd(os_, f64(sc.state), sc.act_id, act)
    for a, r in zip(to_np(out), ref):
        assert err(a, r) < STEP_TOL
    g1 = tuple(rng.normal(size=a.shape).astype(np.float32) for a in sc.state)
    g_act = torch.zeros(sc.n_act, device="cuda")
    g0 = sim.step_backward(to_gpu(sc.state), _cu(act), to_gpu(g1), g_act=g_act)
    gEg, grhog = sim.material_grad()
    sim.sync_errors()
    gref, aref = oracle.step_bwd(os_, f64(sc.state), f64(g1), sc.act_id, act)
    for c, (a, r) in enumerate(zip(to_np(g0), gref)):
        assert err(a, r) < STEP_ADJ_TOL, (c, err(a, r))
    assert err(g_act.cpu().numpy(), aref) < STEP_ADJ_TOL
    assert err(gEg.cpu().numpy(), gE) < STEP_ADJ_TOL, err(gEg.cpu().numpy(), gE)
    assert err(grhog.cpu().numpy(), grho) < STEP_ADJ_TOL, err(grhog.cpu().numpy(), grho)
    sim.close()


@pytest.mark.parametrize("name,sc", _cases(), ids=[c[0] for c in _cases()])
def test_materials_rollout_matches_oracle(name, sc):
    T = 30
    E_p, rho_p = S.material_field(sc, 63)
    acts = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
    rng = np.random.default_rng(64)
    N, d = sc.n_particles, sc.dim
    gT = [(rng.normal(size=(d, N)) / N).astype(np.float32),
          (rng.normal(size=(d, N)) / N).astype(np.float32),
          np.zeros((d * d, N), np.float32), np.zeros((d * d, N), np.float32)]
    os_, gE, grho = _ocase(sc, E_p, rho_p)
    refT, ref0, ref_act = oracle.rollout(os_, f64(sc.state), T, sc.act_id,
                                         acts.astype(np.float64), f64(gT))
    sim = sim_for(sc)
    sim.set_materials(_cu(E_p), _cu(rho_p))
    for k in (0, 8, -3):
        say("materials_rollout", name, N, "k", k)
        sT, g0, gact = sim.rollout(to_gpu(sc.state), _cu(acts), T, ckpt_k=k, gT=to_gpu(gT))
        gEg, grhog = sim.material_grad()
        sim.sync_errors()
        check_state(to_np(sT), refT, 1.0 / sc.n_grid, label=f"{sc.name}")
        for c, (a, r) in enumerate(zip(to_np(g0), ref0)):
            assert err(a, r) < GRAD_TOL, (k, c, err(a, r))
        assert err(gact.cpu().numpy(), ref_act) < GRAD_TOL
        assert err(gEg.cpu().numpy(), gE) < GRAD_TOL, (k, err(gEg.cpu().numpy(), gE))
        assert err(grhog.cpu().numpy(), grho) < GRAD_TOL, (k, err(grhog.cpu().numpy(), grho))
    sim.close()


def test_uniform_field_equals_scene_materials_and_switching_off():
    sc = S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=39)
    T = 20
    acts = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
    N = sc.n_particles
    gT = [np.full((3, N), 1.0 / N, np.float32), np.zeros((3, N), np.float32),
          np.zeros((9, N), np.float32), np.zeros((9, N), np.float32)]
    sim = sim_for(sc)
    say("materials_uniform")
    ref = sim.rollout(to_gpu(sc.state), _cu(acts), T, ckpt_k=8, gT=to_gpu(gT))
    with pytest.raises(MPMError):
        sim.material_grad()                       # no field yet
    sim.set_materials(_cu(np.full(N, sc.E)), _cu(np.full(N, sc.rho)))
    got = sim.rollout(to_gpu(sc.state), _cu(acts), T, ckpt_k=8, gT=to_gpu(gT))
    sim.sync_errors()
    # the field path scatters masses from the records and runs no fused
    # forward kernel: FP32 summation order only
    for a, r in zip(to_np(got[0]) + to_np(got[1]), to_np(ref[0]) + to_np(ref[1])):
        assert err(a, r) < 1e-5
    sim.set_materials(None, None)
    off = sim.rollout(to_gpu(sc.state), _cu(acts), T, ckpt_k=8, gT=to_gpu(gT))
    sim.sync_errors()
    for a, r in zip(to_np(off[0]), to_np(ref[0])):
        assert err(a, r) < 1e-5
    with pytest.raises(MPMError):
        sim.material_grad()
    sim.close()


def test_materials_autograd_wrapper():
    # system identification: the gradient of a loss on the final state with
    # respect to the stiffness and density fields, through torch.autograd
    from paper_1810_01054_amd.autograd import rollout_materials
    sc = S.perturb(S.tiny_3d(n=12, n_particles=30), 8, v_scale=0.3, C_scale=1.0, F_scale=0.05)
    T = 12
    E_p, rho_p = S.material_field(sc, 65)
    acts = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
    rng = np.random.default_rng(66)
    gx = rng.normal(size=sc.x.shape).astype(np.float32)
    os_, gE, grho = _ocase(sc, E_p, rho_p)
    z = [np.zeros_like(a, dtype=np.float64) for a in sc.state]
    oracle.rollout(os_, f64(sc.state), T, sc.act_id, acts.astype(np.float64),
                   [gx.astype(np.float64)] + z[1:])
    sim = sim_for(sc)
    Et, rt = _cu(E_p).requires_grad_(True), _cu(rho_p).requires_grad_(True)
    say("materials_autograd")
    out = rollout_materials(sim, to_gpu(sc.state), _cu(acts), T, Et, rt, ckpt_k=4)
    (out[0] * _cu(gx)).sum().backward()
    sim.sync_errors()
    assert err(Et.grad.cpu().numpy(), gE) < GRAD_TOL
    assert err(rt.grad.cpu().numpy(), grho) < GRAD_TOL
    sim.close()
