"""GPU parity of the friction-projection wall condition (bc = 1: the
supplement's friction projection gradients, (L)) through the C ABI against
the oracle, whose projection is pinned by closed forms and central
differences.  Tolerances as for the sticky walls: one substep 2e-5 (grid,
state) and 1e-4 (adjoints), rollouts 1e-5 (positions) and 1e-3 (gradients).
"""
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


def _box3d_floor(friction):
    sc = S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=41)
    sc.v[0, :] = 0.8                      # sliding along x while it lands
    sc.v[1, :] = -1.0
    sc.bc, sc.friction = 1, float(np.float32(friction))
    return sc


def _step_cases():
    return [
        ("contact2d_c0", S.wall_contact(2, n_particles=60, seed=21, friction=0.0)),
        ("contact2d_c04", S.wall_contact(2, n_particles=60, seed=22, friction=0.4)),
        ("contact3d_c03", S.wall_contact(3, n_particles=80, seed=23, friction=0.3)),
        ("box3d_floor_c05", _box3d_floor(0.5)),
    ]


@pytest.mark.parametrize("name,sc", _step_cases(), ids=[c[0] for c in _step_cases()])
def test_friction_step_forward_and_backward(name, sc):
    say("friction_step", name, sc.n_particles)
    os_ = oscene(sc)
    rng = np.random.default_rng(31)
    act = rng.uniform(-2, 2, sc.n_act).astype(np.float32)
    sim = sim_for(sc)
    out = sim.step_forward(to_gpu(sc.state), torch.tensor(act, device="cuda"))
    m, p, v = [t.cpu().numpy() for t in sim.get_grid()]
    sim.sync_errors()
    om, op = oracle.p2g(os_, f64(sc.state), sc.act_id, act)
    ov = oracle.grid_update(os_, om, op)
    assert err(v, ov) < STEP_TOL, err(v, ov)
    ref = oracle.step_fwd(os_, f64(sc.state), sc.act_id, act)
    for a, r in zip(to_np(out), ref):
        assert err(a, r) < STEP_TOL
    g1 = tuple(rng.normal(size=a.shape).astype(np.float32) for a in sc.state)
    g_act = torch.zeros(sc.n_act, device="cuda")
    g0 = sim.step_backward(to_gpu(sc.state), torch.tensor(act, device="cuda"), to_gpu(g1),
                           g_act=g_act)
    sim.sync_errors()
    gref, aref = oracle.step_bwd(os_, f64(sc.state), f64(g1), sc.act_id, act)
    for c, (a, r) in enumerate(zip(to_np(g0), gref)):
        assert err(a, r) < STEP_ADJ_TOL, (c, err(a, r))
    assert err(g_act.cpu().numpy(), aref) < STEP_ADJ_TOL
    sim.close()


def _rollout_cases():
    return [
        ("contact2d_c04", S.wall_contact(2, n=32, n_particles=1500, seed=24, friction=0.4)),
        ("contact3d_c0", S.wall_contact(3, n=24, n_particles=1200, seed=25, friction=0.0)),
        ("box3d_floor_c05", _box3d_floor(0.5)),
    ]


@pytest.mark.parametrize("name,sc", _rollout_cases(), ids=[c[0] for c in _rollout_cases()])
def test_friction_rollout_matches_oracle(name, sc):
    T = 40
    rng = np.random.default_rng(32)
    acts = rng.uniform(-1.5, 1.5, size=(T, sc.n_act)).astype(np.float32)
    N, d = sc.n_particles, sc.dim
    gT = [(rng.normal(size=(d, N)) / N).astype(np.float32),
          (rng.normal(size=(d, N)) / N).astype(np.float32),
          np.zeros((d * d, N), np.float32), np.zeros((d * d, N), np.float32)]
    refT, ref0, ref_act = oracle.rollout(oscene(sc), f64(sc.state), T, sc.act_id,
                                         acts.astype(np.float64), f64(gT))
    sim = sim_for(sc)
    for k in (0, 8):
        say("friction_rollout", name, N, "k", k)
        sT, g0, gact = sim.rollout(to_gpu(sc.state), torch.tensor(acts, device="cuda"), T,
                                   ckpt_k=k, gT=to_gpu(gT))
        sim.sync_errors()
        check_state(to_np(sT), refT, 1.0 / sc.n_grid, label=f"{sc.name}")
        for c, (a, r) in enumerate(zip(to_np(g0), ref0)):
            assert err(a, r) < GRAD_TOL, (k, c, err(a, r))
        assert err(gact.cpu().numpy(), ref_act) < GRAD_TOL
    sim.close()


def test_friction_scene_arguments_are_checked():
    sc = S.wall_contact(2, n_particles=20, seed=26)
    say("friction_args")
    for bc, c in ((2, 0.0), (1, -0.5), (1, float("nan"))):
        p = sc.params()
        p["bc"], p["friction"] = bc, c
        from paper_1810_01054_amd.sim import Simulator
        with pytest.raises(MPMError):
            Simulator([p], act_id=sc.act_id)


@pytest.mark.parametrize("dim", [2, 3])
def test_friction_on_the_high_faces_and_corners(dim):
    # the contact scene mirrored through the box centre: pressed into the
    # high faces (inward normal -e_a), into the corner of all of them in 3D
    base = S.wall_contact(dim, n=24, n_particles=400, seed=29 + dim, friction=0.35)
    sc = S.wall_contact(dim, n=24, n_particles=400, seed=29 + dim, friction=0.35)
    sc.x = (np.float32(1.0) - base.x).astype(np.float32)
    sc.v = (-base.v).astype(np.float32)
    g = sc.n_grid
    assert (np.floor(sc.x * g - 0.5) >= g - sc.wall - 2).any(axis=1).all()  # every axis' band
    T = 20
    rng = np.random.default_rng(35)
    acts = rng.uniform(-1.5, 1.5, size=(T, sc.n_act)).astype(np.float32)
    N, d = sc.n_particles, sc.dim
    gT = [(rng.normal(size=(d, N)) / N).astype(np.float32),
          (rng.normal(size=(d, N)) / N).astype(np.float32),
          np.zeros((d * d, N), np.float32), np.zeros((d * d, N), np.float32)]
    refT, ref0, ref_act = oracle.rollout(oscene(sc), f64(sc.state), T, sc.act_id,
                                         acts.astype(np.float64), f64(gT))
    sim = sim_for(sc)
    say("friction_high_faces", dim, N)
    sT, g0, gact = sim.rollout(to_gpu(sc.state), torch.tensor(acts, device="cuda"), T,
                               ckpt_k=5, gT=to_gpu(gT))
    sim.sync_errors()
    check_state(to_np(sT), refT, 1.0 / sc.n_grid, label=f"{sc.name}")
    for c, (a, r) in enumerate(zip(to_np(g0), ref0)):
        assert err(a, r) < GRAD_TOL, (c, err(a, r))
    assert err(gact.cpu().numpy(), ref_act) < GRAD_TOL
    sim.close()
