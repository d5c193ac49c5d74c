"""GPU parity for combinations of options the other parity files take one at
a time: per-particle materials under every scatter mode and without
binning, materials on a two-scene batch, the controller without binning,
and friction walls + a material field + binomial checkpointing together.
Oracle comparison as elsewhere: positions 1e-5, gradients 1e-3."""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_01054_amd import scenes as S
from tests.helpers import oscene, f64, err
from tests.gpu_helpers import require_gpu, say, to_gpu, to_np, sim_for, concat_state, check_state

pytestmark = pytest.mark.gpu

POS_TOL = 1e-5
GRAD_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _cu(a, dt=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _seed(sc, seed):
    rng = np.random.default_rng(seed)
    N, d = sc.n_particles, sc.dim
    return [(rng.normal(size=(d, N)) / N).astype(np.float32),
            (rng.normal(size=(d, N)) / N).astype(np.float32),
            np.zeros((d * d, N), np.float32), np.zeros((d * d, N), np.float32)]


def _oracle_mat(sc, E_p, rho_p, T, acts, gT):
    N = sc.n_particles
    gE, grho = np.zeros(N), np.zeros(N)
    os_ = oscene(sc, E_p=E_p.astype(np.float64), rho_p=rho_p.astype(np.float64),
                 gE_p=gE, grho_p=grho)
    refT, ref0, ref_act = oracle.rollout(os_, f64(sc.state), T, sc.act_id,
                                         acts.astype(np.float64), f64(gT))
    return refT, ref0, ref_act, gE, grho


def _check(sim, sc, T, k, acts, gT, ref, mat=True):
    refT, ref0, ref_act, gE, grho = ref
    sT, g0, gact = sim.rollout(to_gpu(sc.state), _cu(acts), T, ckpt_k=k, gT=to_gpu(gT))
    sim.sync_errors()
    check_state(to_np(sT), refT, 1.0 / sc.n_grid, label=f"{sc.name}")
    for c, (a, r) in enumerate(zip(to_np(g0), ref0)):
        assert err(a, r) < GRAD_TOL, (c, err(a, r))
    assert err(gact.cpu().numpy(), ref_act) < GRAD_TOL
    if mat:
        gEg, grhog = sim.material_grad()
        sim.sync_errors()
        assert err(gEg.cpu().numpy(), gE) < GRAD_TOL
        assert err(grhog.cpu().numpy(), grho) < GRAD_TOL


@pytest.mark.parametrize("opts", [dict(scatter=1), dict(scatter=2), dict(sort=False)],
                         ids=["scatter1", "scatter2", "unsorted"])
@pytest.mark.parametrize("dim", [2, 3])
def test_materials_under_every_scatter_mode(opts, dim):
    sc = S.perturb(S.config_1b() if dim == 2 else S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=43),
                   9, v_scale=0.3, C_scale=1.0, F_scale=0.05)
    T = 20
    E_p, rho_p = S.material_field(sc, 81)
    acts = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
    gT = _seed(sc, 82)
    ref = _oracle_mat(sc, E_p, rho_p, T, acts, gT)
    say("materials_mode", dim, opts)
    sim = sim_for(sc, **opts)
    sim.set_materials(_cu(E_p), _cu(rho_p))
    _check(sim, sc, T, 5, acts, gT, ref)
    sim.close()


def test_materials_on_a_two_scene_batch():
    a = S.perturb(S.tiny_2d(n=16, n_particles=40, seed=5), 1, v_scale=0.3, C_scale=1.0, F_scale=0.05)
    b = S.perturb(S.config_1a(), 2, v_scale=0.3, C_scale=1.0, F_scale=0.05)
    b.nu = float(np.float32(0.25))          # a different Poisson ratio per scene
    T = 15
    mats = [S.material_field(sc, 83 + i) for i, sc in enumerate((a, b))]
    sim = sim_for([a, b])
    say("materials_batch", a.n_particles + b.n_particles)
    sim.set_materials(_cu(np.concatenate([m[0] for m in mats])),
                      _cu(np.concatenate([m[1] for m in mats])))
    acts = [oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
            for sc in (a, b)]
    gTs = [_seed(sc, 85 + i) for i, sc in enumerate((a, b))]
    gT = [np.concatenate([g[k] for g in gTs], axis=1) for k in range(4)]
    sT, g0, gact = sim.rollout(to_gpu(concat_state([a, b])), _cu(np.concatenate(acts, axis=1)),
                               T, ckpt_k=4, gT=to_gpu(gT))
    gEg, grhog = sim.material_grad()
    sim.sync_errors()
    off = 0
    for i, sc in enumerate((a, b)):
        refT, ref0, ref_act, gE, grho = _oracle_mat(sc, mats[i][0], mats[i][1], T, acts[i], gTs[i])
        sl = slice(off, off + sc.n_particles)
        check_state([a[:, sl] for a in to_np(sT)], refT, 1.0 / sc.n_grid, label=f"{sc.name}")
        for c in range(4):
            assert err(to_np(g0)[c][:, sl], ref0[c]) < GRAD_TOL
        assert err(gEg.cpu().numpy()[sl], gE) < GRAD_TOL
        assert err(grhog.cpu().numpy()[sl], grho) < GRAD_TOL
        off += sc.n_particles
    sim.close()


def test_controller_without_binning():
    sc = S.tiny_3d(n=12, n_particles=30)
    T = 16
    comp, nc, W, b, target = S.controller_params(sc, seed=15, n_comp=2)
    gT = _seed(sc, 86)
    refT, racts, r0, rW, rb = oracle.rollout_ctrl(
        oscene(sc), f64(sc.state), T, comp, nc, W.astype(np.float64), b.astype(np.float64),
        target.astype(np.float64), act_id=sc.act_id, gradT=f64(gT))
    sim = sim_for(sc, sort=False)
    say("ctrl_unsorted")
    sT, act, g0, gact, gW, gb = sim.rollout_ctrl(to_gpu(sc.state), T, _cu(comp, torch.int32), nc,
                                                 _cu(W), _cu(b), _cu(target), ckpt_k=4,
                                                 gT=to_gpu(gT))
    sim.sync_errors()
    check_state(to_np(sT), refT, 1.0 / sc.n_grid, label=f"{sc.name}")
    assert err(act.cpu().numpy(), racts) < POS_TOL
    for a, r in zip(to_np(g0), r0):
        assert err(a, r) < GRAD_TOL
    assert err(gW.cpu().numpy(), rW) < GRAD_TOL
    assert err(gb.cpu().numpy(), rb) < GRAD_TOL
    sim.close()


def test_friction_materials_and_binomial_together():
    sc = S.wall_contact(3, n=24, n_particles=900, seed=28, friction=0.4)
    T = 24
    E_p, rho_p = S.material_field(sc, 87)
    acts = np.random.default_rng(88).uniform(-1.5, 1.5, size=(T, sc.n_act)).astype(np.float32)
    gT = _seed(sc, 89)
    ref = _oracle_mat(sc, E_p, rho_p, T, acts, gT)
    sim = sim_for(sc)
    sim.set_materials(_cu(E_p), _cu(rho_p))
    say("friction_materials_binomial")
    _check(sim, sc, T, -3, acts, gT, ref)
    sim.close()


def test_graph_replay_follows_the_material_field():
    # a rollout captured without a field must not be replayed once a field is
    # set (other kernels, gradient accumulators), nor the reverse
    sc = S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=44)
    T = 12
    E_p, rho_p = S.material_field(sc, 90)
    acts = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
    gT = _seed(sc, 91)
    graph = sim_for(sc, graphs=True)
    eager = sim_for(sc, graphs=False)
    say("graph_material_toggle")
    outs = {}
    for phase in ("plain", "field", "plain_again"):
        for name, sim in (("graph", graph), ("eager", eager)):
            if phase == "field":
                sim.set_materials(_cu(E_p), _cu(rho_p))
            elif phase == "plain_again":
                sim.set_materials(None, None)
            sT, g0, gact = sim.rollout(to_gpu(sc.state), _cu(acts), T, ckpt_k=4, gT=to_gpu(gT))
            gm = sim.material_grad() if phase == "field" else None
            sim.sync_errors()
            outs[name] = (to_np(sT), to_np(g0), gm)
        (sa, ga, ma), (sb, gb, mb) = outs["graph"], outs["eager"]
        assert err(sa[0], sb[0]) < 1e-6, phase
        for c in range(4):
            assert err(ga[c], gb[c]) < 1e-5, (phase, c)
        if ma is not None:
            # dL/dE_p, dL/drho_p are sums over substeps with cancellation, and
            # the two runs add the scatter's records in different orders (the
            # rank in a cell comes from an LDS atomic): per element they agree
            # to the FP32 adjoint bound of a single substep against the oracle
            assert err(ma[0].cpu().numpy(), mb[0].cpu().numpy()) < 1e-4
            assert err(ma[1].cpu().numpy(), mb[1].cpu().numpy()) < 1e-4
    graph.close()
    eager.close()
