"""GPU parity of the closed-loop controller rollout (section IV, Control:
a^n = tanh(W z^n + b) over the component means of state n) through the C ABI
(mpm_rollout_ctrl) against the oracle's controller rollout, which is pinned
by the open-loop reduction, numpy means and central differences.

Tolerances as for open-loop rollouts: final positions and the actuation the
controller produced 1e-5, gradients (state, dL/ds, dL/dW, dL/db) 1e-3."""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_01054_amd import scenes as S
from paper_1810_01054_amd._lib import MPMError
from tests.helpers import oscene, f64, err
from tests.gpu_helpers import require_gpu, say, to_gpu, to_np, sim_for, check_state

pytestmark = pytest.mark.gpu

POS_TOL = 1e-5
GRAD_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _cases():
    return [
        ("tiny2d_random_comps", S.tiny_2d(n=16, n_particles=40), 2),
        ("tiny3d_random_comps", S.tiny_3d(n=12, n_particles=24), 3),
        ("c1b_actuator_comps", S.config_1b(), None),
        ("box3d_ragged_actuator_comps",
         S.perturb(S.box_3d(32, (8, 5, 9), (17, 12, 15)), 6, v_scale=0.3, C_scale=1.0,
                   F_scale=0.05), None),
    ]


def _cuda(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _loss_seed(sc, seed):
    """dL/dS^T of a seeded linear loss in the final positions and velocities."""
    rng = np.random.default_rng(seed)
    N, d = sc.n_particles, sc.dim
    return [(rng.normal(size=(d, N)) / N).astype(np.float32),
            (rng.normal(size=(d, N)) / N).astype(np.float32),
            np.zeros((d * d, N), np.float32), np.zeros((d * d, N), np.float32)]


def _run(sim, sc, T, k, ctl, gT):
    comp, n_comp, W, b, target = ctl
    return sim.rollout_ctrl(to_gpu(sc.state), T, _cuda(comp, torch.int32), n_comp, _cuda(W),
                            _cuda(b), _cuda(target), ckpt_k=k, gT=to_gpu(gT))


@pytest.mark.parametrize("name,sc,n_comp", _cases(), ids=[c[0] for c in _cases()])
def test_ctrl_rollout_matches_oracle(name, sc, n_comp):
    T = 24
    ctl = S.controller_params(sc, seed=21, n_comp=n_comp)
    comp, nc, W, b, target = ctl
    gT = _loss_seed(sc, 22)
    refT, racts, r0, rW, rb = oracle.rollout_ctrl(
        oscene(sc), f64(sc.state), T, comp, nc, W.astype(np.float64), b.astype(np.float64),
        target.astype(np.float64), act_id=sc.act_id, gradT=f64(gT))
    assert np.abs(racts).max() > 0.05   # the controller acts
    sim = sim_for(sc)
    for k in (0, 8):
        say("ctrl_rollout", name, sc.n_particles, "k", k)
        sT, act, g0, gact, gW, gb = _run(sim, sc, T, k, ctl, gT)
        sim.sync_errors()
        sT = to_np(sT)
        check_state(sT, refT, 1.0 / sc.n_grid, label=f"{sc.name} k={k}")
        assert err(act.cpu().numpy(), racts) < POS_TOL
        g0 = to_np(g0)
        for c in range(4):
            assert err(g0[c], r0[c]) < GRAD_TOL, (k, c, err(g0[c], r0[c]))
        assert err(gW.cpu().numpy(), rW) < GRAD_TOL, (k, err(gW.cpu().numpy(), rW))
        assert err(gb.cpu().numpy(), rb) < GRAD_TOL, (k, err(gb.cpu().numpy(), rb))
    sim.close()


def test_ctrl_zero_gain_equals_open_loop_rollout():
    # W = 0: the controller emits tanh(b) every substep, so the closed-loop
    # rollout equals the open-loop one fed with that schedule
    sc = S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=36)
    T = 20
    comp, nc, W, b, target = S.controller_params(sc, seed=5)
    W[:] = 0.0
    gT = _loss_seed(sc, 6)
    sim = sim_for(sc)
    say("ctrl_zero_gain", sc.n_particles)
    sT, act, g0, gact, gW, gb = _run(sim, sc, T, 8, (comp, nc, W, b, target), gT)
    sim.sync_errors()
    sched = torch.tanh(_cuda(b)).repeat(T, 1).contiguous()
    assert err(act.cpu().numpy(), sched.cpu().numpy()) < 1e-6
    sT2, g02, gact2 = sim.rollout(to_gpu(sc.state), sched, T, ckpt_k=8, gT=to_gpu(gT))
    sim.sync_errors()
    # the open-loop run fuses G2P with the next P2G (3D), the closed-loop run
    # does not: the two differ by FP32 rounding only
    for a, r in zip(to_np(sT), to_np(sT2)):
        assert err(a, r) < 1e-6
    # with W = 0 the controller adds nothing to the state adjoint
    for a, r in zip(to_np(g0), to_np(g02)):
        assert err(a, r) < 1e-5
    assert err(gact.cpu().numpy(), gact2.cpu().numpy()) < 1e-5
    s = 1.0 - np.tanh(b.astype(np.float64)) ** 2
    assert err(gb.cpu().numpy(), gact2.cpu().numpy().sum(0) * s) < 1e-5
    sim.close()


def test_ctrl_backward_reruns_and_autograd():
    from paper_1810_01054_amd.autograd import rollout_ctrl
    sc = S.tiny_3d(n=12, n_particles=24)
    T = 16
    comp, nc, W, b, target = S.controller_params(sc, seed=9, n_comp=2)
    gT = _loss_seed(sc, 10)
    sim = sim_for(sc)
    say("ctrl_backward_reruns")
    sT, act, g0, gact, gW, gb = _run(sim, sc, T, 4, (comp, nc, W, b, target), gT)
    g0b, gactb, gWb, gbb = sim.rollout_ctrl_backward(to_gpu(gT), T, W.shape[1])
    sim.sync_errors()
    for a, r in zip(to_np(g0b), to_np(g0)):
        assert err(a, r) < 1e-6
    assert err(gWb.cpu().numpy(), gW.cpu().numpy()) < 1e-6
    # autograd: L = sum gT . S^T through the torch wrapper
    Wt = _cuda(W).requires_grad_(True)
    bt = _cuda(b).requires_grad_(True)
    x0 = to_gpu(sc.state)
    x0 = (x0[0].requires_grad_(True),) + x0[1:]
    out = rollout_ctrl(sim, x0, T, _cuda(comp, torch.int32), nc, Wt, bt, _cuda(target),
                       ckpt_k=4)
    loss = sum((g * s).sum() for g, s in zip(to_gpu(gT), out[:4]))
    loss.backward()
    sim.sync_errors()
    assert err(Wt.grad.cpu().numpy(), gW.cpu().numpy()) < 1e-6
    assert err(bt.grad.cpu().numpy(), gb.cpu().numpy()) < 1e-6
    assert err(x0[0].grad.cpu().numpy(), to_np(g0)[0]) < 1e-6
    # the open-loop tape has no controller
    sim.rollout(to_gpu(sc.state), act, T, ckpt_k=4)
    with pytest.raises(MPMError):
        sim.rollout_ctrl_backward(to_gpu(gT), T, W.shape[1])
    sim.close()


def test_ctrl_graph_replays_match_eager():
    sc = S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=37)
    T = 20
    ctl = S.controller_params(sc, seed=12)
    gT = _loss_seed(sc, 13)
    eager = sim_for(sc, graphs=False)
    graph = sim_for(sc, graphs=True)
    say("ctrl_graph_eager")
    ref = _run(eager, sc, T, 8, ctl, gT)
    eager.sync_errors()
    for rep in range(3):
        say("ctrl_graph_replay", rep)
        out = _run(graph, sc, T, 8, ctl, gT)
        graph.sync_errors()
        torch.cuda.synchronize()
        assert err(to_np(out[0])[0], to_np(ref[0])[0]) < 1e-6
        assert err(out[1].cpu().numpy(), ref[1].cpu().numpy()) < 1e-6
        assert err(to_np(out[2])[0], to_np(ref[2])[0]) < 1e-5
        assert err(out[4].cpu().numpy(), ref[4].cpu().numpy()) < 1e-5
    eager.close()
    graph.close()


def test_ctrl_argument_errors():
    sc = S.tiny_2d(n=16, n_particles=40)
    comp, nc, W, b, target = S.controller_params(sc, seed=3, n_comp=2)
    sim = sim_for(sc)
    s0 = to_gpu(sc.state)
    say("ctrl_argument_errors")

    def call(comp_, nc_, W_):
        return sim.rollout_ctrl(s0, 4, _cuda(comp_, torch.int32), nc_, _cuda(W_), _cuda(b),
                                _cuda(target))

    bad = comp.copy()
    bad[3] = 2                                  # id beyond n_comp
    with pytest.raises(MPMError):
        call(bad, nc, W)
    empty = np.where(comp == 1, 0, comp).astype(np.int32)  # component 1 empty
    with pytest.raises(MPMError):
        call(empty, nc, W)
    nbig = 25                                   # 2 d n_comp > 96
    with pytest.raises(MPMError):
        call(comp, nbig, np.zeros((sc.n_act, 2 * (1 + 2 * nbig)), np.float32))
    call(comp, nc, W)                           # still usable afterwards
    sim.sync_errors()
    sim.close()
    two = sim_for([sc, sc])                     # one scene per context
    s2 = tuple(torch.cat([a, a], 1) for a in s0)
    with pytest.raises(MPMError):
        two.rollout_ctrl(s2, 4, _cuda(np.concatenate([comp, comp]), torch.int32), nc,
                         _cuda(np.zeros((2 * sc.n_act, W.shape[1]), np.float32)),
                         _cuda(np.zeros(2 * sc.n_act, np.float32)), _cuda(target))
    two.close()
