"""Gradients through the torch.autograd path (actuation bank -> rollout with
checkpoint + recompute -> loss), against the FP64 oracle's reverse pass and
against central finite differences in FP32."""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_01054_amd import scenes as S
from paper_1810_01054_amd.autograd import act_bank, rollout
from tests.gpu_helpers import require_gpu, say, sim_for, to_gpu
from tests.helpers import oscene, f64, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _params(sc):
    t = lambda a: torch.tensor(np.ascontiguousarray(a, np.float32), device="cuda")
    return t(sc.freq), t(sc.amp), t(sc.phase)


def test_autograd_quadruped_vs_oracle_100_steps():
    """Half-size quadruped (32^3 grid, 63k particles, legs on the floor),
    100 substeps, k = 10: dL/d(amp, phase) and dL/dv0 of the centroid loss
    through torch.autograd against the oracle's FP64 adjoint."""
    sc = S.quadruped_3d(32, seed=1813, scale=0.5, name="quadruped_half")
    T, k = 100, 10
    say("autograd quadruped", sc.n_particles)
    freq, amp, phase = _params(sc)
    amp.requires_grad_(True)
    phase.requires_grad_(True)
    x0, v0, C0, F0 = to_gpu(sc.state)
    v0.requires_grad_(True)
    sim = sim_for(sc)
    act = act_bank(T, sc.dt, freq, amp, phase)
    xT, vT, CT, FT = rollout(sim, (x0, v0, C0, F0), act, T, k)
    loss = xT[0].mean()
    loss.backward()
    sim.sync_errors()

    os_ = oscene(sc)
    acts = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase)
    N = sc.n_particles
    gT = [np.zeros((3, N)), np.zeros((3, N)), np.zeros((9, N)), np.zeros((9, N))]
    gT[0][0] = 1.0 / N
    refT, ref0, ref_s = oracle.rollout(os_, f64(sc.state), T, sc.act_id,
                                       acts.astype(np.float32).astype(np.float64), gT)
    ga, gp = oracle.act_bank_bwd(T, sc.dt, sc.freq, sc.amp, sc.phase, ref_s)
    assert rel_err(xT.detach().cpu().numpy(), refT[0]) < 1e-5
    assert rel_err(v0.grad.cpu().numpy(), ref0[1]) < 1e-3
    e_amp = rel_err(amp.grad.cpu().numpy(), ga)
    e_phase = rel_err(phase.grad.cpu().numpy(), gp)
    say("dL/damp rel err", e_amp, "dL/dphase rel err", e_phase,
        "norms", np.linalg.norm(ga), np.linalg.norm(gp))
    assert e_amp < 1e-3 and e_phase < 1e-3


def test_c3_central_fd_on_8_actuation_parameters():
    """Full C3 (504,064 particles, 64^3, T = 512, k = 32): the autograd
    gradient of the centroid x w.r.t. 8 random actuation parameters against
    central differences in FP32 with h in {1e-2, 3e-3, 1e-3} |theta|; the
    best step of each parameter must agree within 5 % (FP32 forward noise
    bounds the FD accuracy: each parameter's error is allowed 5 % of its own
    gradient plus 1 % of the largest gradient component, since components far
    below the largest are under the FP32 FD noise), and the normwise error
    over the 8 within 2 %."""
    sc = S.config_3()
    T, k = 512, 32
    say("c3 fd", sc.n_particles)
    freq, amp, phase = _params(sc)
    x0, v0, C0, F0 = to_gpu(sc.state)
    sim = sim_for(sc)
    a_, p_ = amp.clone().requires_grad_(True), phase.clone().requires_grad_(True)
    act = act_bank(T, sc.dt, freq, a_, p_)
    xT = rollout(sim, (x0, v0, C0, F0), act, T, k)[0]
    xT[0].mean().backward()
    sim.sync_errors()
    grad = torch.cat([a_.grad.flatten(), p_.grad.flatten()]).cpu().numpy().astype(np.float64)
    theta = torch.cat([amp.flatten(), phase.flatten()])
    rng = np.random.default_rng(1813)
    pick = rng.choice(theta.numel(), 8, replace=False)

    def loss_at(th):
        n = amp.numel()
        a2 = th[:n].view_as(amp).contiguous()
        p2 = th[n:].view_as(phase).contiguous()
        with torch.no_grad():
            act2 = act_bank(T, sc.dt, freq, a2, p2)
            out = sim.rollout((x0, v0, C0, F0), act2, T, k)
        return float(out[0][0].double().mean())

    fd, an = [], []
    scale = float(np.abs(grad[pick]).max())
    for i in pick:
        best = None
        for hr in (1e-2, 3e-3, 1e-3):
            h = hr * max(abs(float(theta[i])), 1e-3)
            tp, tm = theta.clone(), theta.clone()
            tp[i] += h
            tm[i] -= h
            d = (loss_at(tp) - loss_at(tm)) / (2 * h)
            err = abs(d - grad[i])
            if best is None or err < best[0]:
                best = (err, d)
        say("param", int(i), "autograd", grad[i], "fd", best[1], "abs err", best[0])
        fd.append(best[1])
        an.append(grad[i])
        assert best[0] <= 5e-2 * abs(grad[i]) + 1e-2 * scale, (int(i), grad[i], best[1])
    assert rel_err(np.array(an), np.array(fd)) < 2e-2
