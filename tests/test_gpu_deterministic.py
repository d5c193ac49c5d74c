"""Deterministic mode (mpm_opts.deterministic): binned rollouts whose sums
run in a fixed order (a cell's particles ranked by index at binning and in
every scatter, dL/ds summed per actuator in a fixed order) are bitwise
reproducible: the same rollout twice, a captured graph against eager
launches, and rollouts with different checkpoint intervals (the reverse pass
then works from recomputed states) give identical bits.  The scenes keep
every particle within its tile box's slack (over the horizons used here no
particle drifts more than one cell), where no float atomics remain.  Each
case is also held to the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_01054_amd import scenes as S
from tests.helpers import oscene, f64, err
from tests.gpu_helpers import require_gpu, say, to_gpu, to_np, sim_for, check_state

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _seed(sc, seed):
    N, d = sc.n_particles, sc.dim
    rng = np.random.default_rng(seed)
    gx = np.zeros((d, N))
    gx[0] += 1.0 / N
    gx += rng.normal(size=(d, N)) / N
    return (gx.astype(np.float32), np.zeros((d, N), np.float32),
            np.zeros((d * d, N), np.float32), np.zeros((d * d, N), np.float32))


def _run(sim, sc, acts, T, k, gT):
    sT, g0, gact = sim.rollout(to_gpu(sc.state), torch.tensor(acts, device="cuda"), T,
                               ckpt_k=k, gT=to_gpu(gT))
    sim.sync_errors()
    return [t.detach().cpu().numpy() for t in (*sT, *g0, gact)]


def _same(a, b, what):
    for i, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), (what, i)


def _oracle_check(sc, acts, T, gT, out):
    refT, ref0, ref_act = oracle.rollout(oscene(sc), f64(sc.state), T, sc.act_id,
                                         acts.astype(np.float64), f64(gT))
    check_state([o.astype(np.float64) for o in out[:4]], refT, 1.0 / sc.n_grid,
                label=f"det {sc.name}")
    for c in range(4):
        assert err(out[4 + c], ref0[c]) < GRAD_TOL, ("xvCF"[c], err(out[4 + c], ref0[c]))
    assert err(out[8], ref_act) < GRAD_TOL


@pytest.mark.parametrize("case", ["2d_c1b", "3d_box"])
def test_deterministic_rollouts_repeat_bit_for_bit(case):
    if case == "2d_c1b":
        sc, T, k = S.config_1b(), 50, 10
    else:
        sc = S.perturb(S.box_3d(24, (6, 3, 7), (14, 9, 13), seed=36), 37, v_scale=0.5,
                       C_scale=0.5, F_scale=0.02)
        T, k = 23, 8
    acts = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
    gT = _seed(sc, 71)
    say("det repeat", case)
    det = sim_for(sc, deterministic=True)
    a = _run(det, sc, acts, T, k, gT)
    b = _run(det, sc, acts, T, k, gT)
    _same(a, b, "same context twice")
    memo = _run(det, sc, acts, T, 0, gT)
    _same(a, memo, f"k={k} vs memo")
    other = sim_for(sc, deterministic=True, graphs=True)
    for rep in range(3):
        c = _run(other, sc, acts, T, k, gT)
        _same(a, c, f"graph replay {rep}")
    _oracle_check(sc, acts, T, gT, a)
    det.close()
    other.close()


def test_deterministic_c2_checkpoint_invariance():
    """C2 (2D 256^2, 98,304 particles, 48 actuators) over 64 substeps: the
    memo tape, checkpoints every 16 and every 64 substeps give the same bits
    (64 substeps keep every particle within one cell of its bin)."""
    sc = S.config_2()
    T = 64
    acts = oracle.act_bank_fwd(T, sc.dt, sc.freq, sc.amp, sc.phase).astype(np.float32)
    gT = _seed(sc, 72)
    sim = sim_for(sc, deterministic=True)
    outs = {}
    for k in (0, 16, 64):
        say("det c2 k", k)
        outs[k] = _run(sim, sc, acts, T, k, gT)
    _same(outs[0], outs[16], "memo vs k=16")
    _same(outs[0], outs[64], "memo vs k=64")
    _oracle_check(sc, acts, T, gT, outs[64])
    sim.close()


def test_deterministic_mode_arguments():
    from paper_1810_01054_amd._lib import MPMError
    sc = S.config_1b()
    with pytest.raises(MPMError):
        sim_for(sc, deterministic=True, sort=False)
    with pytest.raises(MPMError):
        sim_for(sc, deterministic=True, scatter=1)
