"""Pins of the oracle's closed-loop controller rollout (section IV, Control:
a^n = tanh(W z^n + b), z^n = target plus the mean position and velocity of
each component) against the open-loop rollout, numpy means and central
finite differences."""
import numpy as np
import pytest

import oracle
from paper_1810_01054_amd import scenes as S
from tests.helpers import oscene, f64, rel_err


def _setup(dim=2, seed=3, n_comp=2):
    sc = S.tiny_2d(n=16, n_particles=40, seed=seed) if dim == 2 else \
        S.tiny_3d(n=12, n_particles=30, seed=seed)
    rng = np.random.default_rng(seed)
    comp = rng.integers(0, n_comp, size=sc.n_particles).astype(np.int32)
    comp[: n_comp] = np.arange(n_comp)           # every component non-empty
    comp[n_comp] = -1                            # and one particle in none
    nz = dim * (1 + 2 * n_comp)
    W = rng.normal(size=(sc.n_act, nz)) * 0.6
    b = rng.normal(size=sc.n_act) * 0.3
    target = rng.uniform(0.3, 0.7, size=dim)
    return sc, comp, n_comp, W, b, target


def test_zero_gain_controller_is_the_open_loop_rollout():
    # W = 0: a^n = tanh(b) every substep, so the rollout and its reverse pass
    # must equal the open-loop ones; dL/db = sum_n g_act^n (1 - tanh(b)^2)
    sc, comp, n_comp, W, b, target = _setup()
    W = np.zeros_like(W)
    T = 6
    rng = np.random.default_rng(5)
    gT = [rng.normal(size=a.shape) for a in sc.state]
    ref_T, ref_0, ref_act = oracle.rollout(oscene(sc), f64(sc.state), T, sc.act_id,
                                           np.tile(np.tanh(b), (T, 1)), gT)
    sT, acts, g0, gW, gb = oracle.rollout_ctrl(oscene(sc), f64(sc.state), T, comp, n_comp,
                                               W, b, target, act_id=sc.act_id, gradT=gT)
    assert np.allclose(acts, np.tanh(b)[None, :], rtol=1e-15, atol=1e-16)
    for a, r in zip(sT, ref_T):   # (numpy's and libm's tanh may differ by an ulp)
        assert rel_err(a, r) < 1e-14
    for a, r in zip(g0, ref_0):
        assert rel_err(a, r) < 1e-13
    assert rel_err(gb, ref_act.sum(0) * (1 - np.tanh(b) ** 2)) < 1e-12


def test_first_actuation_from_numpy_means():
    sc, comp, n_comp, W, b, target = _setup(dim=3, seed=4, n_comp=3)
    _, acts = oracle.rollout_ctrl(oscene(sc), f64(sc.state), 1, comp, n_comp, W, b, target,
                                  act_id=sc.act_id)
    x, v = np.asarray(sc.x, np.float64), np.asarray(sc.v, np.float64)
    z = [target]
    for c in range(n_comp):
        m = comp == c
        z += [x[:, m].mean(1), v[:, m].mean(1)]
    z = np.concatenate(z)
    assert np.allclose(acts[0], np.tanh(W @ z + b), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_controller_gradients_match_central_differences(dim):
    sc, comp, n_comp, W, b, target = _setup(dim=dim, seed=6 + dim)
    T = 8
    rng = np.random.default_rng(11)
    gT = [rng.normal(size=a.shape) for a in sc.state]   # L = sum gT . S^T
    gT[2][:] = 0.0
    gT[3][:] = 0.0
    st = f64(sc.state)

    def loss(W_, b_, st_):
        sT, _ = oracle.rollout_ctrl(oscene(sc), st_, T, comp, n_comp, W_, b_, target,
                                    act_id=sc.act_id)
        return sum(float((g * s).sum()) for g, s in zip(gT, sT))

    _, _, g0, gW, gb = oracle.rollout_ctrl(oscene(sc), st, T, comp, n_comp, W, b, target,
                                           act_id=sc.act_id, gradT=gT)
    h = 1e-6
    picks = [(j, i) for j in range(W.shape[0]) for i in (0, dim, W.shape[1] - 1)]
    for j, i in picks:
        Wp, Wm = W.copy(), W.copy()
        Wp[j, i] += h
        Wm[j, i] -= h
        fd = (loss(Wp, b, st) - loss(Wm, b, st)) / (2 * h)
        assert abs(fd - gW[j, i]) <= 1e-6 * max(1.0, abs(fd)), (j, i, fd, gW[j, i])
    for j in range(b.size):
        bp, bm = b.copy(), b.copy()
        bp[j] += h
        bm[j] -= h
        fd = (loss(W, bp, st) - loss(W, bm, st)) / (2 * h)
        assert abs(fd - gb[j]) <= 1e-6 * max(1.0, abs(fd)), (j, fd, gb[j])
    # the state adjoint carries the controller's dependence on x and v
    for comp_ix, p in ((0, 0), (1, 3), (0, 7)):
        sp = [a.copy() for a in st]
        sm = [a.copy() for a in st]
        sp[comp_ix][0, p] += h
        sm[comp_ix][0, p] -= h
        fd = (loss(W, b, tuple(sp)) - loss(W, b, tuple(sm))) / (2 * h)
        assert abs(fd - g0[comp_ix][0, p]) <= 1e-6 * max(1.0, abs(fd)), (comp_ix, p)
