"""Pins of the oracle's per-particle materials (E_p and rho_p replacing the
scene's E and rho; m_p = rho_p V0) and of their gradients dL/dE_p,
dL/drho_p (the paper's co-design and system identification).

Pinned against: uniform fields equal to the scene constants reproduce the
scene rollout bit for bit; scaling every E_p and rho_p by one factor leaves
the motion unchanged (mass and stress scale together: p/m, G/m and the
grid velocities are invariant, gravity is an acceleration), so by Euler's
relation sum_p (E_p dL/dE_p + rho_p dL/drho_p) = 0; central differences of
whole rollouts."""
import numpy as np
import pytest

import oracle
from paper_1810_01054_amd import scenes as S
from tests.helpers import oscene, f64, rel_err


def _run(sc, E_p, rho_p, T, acts, gT=None):
    N = sc.n_particles
    gE, grho = np.zeros(N), np.zeros(N)
    os_ = oscene(sc, E_p=np.asarray(E_p, np.float64), rho_p=np.asarray(rho_p, np.float64),
                 gE_p=gE, grho_p=grho)
    st = f64(sc.state)
    g = gT if gT is not None else [np.zeros_like(a) for a in st]
    sT, g0, gact = oracle.rollout(os_, st, T, sc.act_id, acts, g)
    return sT, g0, gact, gE, grho


def _scene(dim, seed):
    sc = S.perturb(S.tiny_2d(n=16, n_particles=40, seed=seed) if dim == 2 else
                   S.tiny_3d(n=12, n_particles=30, seed=seed), seed + 1,
                   v_scale=0.3, C_scale=1.0, F_scale=0.05)
    E_p, rho_p = S.material_field(sc, seed + 2)
    return sc, E_p.astype(np.float64), rho_p.astype(np.float64)


def _loss_seed(sc, seed):
    rng = np.random.default_rng(seed)
    return [rng.normal(size=sc.x.shape), rng.normal(size=sc.v.shape),
            np.zeros(sc.C.shape), np.zeros(sc.F.shape)]


def test_uniform_fields_reproduce_the_scene_rollout():
    sc = S.tiny_2d(n=16, n_particles=40)
    T = 6
    acts = np.random.default_rng(1).uniform(-1, 1, size=(T, sc.n_act))
    gT = _loss_seed(sc, 2)
    ref = oracle.rollout(oscene(sc), f64(sc.state), T, sc.act_id, acts, gT)
    N = sc.n_particles
    got = _run(sc, np.full(N, sc.E), np.full(N, sc.rho), T, acts, gT)
    for a, r in zip(got[0] + got[1], ref[0] + ref[1]):
        assert np.array_equal(a, r)
    assert np.array_equal(got[2], ref[2])


@pytest.mark.parametrize("dim", [2, 3])
def test_scaling_mass_and_stiffness_together_leaves_the_motion(dim):
    sc, E_p, rho_p = _scene(dim, 3 + dim)
    T = 8
    acts = np.random.default_rng(5).uniform(-1, 1, size=(T, sc.n_act))
    a = _run(sc, E_p, rho_p, T, acts)[0]
    # actuation is a stress too (sigma = s diag(axis) enters P), so it scales
    b = _run(sc, 3.0 * E_p, 3.0 * rho_p, T, 3.0 * acts)[0]
    for x, y in zip(a, b):
        assert rel_err(y, x) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_euler_relation_of_the_material_gradients(dim):
    # L(alpha E, alpha rho, alpha s) = L: sum E dL/dE + rho dL/drho + s dL/ds = 0
    sc, E_p, rho_p = _scene(dim, 7 + dim)
    T = 8
    acts = np.random.default_rng(9).uniform(-1, 1, size=(T, sc.n_act))
    gT = _loss_seed(sc, 10)
    _, _, gact, gE, grho = _run(sc, E_p, rho_p, T, acts, gT)
    terms = np.concatenate([E_p * gE, rho_p * grho, (acts * gact).ravel()])
    assert abs(terms.sum()) <= 1e-10 * np.abs(terms).sum(), (terms.sum(), np.abs(terms).sum())
    assert np.abs(E_p * gE).sum() > 1e-3 * np.abs(terms).sum()       # not vacuous
    assert np.abs(rho_p * grho).sum() > 1e-3 * np.abs(terms).sum()


@pytest.mark.parametrize("dim", [2, 3])
def test_material_gradients_match_central_differences(dim):
    sc, E_p, rho_p = _scene(dim, 11 + dim)
    T = 8
    acts = np.random.default_rng(13).uniform(-1, 1, size=(T, sc.n_act))
    gT = _loss_seed(sc, 14)
    _, _, _, gE, grho = _run(sc, E_p, rho_p, T, acts, gT)

    def loss(E_, r_):
        sT = _run(sc, E_, r_, T, acts)[0]
        return sum(float((g * s).sum()) for g, s in zip(gT, sT))

    # relative steps of 1e-4: the E gradients are ~1e-5 against an O(1)
    # loss, so smaller steps drown in cancellation; truncation is O(h^2)
    for p in (0, 7, 19, sc.n_particles - 1):
        h = 1e-4 * E_p[p]
        Ep, Em = E_p.copy(), E_p.copy()
        Ep[p] += h
        Em[p] -= h
        fd = (loss(Ep, rho_p) - loss(Em, rho_p)) / (2 * h)
        assert abs(fd - gE[p]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gE).max()), (p, fd, gE[p])
        h = 1e-4 * rho_p[p]
        rp, rm = rho_p.copy(), rho_p.copy()
        rp[p] += h
        rm[p] -= h
        fd = (loss(E_p, rp) - loss(E_p, rm)) / (2 * h)
        assert abs(fd - grho[p]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(grho).max()), (p, fd, grho[p])
