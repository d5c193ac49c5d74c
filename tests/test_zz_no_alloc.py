"""The allocation-free single substep (mpm_step_forward_noalloc) against the
context path (mpm_step_forward) on the same inputs: two calls in a row, the
second on a smaller scene (the static region keeps the first call's grid,
so the second shows that what must start at zero is cleared).  Both paths
run the same P2G, grid and G2P kernels, but the scatter adds in LDS- and
global-atomic arrival order, so they agree to the FP32 single-step bound
used against the oracle (2e-5, normwise and per element); each is also
checked against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_01054_amd import scenes as S
from paper_1810_01054_amd.sim import step_forward_noalloc
from tests.helpers import oscene, f64, err
from tests.gpu_helpers import require_gpu, say, to_gpu, to_np, sim_for

pytestmark = pytest.mark.gpu

STEP_TOL = 2e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _pert(sc, seed):
    return S.perturb(sc, seed, v_scale=0.3, C_scale=0.5, F_scale=0.02)


def _one(sc, act):
    st = to_gpu(sc.state)
    ids = torch.tensor(sc.act_id, dtype=torch.int32, device="cuda")
    out = tuple(torch.full_like(t, float("nan")) for t in st)
    e = torch.zeros(1, dtype=torch.int32, device="cuda")
    step_forward_noalloc(sc.params(), st, torch.tensor(act, device="cuda"), out, e, ids)
    sim = sim_for(sc)
    ref_ctx = sim.step_forward(st, torch.tensor(act, device="cuda"))
    sim.sync_errors()
    torch.cuda.synchronize()
    assert int(e.item()) == 0
    got, ctx = to_np(out), to_np(ref_ctx)
    ref = oracle.step_fwd(oscene(sc), f64(sc.state), sc.act_id, act.astype(np.float64))
    for k in range(4):
        assert err(got[k], ctx[k]) < STEP_TOL, ("xvCF"[k], err(got[k], ctx[k]))
        assert err(got[k], ref[k]) < STEP_TOL, ("xvCF"[k], err(got[k], ref[k]))
    sim.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_noalloc_step_matches_context_step_twice(dim):
    if dim == 3:
        big = _pert(S.box_3d(32, (5, 4, 6), (20, 16, 19), seed=61), 62)
        small = _pert(S.box_3d(16, (5, 4, 5), (10, 9, 10), seed=63), 64)
    else:
        big = _pert(S.config_1b(), 65)
        small = _pert(S.tiny_2d(n=16, n_particles=40), 66)
    for sc in (big, small):
        say("noalloc", dim, sc.name, sc.n_particles, sc.n_grid)
        act = np.linspace(-1.0, 1.5, max(sc.n_act, 1)).astype(np.float32)[:sc.n_act]
        _one(sc, act)


def test_noalloc_rejects_sizes_beyond_its_region_and_bad_ids():
    from paper_1810_01054_amd._lib import MPMError
    sc = S.box_3d(16, (5, 4, 5), (10, 9, 10), seed=67)
    p = sc.params()
    st = to_gpu(sc.state)
    out = tuple(torch.empty_like(t) for t in st)
    e = torch.zeros(1, dtype=torch.int32, device="cuda")
    act = torch.zeros(sc.n_act, device="cuda")
    big = dict(p, n_grid=65)  # 65^3 nodes > MPM_NOALLOC_MAX_NODES
    with pytest.raises(MPMError):
        step_forward_noalloc(big, st, act, out, e)
    # an actuator id outside [-1, n_act) is reported in the error word and
    # the particle is taken as passive
    ids = torch.tensor(sc.act_id, dtype=torch.int32, device="cuda")
    ids[0] = sc.n_act
    say("noalloc bad id")
    step_forward_noalloc(p, st, act, out, e, ids)
    torch.cuda.synchronize()
    assert int(e.item()) & 8
