"""Independent FP64 PyTorch (CPU) re-implementation of the forward substep.

Test-only.  It is written separately from the C oracle (weights as
polynomials in the fractional offset, vectorised scatter with index_add_,
torch.linalg for det/inverse) so that torch.autograd of it can check the
oracle's hand-derived reverse pass.  Shares no code with the oracle or with
the HIP library.
"""
from __future__ import annotations

import torch


def _mats(A, d):
    # [d*d][N] -> [N][d][d]
    return A.transpose(0, 1).reshape(-1, d, d)


def _flat(M, d):
    return M.reshape(-1, d * d).transpose(0, 1)


def step(params, x, v, C, F, act, act_id):
    d = params["dim"]
    n = params["n_grid"]
    dt, E, nu = params["dt"], params["E"], params["nu"]
    rho, V0, wall = params["rho"], params["V0"], params["wall"]
    g = torch.tensor(params["gravity"][:d], dtype=torch.float64)
    axis = torch.tensor(params["act_axis"][:d], dtype=torch.float64)
    dx = 1.0 / n
    Dinv = 4.0 * n * n
    mu = E / (2 * (1 + nu))
    la = E * nu / ((1 + nu) * (1 - 2 * nu))
    mp = rho * V0
    N = x.shape[1]
    xs = x * n - 0.5
    base = torch.floor(xs.detach()).long()            # [d][N]
    fx = x * n - base.double()                          # [d][N] in [0.5, 1.5)
    w = [0.5 * (1.5 - fx) ** 2, 0.75 - (fx - 1.0) ** 2, 0.5 * (fx - 0.5) ** 2]

    Fm, Cm = _mats(F, d), _mats(C, d)
    J = torch.linalg.det(Fm)
    FiT = torch.linalg.inv(Fm).transpose(1, 2)
    P = mu * (Fm - FiT) + la * torch.log(J)[:, None, None] * FiT
    ids = torch.as_tensor(act_id, dtype=torch.long)
    s = torch.where(ids >= 0, act[ids.clamp(min=0)], torch.zeros((), dtype=torch.float64))
    sigma = s[:, None] * axis[None, :]                  # [N][d]
    Pt = P + Fm * sigma[:, None, :]
    G = -Dinv * dt * V0 * Pt @ Fm.transpose(1, 2) + mp * Cm

    nn = n ** d
    m_grid = torch.zeros(nn, dtype=torch.float64)
    p_grid = torch.zeros(nn, d, dtype=torch.float64)
    offsets = [(a, b) for a in range(3) for b in range(3)] if d == 2 else \
        [(a, b, c) for a in range(3) for b in range(3) for c in range(3)]
    stencil = []
    for off in offsets:
        Nw = torch.ones(N, dtype=torch.float64)
        idx = torch.zeros(N, dtype=torch.long)
        delta = []
        for a in range(d):
            Nw = Nw * w[off[a]][a]
            node = base[a] + off[a]
            idx = idx * n + node
            delta.append(node.double() * dx - x[a])
        delta = torch.stack(delta, 1)                   # [N][d]
        stencil.append((Nw, idx, delta))
        m_grid = m_grid.index_add(0, idx, Nw * mp)
        mom = mp * v.transpose(0, 1) + (G @ delta[:, :, None])[:, :, 0]
        p_grid = p_grid.index_add(0, idx, Nw[:, None] * mom)

    pos = torch.stack(torch.meshgrid(*[torch.arange(n)] * d, indexing="ij"), -1).reshape(-1, d)
    wall_mask = ((pos < wall) | (pos >= n - wall)).any(1)
    has_m = m_grid > 0
    m_safe = torch.where(has_m, m_grid, torch.ones_like(m_grid))
    vg = torch.where(has_m[:, None], p_grid / m_safe[:, None] + dt * g[None, :],
                     torch.zeros_like(p_grid))
    vg = torch.where(wall_mask[:, None], torch.zeros_like(vg), vg)

    vp = torch.zeros(N, d, dtype=torch.float64)
    B = torch.zeros(N, d, d, dtype=torch.float64)
    for Nw, idx, delta in stencil:
        vi = vg[idx]
        vp = vp + Nw[:, None] * vi
        B = B + Nw[:, None, None] * vi[:, :, None] * delta[:, None, :]
    C1 = Dinv * B
    I = torch.eye(d, dtype=torch.float64)[None]
    F1 = (I + dt * C1) @ Fm
    x1 = x + dt * vp.transpose(0, 1)
    return x1, vp.transpose(0, 1).contiguous(), _flat(C1, d), _flat(F1, d), (m_grid, p_grid, vg)
