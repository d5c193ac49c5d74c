"""Seeded synthetic scenes (inputs only).

This module draws random numbers and places particles; it holds none of the
simulation's arithmetic, so both the GPU path and the FP64 oracle can be fed
from it.  Every array is FP32 (what the GPU consumes); the oracle promotes the
same values to FP64.

Recipe (the paper benchmarks a falling cube and soft robots whose geometry it
does not publish, so these stand in for them):

* particles sit on a sub-cell lattice, ``ppa`` per axis per cell (2 -> 4 per
  cell in 2D, 8 in 3D), each jittered by U[-1/4, 1/4) dx per axis
  (``1/(2 ppa)`` of a cell in general);
* v = 0, C = 0, F = I unless a test asks for a perturbed state;
* material: E = 10, nu = 0.3, rho = 1, V0 = (dx/2)^d, dt = 1e-4, gravity
  -9.8 along y, sticky walls 3 nodes thick;
* actuation: every actuator j is driven by a bank of sinusoids
  s_j(t) = sum_k a_jk sin(2 pi f_k t + phi_jk); the generator only draws the
  parameters (a, f, phi), it never evaluates the bank.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

F32 = np.float32


@dataclass
class Scene:
    dim: int
    n_grid: int
    x: np.ndarray                  # [d][N] f32
    v: np.ndarray                  # [d][N] f32
    C: np.ndarray                  # [d*d][N] f32
    F: np.ndarray                  # [d*d][N] f32
    act_id: np.ndarray             # [N] int32, -1 = passive
    n_act: int
    amp: np.ndarray                # [n_act][n_freq] f32
    phase: np.ndarray              # [n_act][n_freq] f32
    freq: np.ndarray               # [n_freq] f32
    wall: int = 3
    dt: float = float(F32(1e-4))
    E: float = float(F32(10.0))
    nu: float = float(F32(0.3))
    rho: float = float(F32(1.0))
    V0: float = 0.0
    gravity: tuple = (0.0, float(F32(-9.8)), 0.0)
    act_axis: tuple = (0.0, 1.0, 0.0)
    name: str = ""
    bc: int = 0                    # wall nodes: 0 sticky, 1 friction projection
    friction: float = 0.0          # friction coefficient of the projection

    @property
    def n_particles(self) -> int:
        return int(self.x.shape[1])

    @property
    def state(self):
        return (self.x, self.v, self.C, self.F)

    def params(self) -> dict:
        """Physical parameters as plain Python floats (FP32-representable)."""
        return dict(dim=self.dim, n_grid=self.n_grid,
                    n_particles=self.n_particles, n_act=self.n_act,
                    wall=self.wall, dt=self.dt, E=self.E, nu=self.nu,
                    rho=self.rho, V0=self.V0, gravity=tuple(self.gravity),
                    act_axis=tuple(self.act_axis), bc=self.bc,
                    friction=self.friction)


def _f32(a) -> float:
    return float(F32(a))


def _lattice_block(rng, dim, n, lo_cell, hi_cell, ppa):
    """Particles on a ppa^d sub-cell lattice over cells [lo, hi) per axis,
    jittered by U[-1/(2 ppa), 1/(2 ppa)) of a cell.  Returns [d][N] f64 cell
    coordinates in cell units (not yet divided by n)."""
    axes = [np.arange(lo_cell[a] * ppa, hi_cell[a] * ppa) for a in range(dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    sub = np.stack([g.reshape(-1) for g in grids]).astype(np.float64)
    pos = (sub + 0.5) / ppa
    jit = rng.uniform(-0.5 / ppa, 0.5 / ppa, size=pos.shape)
    return pos + jit


def _finish(dim, n, pos_cells, act_id, n_act, amp, phase, freq, name,
            ppa=2, **kw) -> Scene:
    dx = 1.0 / n
    x = (pos_cells * dx).astype(F32)
    N = x.shape[1]
    v = np.zeros((dim, N), F32)
    C = np.zeros((dim * dim, N), F32)
    F = np.zeros((dim * dim, N), F32)
    for a in range(dim):
        F[a * dim + a] = 1.0
    V0 = _f32((dx / ppa) ** dim)
    return Scene(dim=dim, n_grid=n, x=x, v=v, C=C, F=F,
                 act_id=np.ascontiguousarray(act_id, np.int32), n_act=n_act,
                 amp=np.ascontiguousarray(amp, F32),
                 phase=np.ascontiguousarray(phase, F32),
                 freq=np.ascontiguousarray(freq, F32), V0=V0, name=name, **kw)


def block_2d(n=64, lo=(0.2, 0.1), hi=(0.45, 0.35), n_columns=4, seed=1811,
             name="block2d") -> Scene:
    """One 2D block, 4 particles per cell, actuators = equal-width vertical
    strips by initial x, each one sinusoid at 10 Hz with a ~ U[0.5, 2] and
    phi ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    lo_c = [int(round(lo[a] * n)) for a in range(2)]
    hi_c = [int(round(hi[a] * n)) for a in range(2)]
    pos = _lattice_block(rng, 2, n, lo_c, hi_c, 2)
    width = hi_c[0] - lo_c[0]
    col = np.floor((pos[0] - lo_c[0]) / width * n_columns).astype(np.int64)
    act_id = np.clip(col, 0, n_columns - 1).astype(np.int32)
    amp = rng.uniform(0.5, 2.0, size=(n_columns, 1))
    phase = rng.uniform(0.0, 2 * np.pi, size=(n_columns, 1))
    return _finish(2, n, pos, act_id, n_columns, amp, phase, [10.0], name)


def config_1a() -> Scene:
    """2D, 64^2, block [0.2,0.45]x[0.1,0.35]: 16x16 cells, N = 1,024."""
    return block_2d(64, (0.2, 0.1), (0.45, 0.35), seed=1811, name="c1a_2d64_1k")


def config_1b() -> Scene:
    """2D, 64^2, block [0.2,0.7]x[0.1,0.6]: 32x32 cells, N = 4,096."""
    return block_2d(64, (0.2, 0.1), (0.7, 0.6), seed=1812, name="c1b_2d64_4k")


def config_2(seed=1812) -> Scene:
    """2D, 256^2: six 64x64-cell blocks (3 columns x 2 rows), N = 98,304.
    Each block has 8 actuator groups (2 rows x 4 columns of its cells); each
    group is a bank of 4 sinusoids f_k = 10k Hz, a ~ U[-1, 1],
    phi ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    n = 256
    x0s = [0.05, 0.375, 0.70]
    pos_all, ids_all = [], []
    blk = 0
    for row in range(2):
        y0 = 4 + row * (64 + 2)
        for x0 in x0s:
            xj = int(rng.integers(-2, 3))
            xc = int(round(x0 * n)) + xj
            pos = _lattice_block(rng, 2, n, (xc, y0), (xc + 64, y0 + 64), 2)
            gx = np.clip(np.floor((pos[0] - xc) / 16.0), 0, 3).astype(np.int64)
            gy = np.clip(np.floor((pos[1] - y0) / 32.0), 0, 1).astype(np.int64)
            ids_all.append((blk * 8 + gy * 4 + gx).astype(np.int32))
            pos_all.append(pos)
            blk += 1
    pos = np.concatenate(pos_all, axis=1)
    act_id = np.concatenate(ids_all)
    n_act = 48
    freq = [10.0, 20.0, 30.0, 40.0]
    amp = rng.uniform(-1.0, 1.0, size=(n_act, 4))
    phase = rng.uniform(0.0, 2 * np.pi, size=(n_act, 4))
    return _finish(2, n, pos, act_id, n_act, amp, phase, freq, "c2_2d256_98k")


def quadruped_3d(n=64, seed=1813, scale=1.0, name="c3_3d64_504k") -> Scene:
    """3D quadruped, 8 particles per cell.  Cell boxes (at n = 64):
    body [6,58) x [26,46) x [10,54); four 14 x 22 x 14 legs at the body's
    corners over y in [4,26).  63,008 cells, N = 504,064.  16 actuators: the
    2 x 2 (x, z) quadrant columns of each leg, axis y, one 10 Hz sinusoid each
    with a ~ U[0.5, 2], phi ~ U[0, 2 pi).  ``scale`` shrinks the boxes (for
    smaller grids); the floor offset stays 4 cells."""
    rng = np.random.default_rng(seed)

    def sc(c):
        return int(round(c * scale))

    body = ((sc(6), 4 + sc(22), sc(10)), (sc(58), 4 + sc(42), sc(54)))
    legs = []
    for lx in (0, 1):
        for lz in (0, 1):
            x_lo = sc(6) if lx == 0 else sc(58) - sc(14)
            z_lo = sc(10) if lz == 0 else sc(54) - sc(14)
            legs.append(((x_lo, 4, z_lo),
                         (x_lo + sc(14), 4 + sc(22), z_lo + sc(14))))
    pos_all, ids_all = [], []
    pos = _lattice_block(rng, 3, n, body[0], body[1], 2)
    pos_all.append(pos)
    ids_all.append(-np.ones(pos.shape[1], np.int32))
    for li, (lo, hi) in enumerate(legs):
        pos = _lattice_block(rng, 3, n, lo, hi, 2)
        hx = (hi[0] - lo[0]) / 2.0
        hz = (hi[2] - lo[2]) / 2.0
        qx = np.clip(np.floor((pos[0] - lo[0]) / hx), 0, 1).astype(np.int64)
        qz = np.clip(np.floor((pos[2] - lo[2]) / hz), 0, 1).astype(np.int64)
        ids_all.append((li * 4 + qx * 2 + qz).astype(np.int32))
        pos_all.append(pos)
    pos = np.concatenate(pos_all, axis=1)
    act_id = np.concatenate(ids_all)
    amp = rng.uniform(0.5, 2.0, size=(16, 1))
    phase = rng.uniform(0.0, 2 * np.pi, size=(16, 1))
    return _finish(3, n, pos, act_id, 16, amp, phase, [10.0], name)


def config_3() -> Scene:
    return quadruped_3d(64, 1813, 1.0, "c3_3d64_504k")


def box_3d(n=32, lo=(8, 4, 8), hi=(16, 12, 16), n_columns=4, seed=1820,
           name="box3d") -> Scene:
    """One 3D box of cells [lo, hi), 8 particles per cell, actuators = equal
    x-strips, one 10 Hz sinusoid each."""
    rng = np.random.default_rng(seed)
    pos = _lattice_block(rng, 3, n, lo, hi, 2)
    width = hi[0] - lo[0]
    col = np.floor((pos[0] - lo[0]) / width * n_columns).astype(np.int64)
    act_id = np.clip(col, 0, n_columns - 1).astype(np.int32)
    amp = rng.uniform(0.5, 2.0, size=(n_columns, 1))
    phase = rng.uniform(0.0, 2 * np.pi, size=(n_columns, 1))
    return _finish(3, n, pos, act_id, n_columns, amp, phase, [10.0], name)


def grid_choices_2d(N: int, sizes=(64, 128, 256), ppc=4, fill=0.4):
    """Grids among ``sizes`` whose interior holds N particles within ``fill``
    of the interior cells (walls 3 nodes thick)."""
    return [n for n in sizes if N <= fill * (n - 6) ** 2 * ppc]


def grid_choices_3d(N: int, sizes=(32, 48, 64), ppc=8, fill=0.4):
    return [n for n in sizes if N <= fill * (n - 6) ** 3 * ppc]


def floor_block(rng, dim, n, N, n_columns=4, name="") -> Scene:
    """One block of about N particles resting on the floor (bottom at 4 dx),
    aspect ratio U[0.5, 2], placed at a random x (and z) inside the walls."""
    ppc = 2 ** dim
    cells = max(1, int(round(N / ppc)))
    aspect = rng.uniform(0.5, 2.0)
    inner = n - 8
    if dim == 2:
        w = int(np.clip(round(np.sqrt(cells * aspect)), 1, inner))
        h = int(np.clip(round(cells / w), 1, inner - 1))
        x_lo = 4 + int(rng.integers(0, max(1, inner - w + 1)))
        lo, hi = (x_lo, 4), (x_lo + w, 4 + h)
    else:
        w = int(np.clip(round((cells * aspect) ** (1.0 / 3.0)), 1, inner))
        dpt = w
        h = int(np.clip(round(cells / (w * dpt)), 1, inner - 1))
        x_lo = 4 + int(rng.integers(0, max(1, inner - w + 1)))
        z_lo = 4 + int(rng.integers(0, max(1, inner - dpt + 1)))
        lo, hi = (x_lo, 4, z_lo), (x_lo + w, 4 + h, z_lo + dpt)
    pos = _lattice_block(rng, dim, n, lo, hi, 2)
    width = hi[0] - lo[0]
    col = np.floor((pos[0] - lo[0]) / width * n_columns).astype(np.int64)
    act_id = np.clip(col, 0, n_columns - 1).astype(np.int32)
    amp = rng.uniform(0.5, 2.0, size=(n_columns, 1))
    phase = rng.uniform(0.0, 2 * np.pi, size=(n_columns, 1))
    return _finish(dim, n, pos, act_id, n_columns, amp, phase, [10.0], name)


def config_4(n_scenes=64, seed=1814) -> List[Scene]:
    """64 independent 2D scenes, N log-uniform in [2k, 60k], grid drawn
    uniformly among {64, 128, 256}^2 that hold N within 40 % of the interior."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_scenes):
        N = int(np.exp(rng.uniform(np.log(2000), np.log(60000))))
        choices = grid_choices_2d(N)
        n = int(choices[int(rng.integers(0, len(choices)))])
        out.append(floor_block(rng, 2, n, N, name=f"c4_s{s}"))
    return out


@dataclass
class Request:
    arrival: float
    scene: Scene
    T: int


def config_5(n_requests=1000, rate=10.0, seed=1815, max_3d=500_000):
    """Poisson arrivals of forward+gradient rollout requests: half 2D
    (N log-uniform [4k, 100k], grids {64,128,256}^2), half 3D (N log-uniform
    [50k, max_3d], grids {32,48,64}^3), T ~ U{100..500}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < 0.5:
            N = int(np.exp(rng.uniform(np.log(4000), np.log(100000))))
            ch = grid_choices_2d(N)
            n = int(ch[int(rng.integers(0, len(ch)))])
            sc = floor_block(rng, 2, n, N, name=f"c5_r{r}_2d")
        else:
            N = int(np.exp(rng.uniform(np.log(50000), np.log(max_3d))))
            ch = grid_choices_3d(N)
            n = int(ch[int(rng.integers(0, len(ch)))])
            sc = floor_block(rng, 3, n, N, name=f"c5_r{r}_3d")
        T = int(rng.integers(100, 501))
        out.append(Request(arrival=t, scene=sc, T=T))
    return out


def perturb(scene: Scene, seed: int, v_scale=0.5, C_scale=2.0, F_scale=0.05,
            act_scale=1.0) -> Scene:
    """A copy of ``scene`` with random v, C and F = I + noise, for tests that
    need every term of the substep to be non-zero."""
    rng = np.random.default_rng(seed)
    d, N = scene.dim, scene.n_particles
    out = Scene(**{**scene.__dict__})
    out.v = rng.uniform(-v_scale, v_scale, size=(d, N)).astype(F32)
    out.C = rng.uniform(-C_scale, C_scale, size=(d * d, N)).astype(F32)
    F = rng.uniform(-F_scale, F_scale, size=(d * d, N))
    for a in range(d):
        F[a * d + a] += 1.0
    out.F = F.astype(F32)
    out.x = scene.x.copy()
    out.act_id = scene.act_id.copy()
    return out


def tiny_2d(n=16, n_particles=40, seed=7, n_act=3, spread=(0.35, 0.65)) -> Scene:
    """A handful of random particles in the middle of a small 2D grid, with
    random v, C, F near I and random actuator ids (tests of the reverse pass)."""
    return _tiny(2, n, n_particles, seed, n_act, spread)


def tiny_3d(n=12, n_particles=24, seed=8, n_act=3, spread=(0.35, 0.65)) -> Scene:
    return _tiny(3, n, n_particles, seed, n_act, spread)


def _tiny(dim, n, N, seed, n_act, spread) -> Scene:
    rng = np.random.default_rng(seed)
    pos = rng.uniform(spread[0] * n, spread[1] * n, size=(dim, N))
    act_id = rng.integers(-1, n_act, size=N).astype(np.int32)
    amp = rng.uniform(0.5, 2.0, size=(n_act, 1))
    phase = rng.uniform(0.0, 2 * np.pi, size=(n_act, 1))
    sc = _finish(dim, n, pos, act_id, n_act, amp, phase, [10.0], f"tiny{dim}d")
    return perturb(sc, seed + 1000)


def shuffled(scene: Scene, seed: int) -> Scene:
    """The same particles in a random order (for order-independence tests)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(scene.n_particles)
    out = Scene(**{**scene.__dict__})
    out.x = np.ascontiguousarray(scene.x[:, perm])
    out.v = np.ascontiguousarray(scene.v[:, perm])
    out.C = np.ascontiguousarray(scene.C[:, perm])
    out.F = np.ascontiguousarray(scene.F[:, perm])
    out.act_id = np.ascontiguousarray(scene.act_id[perm])
    return out


def controller_params(scene: Scene, seed: int, n_comp: Optional[int] = None,
                      w_scale: float = 0.6, b_scale: float = 0.3):
    """Seeded parameters of a closed-loop controller a = tanh(W z + b) over
    ``scene``: components (the robot's parts whose mean position and velocity
    the controller reads) are the actuator groups when ``n_comp`` is None
    (passive particles in none), else uniform draws over n_comp components
    with every component non-empty and the last particle in none.
    W ~ N(0, w_scale^2) of shape [n_act][d (1 + 2 n_comp)], b ~ N(0,
    b_scale^2), target ~ U[0.3, 0.7)^d.  Returns (comp_id int32 [N], n_comp,
    W, b, target), all FP32."""
    rng = np.random.default_rng(seed)
    N, d = scene.n_particles, scene.dim
    if n_comp is None:
        comp = np.asarray(scene.act_id, np.int32).copy()
        n_comp = scene.n_act
    else:
        comp = rng.integers(0, n_comp, size=N).astype(np.int32)
        comp[:n_comp] = np.arange(n_comp, dtype=np.int32)
        comp[-1] = -1
    nz = d * (1 + 2 * n_comp)
    W = (rng.normal(size=(scene.n_act, nz)) * w_scale).astype(F32)
    b = (rng.normal(size=scene.n_act) * b_scale).astype(F32)
    target = rng.uniform(0.3, 0.7, size=d).astype(F32)
    return comp, n_comp, W, b, target


def wall_contact(dim: int = 2, n: int = 16, n_particles: int = 40, seed: int = 9,
                 friction: float = 0.3, speed: float = 1.5, n_act: int = 2) -> Scene:
    """A small body pressed into the corner of the floor and the low-x wall,
    with the friction-projection boundary (bc = 1): particles uniform over
    cells [2.6, 5.5) on every axis (so their stencils reach the 3-node wall
    bands of the floor and of the x = 0 wall), velocity toward the floor and
    the wall with a tangential part, v ~ speed * (-0.6, -1, 0.4) + N(0,
    0.1^2) per component, C = 0, F = I + N(0, 0.02^2); actuators by x half."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(2.6, 5.5, size=(dim, n_particles))   # in cells
    dirn = np.array([-0.6, -1.0, 0.4][:dim])
    v = speed * dirn[:, None] + rng.normal(scale=0.1, size=(dim, n_particles))
    F = np.tile(np.eye(dim).reshape(-1, 1), (1, n_particles))
    F = F + rng.normal(scale=0.02, size=F.shape)
    act_id = (pos[0] >= 4.05).astype(np.int32) % max(n_act, 1)
    amp = rng.uniform(0.5, 2.0, size=(n_act, 1))
    phase = rng.uniform(0.0, 2 * np.pi, size=(n_act, 1))
    sc = _finish(dim, n, pos, act_id, n_act, amp, phase, [10.0], f"contact{dim}d")
    sc.v = v.astype(F32)
    sc.F = F.astype(F32)
    sc.bc, sc.friction = 1, _f32(friction)
    return sc


def material_field(scene: Scene, seed: int, E_spread: float = 0.5,
                   rho_spread: float = 0.3):
    """Seeded per-particle materials (a stiffness and density field for
    co-design / identification): E_p = E (1 + U[-E_spread, E_spread)),
    rho_p = rho (1 + U[-rho_spread, rho_spread)), FP32 [N] each."""
    rng = np.random.default_rng(seed)
    N = scene.n_particles
    E_p = scene.E * (1.0 + rng.uniform(-E_spread, E_spread, size=N))
    rho_p = scene.rho * (1.0 + rng.uniform(-rho_spread, rho_spread, size=N))
    return E_p.astype(F32), rho_p.astype(F32)


def analytic_block(kind: str, seed: int = 61) -> Scene:
    """The analytic accuracy cases of section IV (Table III), as a 3D block
    of 5 x 4 x 5 cells (800 particles) on a 32^3 grid sliding along x at
    0.5: "A1" in free flight (no gravity, lifted clear of the walls); "A2"
    pressed into a friction-less floor (gravity, v_y = -0.3, friction
    projection with c = 0).  In both, the centroid's x after T substeps
    moves by exactly T dt per unit of a uniform initial x-velocity shift."""
    sc = box_3d(32, (12, 4, 12), (17, 8, 17), seed=seed, name=f"analytic_{kind}")
    sc.v[0, :] = 0.5
    if kind == "A1":
        sc.gravity = (0.0, 0.0, 0.0)
        sc.x[1, :] += F32(6 / 32)
    elif kind == "A2":
        sc.bc, sc.friction = 1, 0.0
        sc.v[1, :] = -0.3
    else:
        raise ValueError(kind)
    return sc
