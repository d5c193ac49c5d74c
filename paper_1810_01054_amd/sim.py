"""Python face of libmpm: a context over a batch of scenes, with torch tensors
for device memory and the current torch stream for ordering.

Every method marshals arguments into one C-ABI call; no arithmetic of the
method runs here.  Particle state tensors are FP32, contiguous, on the GPU,
shaped like the C layout: x, v [d, N_tot], C, F [d*d, N_tot].
"""
from __future__ import annotations

import ctypes
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import check

StateT = Tuple[torch.Tensor, torch.Tensor, torch.Tensor, torch.Tensor]


def _stream_ptr(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_tensor(t: torch.Tensor, shape, name):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")


def scene_struct(p: dict) -> _lib.Scene:
    s = _lib.Scene()
    s.dim, s.n_grid, s.n_particles = p["dim"], p["n_grid"], p["n_particles"]
    s.n_act, s.wall, s.bc = p.get("n_act", 0), p.get("wall", 3), p.get("bc", 0)
    s.friction = p.get("friction", 0.0)
    s.dt, s.E, s.nu = p["dt"], p["E"], p["nu"]
    s.rho, s.V0 = p["rho"], p["V0"]
    g = p.get("gravity", (0.0, -9.8, 0.0))
    ax = p.get("act_axis", (0.0, 1.0, 0.0))
    for k in range(3):
        s.gravity[k] = g[k]
        s.act_axis[k] = ax[k]
    return s


class Simulator:
    """A libmpm context over ``scenes`` (dicts with the mpm_scene fields, e.g.
    ``paper_1810_01054_amd.scenes.Scene.params()``)."""

    def __init__(self, scenes: Sequence[dict], act_id: Optional[np.ndarray] = None,
                 tile: int = 0, sort: bool = True, scatter: int = 0,
                 recompute_grids: bool = False, graphs: bool = False, stream=None,
                 fusion: int = 0, deterministic: bool = False, persistent: bool = False,
                 rebin: int = 0):
        self.L = _lib.lib()
        self.scenes = [dict(s) for s in scenes]
        self.dim = self.scenes[0]["dim"]
        arr = (_lib.Scene * len(scenes))(*[scene_struct(s) for s in self.scenes])
        ids = None
        if act_id is not None:
            ids_np = np.ascontiguousarray(act_id, dtype=np.int32)
            self._ids = ids_np
            ids = ids_np.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        opts = _lib.Opts()
        opts.tile, opts.sort, opts.scatter = tile, int(bool(sort)), scatter
        opts.recompute_grids = int(bool(recompute_grids))
        opts.graphs = int(bool(graphs))
        opts.fusion = int(fusion)
        opts.deterministic = int(bool(deterministic))
        opts.persistent = int(bool(persistent))
        opts.rebin = int(rebin)  # 0 off, 1 (or True) every checkpoint, 2 on overflow
        self.ctx = ctypes.c_void_p()
        self._stream = stream
        check(self.L.mpm_init(ctypes.byref(self.ctx), arr, len(scenes), ids,
                              _stream_ptr(stream), ctypes.byref(opts)), "mpm_init")
        n, na, g = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        check(self.L.mpm_info(self.ctx, ctypes.byref(n), ctypes.byref(na), ctypes.byref(g)))
        self.N, self.n_act, self.G = n.value, na.value, g.value

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            self.L.mpm_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        check(self.L.mpm_set_stream(self.ctx, _stream_ptr(self._stream)))

    # -- helpers -------------------------------------------------------------
    def empty_state(self, device="cuda") -> StateT:
        d, N = self.dim, self.N
        return (torch.empty(d, N, device=device), torch.empty(d, N, device=device),
                torch.empty(d * d, N, device=device), torch.empty(d * d, N, device=device))

    def zeros_state(self, device="cuda") -> StateT:
        return tuple(torch.zeros_like(t) for t in self.empty_state(device))

    def _state(self, s: StateT, name: str) -> _lib.State:
        d, N = self.dim, self.N
        shapes = [(d, N), (d, N), (d * d, N), (d * d, N)]
        for t, sh, nm in zip(s, shapes, "xvCF"):
            _check_tensor(t, sh, f"{name}.{nm}")
        return _lib.State(*[t.data_ptr() for t in s])

    def _act(self, act: Optional[torch.Tensor], rows: Optional[int]):
        if self.n_act == 0:
            return None
        shape = (self.n_act,) if rows is None else (rows, self.n_act)
        _check_tensor(act, shape, "act")
        return _ptr(act)

    # -- C ABI ---------------------------------------------------------------
    def step_forward(self, s: StateT, act: Optional[torch.Tensor] = None,
                     out: Optional[StateT] = None) -> StateT:
        self._sync_stream()
        out = out if out is not None else self.empty_state()
        a, o = self._state(s, "s_n"), self._state(out, "s_np1")
        check(self.L.mpm_step_forward(self.ctx, ctypes.byref(a), self._act(act, None),
                                      ctypes.byref(o)), "mpm_step_forward")
        return out

    def step_backward(self, s: StateT, act: Optional[torch.Tensor], g_next: StateT,
                      g_act: Optional[torch.Tensor] = None,
                      out: Optional[StateT] = None) -> StateT:
        self._sync_stream()
        out = out if out is not None else self.empty_state()
        a, g1, g0 = (self._state(s, "s_n"), self._state(g_next, "g_np1"),
                     self._state(out, "g_n"))
        if g_act is not None:
            _check_tensor(g_act, (self.n_act,), "g_act")
        check(self.L.mpm_step_backward(self.ctx, ctypes.byref(a), self._act(act, None),
                                       ctypes.byref(g1), ctypes.byref(g0), _ptr(g_act)),
              "mpm_step_backward")
        return out

    def rollout(self, s0: StateT, act: Optional[torch.Tensor], T: int, ckpt_k: int = 0,
                gT: Optional[StateT] = None):
        """Forward T substeps (tape kept).  With gT also the reverse pass:
        returns (sT, g0, g_act)."""
        self._sync_stream()
        sT = self.empty_state()
        a0, aT = self._state(s0, "s0"), self._state(sT, "sT")
        act_p = self._act(act, T) if T > 0 else None
        if gT is None:
            check(self.L.mpm_rollout(self.ctx, T, ckpt_k, ctypes.byref(a0), act_p,
                                     ctypes.byref(aT), None, None, None), "mpm_rollout")
            return sT
        g0 = self.empty_state()
        g_act = torch.empty(T, self.n_act, device="cuda") if self.n_act else None
        gg, g00 = self._state(gT, "gT"), self._state(g0, "g0")
        check(self.L.mpm_rollout(self.ctx, T, ckpt_k, ctypes.byref(a0), act_p,
                                 ctypes.byref(aT), ctypes.byref(gg), ctypes.byref(g00),
                                 _ptr(g_act)), "mpm_rollout")
        return sT, g0, g_act

    def rollout_backward(self, gT: StateT, T: int):
        self._sync_stream()
        g0 = self.empty_state()
        g_act = torch.empty(T, self.n_act, device="cuda") if self.n_act else None
        gg, g00 = self._state(gT, "gT"), self._state(g0, "g0")
        check(self.L.mpm_rollout_backward(self.ctx, ctypes.byref(gg), ctypes.byref(g00),
                                          _ptr(g_act)), "mpm_rollout_backward")
        return g0, g_act

    def _controller(self, comp_id: torch.Tensor, n_comp: int, W: torch.Tensor,
                    b: torch.Tensor, target: torch.Tensor) -> _lib.Controller:
        nz = self.dim * (1 + 2 * n_comp)
        if comp_id.dtype != torch.int32 or not comp_id.is_cuda or \
                not comp_id.is_contiguous() or tuple(comp_id.shape) != (self.N,):
            raise ValueError(f"comp_id must be a contiguous cuda int32 tensor of shape ({self.N},)")
        _check_tensor(W, (self.n_act, nz), "W")
        _check_tensor(b, (self.n_act,), "b")
        _check_tensor(target, (self.dim,), "target")
        return _lib.Controller(n_comp, 0, comp_id.data_ptr(), W.data_ptr(), b.data_ptr(),
                               target.data_ptr())

    def rollout_ctrl(self, s0: StateT, T: int, comp_id: torch.Tensor, n_comp: int,
                     W: torch.Tensor, b: torch.Tensor, target: torch.Tensor,
                     ckpt_k: int = 0, gT: Optional[StateT] = None):
        """Closed-loop rollout a^n = tanh(W z^n + b) (mpm_rollout_ctrl).
        Returns (sT, act); with gT (sT, act, g0, g_act, g_W, g_b)."""
        self._sync_stream()
        ctl = self._controller(comp_id, n_comp, W, b, target)
        sT = self.empty_state()
        act = torch.empty(T, self.n_act, device="cuda")
        a0, aT = self._state(s0, "s0"), self._state(sT, "sT")
        if gT is None:
            check(self.L.mpm_rollout_ctrl(self.ctx, T, ckpt_k, ctypes.byref(a0),
                                          ctypes.byref(ctl), ctypes.byref(aT), _ptr(act),
                                          None, None, None, None, None), "mpm_rollout_ctrl")
            return sT, act
        g0 = self.empty_state()
        g_act = torch.empty(T, self.n_act, device="cuda")
        g_W, g_b = torch.empty_like(W), torch.empty_like(b)
        gg, g00 = self._state(gT, "gT"), self._state(g0, "g0")
        check(self.L.mpm_rollout_ctrl(self.ctx, T, ckpt_k, ctypes.byref(a0), ctypes.byref(ctl),
                                      ctypes.byref(aT), _ptr(act), ctypes.byref(gg),
                                      ctypes.byref(g00), _ptr(g_act), _ptr(g_W), _ptr(g_b)),
              "mpm_rollout_ctrl")
        return sT, act, g0, g_act, g_W, g_b

    def rollout_ctrl_backward(self, gT: StateT, T: int, nz: int):
        self._sync_stream()
        g0 = self.empty_state()
        g_act = torch.empty(T, self.n_act, device="cuda")
        g_W = torch.empty(self.n_act, nz, device="cuda")
        g_b = torch.empty(self.n_act, device="cuda")
        gg, g00 = self._state(gT, "gT"), self._state(g0, "g0")
        check(self.L.mpm_rollout_ctrl_backward(self.ctx, ctypes.byref(gg), ctypes.byref(g00),
                                               _ptr(g_act), _ptr(g_W), _ptr(g_b)),
              "mpm_rollout_ctrl_backward")
        return g0, g_act, g_W, g_b

    def set_materials(self, E_p: Optional[torch.Tensor] = None,
                      rho_p: Optional[torch.Tensor] = None):
        """Per-particle Young's modulus / density [N] (None: the scene's)."""
        self._sync_stream()
        for t, nm in ((E_p, "E_p"), (rho_p, "rho_p")):
            if t is not None:
                _check_tensor(t, (self.N,), nm)
        self._mat = (E_p, rho_p)  # kept alive until the library has copied them
        check(self.L.mpm_set_materials(self.ctx, _ptr(E_p), _ptr(rho_p)), "mpm_set_materials")

    def material_grad(self):
        """(dL/dE_p, dL/drho_p) [N] of the last reverse pass."""
        self._sync_stream()
        gE = torch.empty(self.N, device="cuda")
        grho = torch.empty(self.N, device="cuda")
        check(self.L.mpm_material_grad(self.ctx, _ptr(gE), _ptr(grho)), "mpm_material_grad")
        return gE, grho

    def get_grid(self):
        self._sync_stream()
        m = torch.empty(self.G, device="cuda")
        p = torch.empty(self.dim, self.G, device="cuda")
        v = torch.empty(self.dim, self.G, device="cuda")
        check(self.L.mpm_get_grid(self.ctx, _ptr(m), _ptr(p), _ptr(v)), "mpm_get_grid")
        return m, p, v

    def set_horizons(self, t_end=None):
        """mpm_set_horizons: scene s is held fixed from substep t_end[s] on
        (None removes the horizons)."""
        if t_end is None:
            check(self.L.mpm_set_horizons(self.ctx, None), "mpm_set_horizons")
            return
        arr = np.ascontiguousarray(t_end, dtype=np.int32)
        if arr.shape != (len(self.scenes),):
            raise ValueError(f"t_end needs one entry per scene ({len(self.scenes)})")
        self._horizons = arr
        check(self.L.mpm_set_horizons(self.ctx, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
              "mpm_set_horizons")

    def profile(self, kernels=()):
        """Bracket the named kernels (see _lib.KERNELS) with HIP events."""
        mask = 0
        for k in kernels:
            mask |= 1 << _lib.KERNELS.index(k)
        check(self.L.mpm_profile(self.ctx, mask))

    def profile_read(self) -> dict:
        """{kernel: (launches, total ms)} since the last read (synchronises)."""
        n = len(_lib.KERNELS)
        cnt = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        check(self.L.mpm_profile_read(self.ctx, cnt, ms))
        return {k: (cnt[i], ms[i]) for i, k in enumerate(_lib.KERNELS)}

    def sync_errors(self):
        check(self.L.mpm_sync_errors(self.ctx), "device error")

    def tape_binnings(self) -> int:
        """Binnings the current tape's forward pass used (mpm_tape_binnings)."""
        n = ctypes.c_int32()
        check(self.L.mpm_tape_binnings(self.ctx, ctypes.byref(n)), "mpm_tape_binnings")
        return n.value

    def tape_generation(self) -> int:
        """The context's tape generation (mpm_tape_generation): changes with
        every rollout and every set_materials."""
        g = ctypes.c_uint64()
        check(self.L.mpm_tape_generation(self.ctx, ctypes.byref(g)), "mpm_tape_generation")
        return g.value


def step_forward_noalloc(scene: dict, s: StateT, act: Optional[torch.Tensor],
                         out: StateT, err: torch.Tensor,
                         act_id: Optional[torch.Tensor] = None, stream=None) -> None:
    """mpm_step_forward_noalloc: one substep of one scene with no context and
    no allocation (the library's static per-GPU region holds the grid).
    ``out`` and ``err`` (int32 [1] on the GPU, device error bits OR-ed in)
    are the caller's; ``act_id`` is an int32 CUDA tensor [N] or None."""
    L = _lib.lib()
    d, N = scene["dim"], scene["n_particles"]
    shapes = [(d, N), (d, N), (d * d, N), (d * d, N)]
    for st, nm in ((s, "s_n"), (out, "s_np1")):
        for t, sh, c in zip(st, shapes, "xvCF"):
            _check_tensor(t, sh, f"{nm}.{c}")
    if not (err.is_cuda and err.dtype == torch.int32 and err.numel() >= 1):
        raise ValueError("err must be an int32 CUDA tensor")
    if act_id is not None and not (act_id.is_cuda and act_id.dtype == torch.int32
                                   and act_id.is_contiguous() and act_id.numel() == N):
        raise ValueError(f"act_id must be a contiguous int32 CUDA tensor of {N} entries")
    n_act = scene.get("n_act", 0)
    if n_act:
        _check_tensor(act, (n_act,), "act")
    sc = scene_struct(scene)
    a = _lib.State(*[t.data_ptr() for t in s])
    o = _lib.State(*[t.data_ptr() for t in out])
    check(L.mpm_step_forward_noalloc(ctypes.byref(sc), _ptr(act_id), ctypes.byref(a),
                                     _ptr(act) if n_act else None, ctypes.byref(o),
                                     _ptr(err), _stream_ptr(stream)),
          "mpm_step_forward_noalloc")


def act_bank_forward(T: int, dt: float, freq: torch.Tensor, amp: torch.Tensor,
                     phase: torch.Tensor, stream=None) -> torch.Tensor:
    L = _lib.lib()
    n_act, n_freq = amp.shape
    act = torch.empty(T, n_act, device=amp.device)
    for t, nm, sh in ((freq, "freq", (n_freq,)), (amp, "amp", (n_act, n_freq)),
                      (phase, "phase", (n_act, n_freq))):
        _check_tensor(t, sh, nm)
    check(L.mpm_act_bank_forward(_stream_ptr(stream), T, n_act, n_freq, dt, _ptr(freq),
                                 _ptr(amp), _ptr(phase), _ptr(act)), "act_bank_forward")
    return act


def act_bank_backward(T: int, dt: float, freq, amp, phase, g_act, stream=None):
    L = _lib.lib()
    n_act, n_freq = amp.shape
    _check_tensor(g_act, (T, n_act), "g_act")
    ga = torch.empty_like(amp)
    gp = torch.empty_like(phase)
    check(L.mpm_act_bank_backward(_stream_ptr(stream), T, n_act, n_freq, dt, _ptr(freq),
                                  _ptr(amp), _ptr(phase), _ptr(g_act), _ptr(ga), _ptr(gp)),
          "act_bank_backward")
    return ga, gp
