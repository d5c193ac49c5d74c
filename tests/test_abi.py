"""CPU-side checks of the C ABI: the library loads (no GPU needed to load it)
and exports every entry point declared in include/mpm.h; host-side argument
checks reject bad input before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["mpm_init", "mpm_step_forward", "mpm_step_backward", "mpm_rollout",
              "mpm_rollout_backward", "mpm_destroy", "mpm_sync_errors", "mpm_strerror"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1810_01054_amd import _lib
    L = _lib.lib()
    for n in _declared():
        assert hasattr(L, n), f"libmpm.so does not export {n}"
    assert sorted(_lib.EXPORTS) == _declared()


def test_strerror_and_arg_checks_need_no_gpu():
    from paper_1810_01054_amd import _lib
    L = _lib.lib()
    assert L.mpm_strerror(-3) == b"particle stencil outside the grid"
    assert L.mpm_strerror(0) == b"ok"
    # host-side validation returns before any HIP call
    ctx = ctypes.c_void_p()
    assert L.mpm_init(ctypes.byref(ctx), None, 0, None, None, None) == -1
    sc = _lib.Scene()
    sc.dim, sc.n_grid, sc.n_particles = 4, 16, 10   # bad dimension
    assert L.mpm_init(ctypes.byref(ctx), ctypes.byref(sc), 1, None, None, None) == -1
    sc.dim, sc.dt, sc.V0, sc.rho, sc.E, sc.nu = 2, 1e-4, 1e-4, 1.0, 10.0, 0.6  # nu >= 0.5
    assert L.mpm_init(ctypes.byref(ctx), ctypes.byref(sc), 1, None, None, None) == -1
    assert L.mpm_step_forward(None, None, None, None) == -1
    assert L.mpm_rollout_backward(None, None, None, None) == -1
    assert L.mpm_act_bank_forward(None, -1, 1, 1, 1e-4, None, None, None, None) == -1


def test_oracle_and_product_share_no_code():
    """The product library never names the oracle, and the oracle never names
    the product."""
    pkg = os.path.join(ROOT, "paper_1810_01054_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "mpm_oracle" not in txt, f
                assert "liboracle" not in txt, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "from paper_1810_01054_amd" not in txt, f
            assert "import paper_1810_01054_amd" not in txt, f
            assert "libmpm.so" not in txt, f
            for inc in re.findall(r'#include\s+"([^"]+)"', txt):
                assert inc == "mpm_oracle.h", (f, inc)
