"""The oracle pins have teeth: plausible one-line mistakes planted in a copy of
the oracle source (compiled on the CPU into a temporary library) must each
make at least one pin fail.  The real oracle is never modified."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1810_01054_amd import scenes as S
from tests import test_oracle_pins as pins

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "mpm_oracle.c")).read()

# (name, exact text in mpm_oracle.c, replacement)
MUTANTS = [
    ("apic_term_dropped", "+ mp * Cp[k];", "+ 0.0 * Cp[k];"),
    ("stress_sign", "out->G[k] = -Dinv * s->dt", "out->G[k] = Dinv * s->dt"),
    ("stress_transposed", "matmul_nt_d(d, out->Pt, Fp, PFt);", "matmul_tn_d(d, out->Pt, Fp, PFt);"),
    ("actuation_sigma_F", "Fp[a * d + b] * out->sigma[b];", "Fp[a * d + b] * out->sigma[a];"),
    ("lame_mu", "*mu = E / (2.0 * (1.0 + nu));", "*mu = E / (1.0 + nu);"),
    ("gravity_dropped", "v[a] = v[a] + s->dt * s->gravity[a];", "v[a] = v[a] + 0.0 * s->gravity[a];"),
    ("wall_off_by_one", "ia >= n - s->wall", "ia > n - s->wall"),
    ("g2p_C_transposed", "B[a * d + b] += Nw * via * delta[b];", "B[b * d + a] += Nw * via * delta[b];"),
    ("F_update_order", "matmul_d(d, Ipc, Fp, Fn);", "matmul_d(d, Fp, Ipc, Fn);"),
    ("bspline_tail", "return 0.5 * (1.5 - a) * (1.5 - a);", "return 0.5 * (1.5 - a) * (1.4 - a);"),
    ("rev_E_sign", "mbar[i] = -vdot / m;", "mbar[i] = vdot / m;"),
    ("rev_E_post_gravity", "double vhat = gpm[a * nn + i] / m;", "double vhat = gvel[a * nn + i];"),
    ("rev_F_mass", "vb[a] += Nw * mp * pb[a];", "vb[a] += Nw * pb[a];"),
    ("rev_J_Cterm_sign", "xb[c] += -Nw * Dinv * cterm - Nw * pterm;", "xb[c] += Nw * Dinv * cterm - Nw * pterm;"),
    ("rev_J_pterm_dropped", "xb[c] += -Nw * Dinv * cterm - Nw * pterm;", "xb[c] += -Nw * Dinv * cterm;"),
    ("rev_J_mass_term", "+ s_p + mp * mb;", "+ s_p;"),
    ("rev_H_update_transposed", "matmul_tn_d(d, Ipc, gF1p, Fb);", "matmul_d(d, Ipc, gF1p, Fb);"),
    ("rev_H_hessian_sign", "(mu - la * sp.lnJ) * T2[k]", "(mu + la * sp.lnJ) * T2[k]"),
    ("rev_H_Gterm_dropped", "for (int k = 0; k < d * d; ++k) Fb[k] += kG * T1[k];", ""),
    ("rev_B_transposed", "matmul_nt_d(d, gF1p, Fp, GFt);\n    for (int k = 0; k < d * d; ++k) Ct[k] = gC1p[k] + dt * GFt[k];\n    /* (C)",
     "matmul_tn_d(d, gF1p, Fp, GFt);\n    for (int k = 0; k < d * d; ++k) Ct[k] = gC1p[k] + dt * GFt[k];\n    /* (C)"),
    ("rev_K_transposed", "sig_aa += Fp[g * d + a] * Ptb[g * d + a];", "sig_aa += Fp[a * d + g] * Ptb[g * d + a];"),
    ("rev_A_dt_dropped", "for (int a = 0; a < d; ++a) vt[a] = gv1p[a] + dt * gx1p[a];\n    /* (B)",
     "for (int a = 0; a < d; ++a) vt[a] = gv1p[a] + gx1p[a];\n    /* (B)"),
]


# Mistakes in the controller rollout, caught by the controller pins.
CTRL_MUTANTS = [
    ("ctrl_tanh_derivative", "double g = sb[j] * (1.0 - a[j] * a[j]);", "double g = sb[j];"),
    ("ctrl_mean_not_sum", "a0[(size_t)k * N + p] += zb[d + 2 * d * c + k] / (double)count[c];",
     "a0[(size_t)k * N + p] += zb[d + 2 * d * c + k];"),
    ("ctrl_velocity_slot", "z[d + 2 * d * c + d + a] += v[(size_t)a * N + p];",
     "z[d + 2 * d * c + a] += v[(size_t)a * N + p];"),
    ("ctrl_W_transposed", "zb[i] += W[(size_t)j * nz + i] * g;", "zb[i] += W[(size_t)i * nact + j] * g;"),
]


# Mistakes in the friction projection (L) and the wall condition built on
# it, caught by the friction pins.
FRICTION_MUTANTS = [
    ("fric_coulomb_sign", "double lts = fmax(lt + c * fmin(ln, 0.0), 0.0);",
     "double lts = fmax(lt - c * fmin(ln, 0.0), 0.0);"),
    ("fric_separating_dropped",
     "vs[a] = lts * (vt[a] / lt) + fmax(ln, 0.0) * nrm[a];", "vs[a] = lts * (vt[a] / lt);"),
    ("fric_high_face_normal", "sg[k++] = -1.0;", "sg[k++] = 1.0;"),
    ("fric_rev_HR_dropped", "double ltb = -s / (lt * lt) + ltsb * HR;",
     "double ltb = -s / (lt * lt) + ltsb;"),
    ("fric_rev_c_term_sign", "lnb += ltsb * HR * c * (-ln >= 0.0 ? 1.0 : 0.0);",
     "lnb -= ltsb * HR * c * (-ln >= 0.0 ? 1.0 : 0.0);"),
    ("fric_rev_normal_pass_dropped", "lnb += (ln >= 0.0 ? 1.0 : 0.0) * nv;", ""),
    ("fric_rev_vt_scale", "vtb[a] = (ltb * vt[a] + vthb[a]) / lt;",
     "vtb[a] = ltb * vt[a] + vthb[a];"),
    ("fric_rev_grid_skipped", "wall_bc_bwd(s, i, v, vb);", ""),
]


def _run_friction_pins():
    from tests import test_oracle_friction as fr
    failed = []
    for name, fn in [
            ("frictionless", lambda: fr.test_frictionless_wall_removes_only_an_approaching_normal_component(3)),
            ("coulomb", lambda: fr.test_coulomb_friction_shortens_the_tangential_velocity(2)),
            ("separating", lambda: fr.test_separating_velocity_passes_and_energy_never_grows(3)),
            ("reverse_fd", lambda: fr.test_projection_reverse_matches_central_differences(3)),
            ("grid_clamp", lambda: fr.test_grid_frictionless_walls_clamp_each_face_normal(2)),
            ("rollout_fd", lambda: fr.test_contact_rollout_gradients_match_central_differences(2, 0.4))]:
        try:
            fn()
        except (AssertionError, oracle.OracleError, ValueError):
            failed.append(name)
    return failed


# Mistakes in the per-particle material gradients, caught by the material
# pins (Euler relation, central differences).
MATERIAL_MUTANTS = [
    ("mat_mass_grid_term_dropped", "double mbp = Nmb;", "double mbp = 0.0;"),
    ("mat_mass_apic_term_dropped", "for (int k = 0; k < d * d; ++k) mbp += Cp[k] * Gb[k];", ""),
    ("mat_mass_velocity_term_dropped", "for (int a = 0; a < d; ++a) mbp += vp[a] * Spb[a];", ""),
    ("mat_mu_without_inverse", "mub += Ptb[k] * (Fp[k] - sp.FiT[k]);", "mub += Ptb[k] * Fp[k];"),
    ("mat_lambda_without_lnJ", "s->gE_p[p] += mub * dmu_dE + sp.lnJ * inner * dla_dE;",
     "s->gE_p[p] += mub * dmu_dE + inner * dla_dE;"),
    ("mat_rho_without_V0", "s->grho_p[p] += s->V0 * mbp;", "s->grho_p[p] += mbp;"),
    ("mat_forward_mass_scene", "*mp = (s->rho_p ? s->rho_p[p] : s->rho) * s->V0;",
     "*mp = s->rho * s->V0;"),
]


def _run_material_pins():
    from tests import test_oracle_materials as mt
    failed = []
    for name, fn in [("uniform", mt.test_uniform_fields_reproduce_the_scene_rollout),
                     ("scaling", lambda: mt.test_scaling_mass_and_stiffness_together_leaves_the_motion(2)),
                     ("euler", lambda: mt.test_euler_relation_of_the_material_gradients(2)),
                     ("fd", lambda: mt.test_material_gradients_match_central_differences(2))]:
        try:
            fn()
        except (AssertionError, oracle.OracleError, ValueError):
            failed.append(name)
    return failed


def _run_ctrl_pins():
    from tests import test_oracle_ctrl as ctrl
    failed = []
    for name, fn in [("zero_gain", ctrl.test_zero_gain_controller_is_the_open_loop_rollout),
                     ("means", ctrl.test_first_actuation_from_numpy_means),
                     ("fd2", lambda: ctrl.test_controller_gradients_match_central_differences(2))]:
        try:
            fn()
        except (AssertionError, oracle.OracleError, ValueError):
            failed.append(name)
    return failed


def _run_pins():
    """Run a fast subset of the pins; return the names of those that fail."""
    failed = []
    checks = [
        ("bspline", lambda: pins.test_bspline_moments(64.0)),
        ("lame", lambda: pins.test_neohookean_is_energy_gradient(3)),
        ("mass_momentum", lambda: pins.test_p2g_mass_and_momentum(S.tiny_2d)),
        ("second_moment", lambda: pins.test_p2g_second_moment_reproduces_C(3)),
        ("energy", lambda: pins.test_p2g_stress_is_energy_gradient(S.tiny_2d)),
        ("affine", lambda: pins.test_affine_field_reproduced(2)),
        ("translation", lambda: pins.test_rigid_translation_and_shift(2)),
        ("gravity_wall", pins.test_gravity_and_wall_freeze),
        ("wall_band", lambda: pins.test_grid_update_wall_band(2)),
        ("free_flight", lambda: pins.test_free_flight_closed_forms(2)),
        ("torch_fwd", lambda: pins.test_forward_matches_independent_torch(S.tiny_2d)),
        ("torch_rev", lambda: pins.test_reverse_matches_torch_autograd(S.tiny_2d)),
        ("fd", lambda: pins.test_rollout_gradient_central_fd(S.tiny_2d, 4)),
    ]
    for name, fn in checks:
        try:
            fn()
        except (AssertionError, oracle.OracleError, np.linalg.LinAlgError, ValueError):
            failed.append(name)
    return failed


def test_unmutated_source_passes_subset():
    assert _run_pins() == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    assert SRC.count(old) == 1, f"mutation anchor for {name} not unique"
    src = tmp_path / "mutant.c"
    src.write_text(SRC.replace(old, new))
    hdr = os.path.join(os.path.dirname(oracle.__file__), "mpm_oracle.h")
    (tmp_path / "mpm_oracle.h").write_text(open(hdr).read())
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", str(lib), str(src), "-lm"], check=True)
    with oracle.use_library(str(lib)):
        failed = _run_pins()
    assert failed, f"mutant {name} passed every pin"


@pytest.mark.parametrize("name,old,new", CTRL_MUTANTS, ids=[m[0] for m in CTRL_MUTANTS])
def test_controller_mutant_is_caught(name, old, new, tmp_path):
    assert SRC.count(old) == 1, f"mutation anchor for {name} not unique"
    src = tmp_path / "mutant.c"
    src.write_text(SRC.replace(old, new))
    hdr = os.path.join(os.path.dirname(oracle.__file__), "mpm_oracle.h")
    (tmp_path / "mpm_oracle.h").write_text(open(hdr).read())
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", str(lib), str(src), "-lm"], check=True)
    with oracle.use_library(str(lib)):
        failed = _run_ctrl_pins()
    assert failed, f"mutant {name} passed every controller pin"


@pytest.mark.parametrize("name,old,new", FRICTION_MUTANTS, ids=[m[0] for m in FRICTION_MUTANTS])
def test_friction_mutant_is_caught(name, old, new, tmp_path):
    assert SRC.count(old) == 1, f"mutation anchor for {name} not unique"
    src = tmp_path / "mutant.c"
    src.write_text(SRC.replace(old, new))
    hdr = os.path.join(os.path.dirname(oracle.__file__), "mpm_oracle.h")
    (tmp_path / "mpm_oracle.h").write_text(open(hdr).read())
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", str(lib), str(src), "-lm"], check=True)
    with oracle.use_library(str(lib)):
        failed = _run_friction_pins()
    assert failed, f"mutant {name} passed every friction pin"


@pytest.mark.parametrize("name,old,new", MATERIAL_MUTANTS, ids=[m[0] for m in MATERIAL_MUTANTS])
def test_material_mutant_is_caught(name, old, new, tmp_path):
    assert SRC.count(old) == 1, f"mutation anchor for {name} not unique"
    src = tmp_path / "mutant.c"
    src.write_text(SRC.replace(old, new))
    hdr = os.path.join(os.path.dirname(oracle.__file__), "mpm_oracle.h")
    (tmp_path / "mpm_oracle.h").write_text(open(hdr).read())
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", str(lib), str(src), "-lm"], check=True)
    with oracle.use_library(str(lib)):
        failed = _run_material_pins()
    assert failed, f"mutant {name} passed every material pin"
