"""Mutation check of the oracle's pins (CPU only).

Each mutant plants one plausible mistake in a copy of the oracle source: a
dropped term, a wrong sign, index or weight, a transposed operand.  The
copy is built into a temporary library that the pin suite
(`test_oracle_pins.py`) then loads through ORACLE_LIB; the pins must fail
for every mutant.  The committed oracle is never modified.

Alternative *readings* of the paper (the Roe sound-speed form, open or closed
stencil cones, the stencil size) are deliberately not mutants: the paper's
data cannot tell them apart, so no invariant pins them.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

from oracle import build as oracle_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, exact text in the oracle source, replacement)
MUTANTS = [
    ("gauss_weight", "w[i] = 1.0 / ((1.0 - x * x) * dp * dp);",
     "w[i] = 0.5 / ((1.0 - x * x) * dp * dp);"),
    ("basis_mean", "return ipow(xi, b.ea[l]) * ipow(eta, b.eb[l]) - b.mean[l];",
     "return ipow(xi, b.ea[l]) * ipow(eta, b.eb[l]) - 0.5 * b.mean[l];"),
    ("qr_reflector", "double bta = 2.0 / vtv;", "double bta = 1.0 / vtv;"),
    ("lsq_mean_volume", "S.qr.a[(size_t)l * want + s] = acc * a2 - S.vol[s] * B.mean[l];",
     "S.qr.a[(size_t)l * want + s] = acc * a2 - B.mean[l];"),
    ("lsq_rhs_volume", "b[s] = S.vol[s] * (U[4 * S.cells[s] + v] - u0);",
     "b[s] = (U[4 * S.cells[s] + v] - u0);"),
    ("beta_multiplicity", "      beta += acc;\n",
     "      beta += (ax > 0 && ay > 0) ? 2.0 * acc : acc;\n"),
    ("gamma_power", "return 1.0 / ipow(x, p.power);", "return 1.0 / ipow(x, p.power - 2);"),
    ("cutoff_equality", "if (s.chiK >= p.ct) {", "if (s.chiK > p.ct) {"),
    ("step_two_normalisation", "s.chi_small[k] = g[k] / sum_small;",
     "s.chi_small[k] = g[k] / sum_all;"),
    ("near_tie_absolute", "return std::fabs(chi / p.ct - 1.0) <= p.tie_rel;",
     "return std::fabs(chi - p.ct) <= p.tie_rel;"),
    ("small_weights", "abar[l] = acc / (double)cnt;", "abar[l] = acc;"),
    ("face_point_direction", "else if (e == 1) { xi = 1.0 - t; eta = t; }",
     "else if (e == 1) { xi = t; eta = 1.0 - t; }"),
    ("hll_dissipation_sign", "SL * SR * (R[c] - L[c])", "SL * SR * (L[c] - R[c])"),
    ("roe_weight", "T D = std::sqrt(R[0] / L[0]);", "T D = std::sqrt(L[0] / R[0]);"),
    ("left_wave_speed", "T SL = min_re(unL - cL, ut - ct);", "T SL = min_re(unL - cL, ut + ct);"),
    ("rotate_back", "out[1] = F[1] * nx - F[2] * ny;", "out[1] = F[1] * nx + F[2] * ny;"),
    ("face_point_pairing",
     "uR = &fp[((size_t)R * 3 * nq + eR * nq + (nq - 1 - k)) * 4];",
     "uR = &fp[((size_t)R * 3 * nq + eR * nq + k) * 4];"),
    ("face_side_sign", "double s = (m.fL[f] == i && m.fLe[f] == e) ? 1.0 : -1.0;",
     "double s = (m.fL[f] == i && m.fLe[f] == e) ? 1.0 : 1.0;"),
    ("residual_sign", "Ri[c] = -acc[c] / m.area[i];", "Ri[c] = acc[c] / m.area[i];"),
    ("dt_face_length", "den += m->flen[f] * (std::fabs(un) + c);", "den += (std::fabs(un) + c);"),
    ("rk_stage_two", "U2[t] = 0.75 * U[t] + 0.25 * U1[t] + 0.25 * (dt * R[t]);",
     "U2[t] = 0.25 * U[t] + 0.75 * U1[t] + 0.25 * (dt * R[t]);"),
    ("vjp_face_adjoint",
     "pb[c] = lam[4 * (size_t)R + c] / m->area[R] - lam[4 * (size_t)L + c] / m->area[L];",
     "pb[c] = lam[4 * (size_t)R + c] / m->area[L] - lam[4 * (size_t)L + c] / m->area[R];"),
    ("vjp_target_sign", "          Ubar[4 * (size_t)i + v] -= d;",
     "          Ubar[4 * (size_t)i + v] += d;"),
    ("cweno_small_linear_weight", "for (int k = 0; k < 3; ++k) d[k] = (1.0 - d[3]) / 3.0;",
     "for (int k = 0; k < 3; ++k) d[k] = (1.0 - d[3]);"),
    ("cweno_optimal_subtraction", "for (int k = 0; k < 3; ++k) opt -= d[k] * coef[k][l];",
     "for (int k = 0; k < 3; ++k) opt += d[k] * coef[k][l];"),
    ("cweno_large_scaling", "abar[l] = (w[3] / d[3]) * opt;", "abar[l] = w[3] * opt;"),
    ("char_acoustic_energy", "{1.0, vx - c * nx, vy - c * ny, H - c * un},",
     "{1.0, vx - c * nx, vy - c * ny, H + c * un},"),
    ("char_shear_energy", "{0.0, -ny, nx, ut},", "{0.0, -ny, nx, un},"),
    ("char_inverse_elimination", "for (int k = 0; k < 8; ++k) a[r][k] -= f * a[col][k];",
     "for (int k = 0; k < 8; ++k) a[r][k] += f * a[col][k];"),
    ("char_face_normal", "    edge_normal(m, i, e, nx, ny);\n",
     "    edge_normal(m, i, (e + 1) % 3, nx, ny);\n"),
    ("char_projection_state", "char_basis(u0, nx, ny, m.prm.gamma, R, L);",
     "char_basis(&U[4 * (size_t)cd.st[3].cells[1]], nx, ny, m.prm.gamma, R, L);"),
    ("char_projection_transposed", "wc[k][l] += L[4 * v + j] * coef[j][k][l];",
     "wc[k][l] += L[4 * j + v] * coef[j][k][l];"),
    ("char_back_transform", "val += R[4 * c + v] * dw[v][kq];", "val += L[4 * c + v] * dw[v][kq];"),
    ("char_flags_edge", "    flags3[e] = fe;\n", "    flags3[(e + 1) % 3] = fe;\n"),
    ("wall_normal_reversal", "uR[1] = -mn * nx - mt * ny;", "uR[1] = mn * nx - mt * ny;"),
    ("wall_tangent_sign", "uR[2] = -mn * ny + mt * nx;", "uR[2] = -mn * ny - mt * nx;"),
    ("prescribed_state_ignored", "for (int c = 0; c < 4; ++c) uR[c] = T(m.bstate[4 * (size_t)b + c]);",
     "for (int c = 0; c < 4; ++c) uR[c] = uL[c];"),
    ("boundary_kind_swap", "  } else if (m.bkind[b] == 2) {", "  } else if (m.bkind[b] == 1) {"),
    ("stencil_fill_order", "    std::sort(rest.begin(), rest.end());\n", "\n"),
    ("vjp_boundary_sign", "for (int c = 0; c < 4; ++c) pb[c] = -lam[4 * (size_t)L + c] / m->area[L];",
     "for (int c = 0; c < 4; ++c) pb[c] = lam[4 * (size_t)L + c] / m->area[L];"),
    ("vjp_boundary_outer_fixed",
     "          if (bnd) boundary_state(*m, m->bidx[f], a, m->fn[2 * f], m->fn[2 * f + 1], b);\n",
     "          if (bnd) { cplx a0[4]; for (int t = 0; t < 4; ++t) a0[t] = cplx(a[t].real(), 0.0);"
     " boundary_state(*m, m->bidx[f], a0, m->fn[2 * f], m->fn[2 * f + 1], b); }\n"),
]

# the pin expected to catch each mutant: it runs first, and the whole pin
# suite only if it passes
FIRST_PIN = {
    "gauss_weight": "test_gauss_legendre_matches_numpy",
    "basis_mean": "test_polynomial_reproduction",
    "qr_reflector": "test_lsq_matches_numpy_lstsq",
    "lsq_mean_volume": "test_polynomial_reproduction",
    "lsq_rhs_volume": "test_polynomial_reproduction",
    "beta_multiplicity": "test_smoothness_closed_forms",
    "gamma_power": "test_selection_threshold_and_near_tie",
    "cutoff_equality": "test_selection_exact_equality_counts_as_smooth",
    "step_two_normalisation": "test_selection_step_two_renormalises_small_stencils",
    "near_tie_absolute": "test_selection_threshold_and_near_tie",
    "small_weights": "test_vjp_dot_product",
    "face_point_direction": "test_polynomial_reproduction",
    "hll_dissipation_sign": "test_hll_resolves_isolated_shock",
    "roe_weight": "test_hll_resolves_isolated_shock",
    "left_wave_speed": "test_hll_antisymmetry_and_rotation",
    "rotate_back": "test_hll_consistency",
    "face_point_pairing": "test_residual_cells_match_full",
    "face_side_sign": "test_free_stream_and_conservation",
    "residual_sign": "test_residual_cells_match_full",
    "dt_face_length": "test_dt_closed_form_regular_mesh",
    "rk_stage_two": "test_vjp_rk_step_against_differences",
    "vjp_face_adjoint": "test_vjp_dot_product",
    "vjp_target_sign": "test_vjp_dot_product",
    "cweno_small_linear_weight": "test_cweno_weights_special_cases",
    "cweno_optimal_subtraction": "test_cweno_reproduces_quadratics",
    "cweno_large_scaling": "test_cweno_reproduces_quadratics",
    "char_acoustic_energy": "test_char_basis_diagonalises_the_flux_jacobian",
    "char_shear_energy": "test_char_basis_diagonalises_the_flux_jacobian",
    "char_inverse_elimination": "test_char_basis_diagonalises_the_flux_jacobian",
    "char_face_normal": "test_char_reconstruction_is_componentwise_on_the_projected_field",
    "char_projection_state": "test_char_nonphysical_mean_keeps_conservative_variables",
    "char_projection_transposed": "test_char_reconstruction_is_componentwise_on_the_projected_field",
    "char_back_transform": "test_char_reconstruction_is_componentwise_on_the_projected_field",
    "char_flags_edge": "test_char_reconstruction_is_componentwise_on_the_projected_field",
    "wall_normal_reversal": "test_closed_box_conserves_mass_and_energy",
    "wall_tangent_sign": "test_boundary_face_flux_on_uniform_interior",
    "prescribed_state_ignored": "test_boundary_face_flux_on_uniform_interior",
    "boundary_kind_swap": "test_box_free_stream",
    "stencil_fill_order": "test_box_stencils_follow_the_rule",
    "vjp_boundary_sign": "test_box_vjp_dot_product_and_differences",
    "vjp_boundary_outer_fixed": "test_box_vjp_dot_product_and_differences",
}


def _run_mutant(tmp, name, old, new, src):
    assert src.count(old) == 1, f"mutation site of {name} not found exactly once"
    d = os.path.join(tmp, name)
    os.makedirs(d, exist_ok=True)
    cpp = os.path.join(d, "teno_oracle.cpp")
    with open(cpp, "w") as fh:
        fh.write(src.replace(old, new))
    lib = os.path.join(d, "liboracle.so")
    cmd = list(oracle_build.CMD)
    cmd[cmd.index("-o") + 1] = lib
    cmd[-1] = cpp
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    pins = os.path.join(ROOT, "tests", "test_oracle_pins.py")
    r = subprocess.run([sys.executable, "-m", "pytest", pins + "::" + FIRST_PIN[name], "-x", "-q",
                        "-p", "no:cacheprovider", "-p", "no:randomly"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    if r.returncode == 1:
        return name, 1, (r.stdout.strip().splitlines() or [""])[-1]
    # the named pin missed it: the fast pins, then the convergence runs
    for sel in ("not convergence", "convergence"):
        r = subprocess.run([sys.executable, "-m", "pytest",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-x", "-q",
                            "-k", sel, "-p", "no:cacheprovider", "-p", "no:randomly"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        last = (r.stdout.strip().splitlines() or [""])[-1]
        if r.returncode != 0:
            break
    return name, r.returncode, last


def test_every_mutant_fails_a_pin(tmp_path):
    src = open(oracle_build.SRC).read()
    workers = max(1, min(6, (os.cpu_count() or 2) - 2))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda m: _run_mutant(str(tmp_path), *m, src), MUTANTS))
    survivors = [(n, last) for n, rc, last in results if rc == 0]
    errors = [(n, rc, last) for n, rc, last in results if rc not in (0, 1)]
    assert not errors, f"mutant runs that did not end in test failures: {errors}"
    assert not survivors, f"mutants no pin detects: {survivors}"
