"""Mutation check of the tetrahedral oracle's pins (CPU only).

Each mutant plants one plausible mistake in a copy of oracle/teno3_oracle.cpp
(a dropped factor, a wrong sign, weight, vertex order or pairing); the copy is
built into a temporary library that test_oracle3_pins.py loads through
ORACLE3_LIB, and the pins must fail for every mutant.  Readings of the paper
(the Roe sound-speed form, open or closed cones, stencil sizes) are not
mutants: nothing printed in the paper tells them apart.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

from oracle import build as oracle_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("face_rule_weight", "orbit3(0.445948490915965, 0.223381589678011);",
     "orbit3(0.445948490915965, 0.213381589678011);"),
    ("basis_mean_volume", "b.mean.push_back(acc * 6.0);", "b.mean.push_back(acc * 2.0);"),
    ("qr_reflector", "double bta = 2.0 / vtv;", "double bta = 1.0 / vtv;"),
    ("lsq_rhs_volume", "b[s] = S.vol[s] * (U[NV * (size_t)S.cells[s] + v] - u0);",
     "b[s] = (U[NV * (size_t)S.cells[s] + v] - u0);"),
    ("reference_volume", "S.vol[s] = jac / 6.0;", "S.vol[s] = jac / 2.0;"),
    ("member_unwrap", "p[a] = Xj[3 * v + a] + sh[a] - X0[a];", "p[a] = Xj[3 * v + a] - X0[a];"),
    ("inverse_map_row", "cross(col1, col2, r0);", "cross(col2, col1, r0);"),
    ("beta_multiplicity", "        beta += acc;\n",
     "        beta += ((ax > 0) + (ay > 0) + (az > 0) > 1) ? 2.0 * acc : acc;\n"),
    ("gamma_power", "double gamma_of(double beta, const oracle3_params& p) { return 1.0 / ipow(beta + p.eps, p.power); }",
     "double gamma_of(double beta, const oracle3_params& p) { return 1.0 / ipow(beta + p.eps, p.power - 2); }"),
    ("cutoff_equality", "if (s.chiK >= p.ct) {", "if (s.chiK > p.ct) {"),
    ("step_two_normalisation", "s.chi_small[k] = g[k] / sum_small;", "s.chi_small[k] = g[k] / sum_all;"),
    ("small_weights", "abar[l] = acc / (double)cnt;", "abar[l] = acc;"),
    ("cone_third_vertex", "return al * D >= 0.0 && be * D >= 0.0 && ga * D >= 0.0;",
     "return al * D >= 0.0 && be * D >= 0.0;"),
    ("face_vertex_order", "const int FV[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};",
     "const int FV[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 2, 1}};"),
    ("reference_vertices", "static const double V[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};",
     "static const double V[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 0, 1}, {0, 1, 0}};"),
    ("face_point_pairing", "uR = &fp[(((size_t)R * 4 + eR) * npt + m.pair[(size_t)f * npt + k]) * NV];",
     "uR = &fp[(((size_t)R * 4 + eR) * npt + k) * NV];"),
    ("hll_dissipation_sign", "SL * SR * (R[c] - L[c])", "SL * SR * (L[c] - R[c])"),
    ("roe_weight", "const double D = std::sqrt(R[0] / L[0]);", "const double D = std::sqrt(L[0] / R[0]);"),
    ("left_wave_speed", "const double SL = std::min(unL - cL, ut - ct);",
     "const double SL = std::min(unL - cL, ut + ct);"),
    ("rotate_back_tangents", "out[1 + a] = F[1] * n[a] + F[2] * t1[a] + F[3] * t2[a];",
     "out[1 + a] = F[1] * n[a] + F[2] * t2[a] + F[3] * t1[a];"),
    ("face_side_sign", "const double s = (m.fL[f] == i && m.fLe[f] == e) ? 1.0 : -1.0;",
     "const double s = (m.fL[f] == i && m.fLe[f] == e) ? 1.0 : 1.0;"),
    ("residual_sign", "Ri[c] = -acc[c] / m.vol[i];", "Ri[c] = acc[c] / m.vol[i];"),
    ("dt_face_area", "den += m->farea[f] * (std::fabs(vx * nn[0] + vy * nn[1] + vz * nn[2]) + c);",
     "den += (std::fabs(vx * nn[0] + vy * nn[1] + vz * nn[2]) + c);"),
    ("rk_stage_two", "U2[t] = 0.75 * U[t] + 0.25 * U1[t] + 0.25 * (dt * R[t]);",
     "U2[t] = 0.25 * U[t] + 0.75 * U1[t] + 0.25 * (dt * R[t]);"),
    ("wall_reflection", "uR[1 + a] = uL[1 + a] - 2.0 * mn * n[a];", "uR[1 + a] = uL[1 + a] - mn * n[a];"),
]

# the pin expected to catch each mutant: it runs first, and the whole pin
# suite only if it passes
FIRST_PIN = {
    "face_rule_weight": "test_face_rules_exact_and_symmetric",
    "basis_mean_volume": "test_basis_graded_and_zero_mean",
    "qr_reflector": "test_polynomial_reproduction",
    "lsq_rhs_volume": "test_polynomial_reproduction",
    "reference_volume": "test_polynomial_reproduction",
    "member_unwrap": "test_polynomial_reproduction",
    "inverse_map_row": "test_polynomial_reproduction",
    "beta_multiplicity": "test_smoothness_closed_forms",
    "gamma_power": "test_selection_threshold_and_step_two",
    "cutoff_equality": "test_selection_threshold_and_step_two",
    "step_two_normalisation": "test_selection_threshold_and_step_two",
    "small_weights": "test_kept_small_stencils_are_averaged",
    "cone_third_vertex": "test_stencil_cones_and_order",
    "face_vertex_order": "test_geometry_closes_and_normals_point_out",
    "reference_vertices": "test_polynomial_reproduction",
    "face_point_pairing": "test_linear_field_residual_is_face_quadrature_of_exact_flux",
    "hll_dissipation_sign": "test_hll3_resolves_isolated_shock",
    "roe_weight": "test_hll3_resolves_isolated_shock",
    "left_wave_speed": "test_hll3_antisymmetry_and_rotation",
    "rotate_back_tangents": "test_hll3_consistency_and_upwinding",
    "face_side_sign": "test_free_stream_and_conservation",
    "residual_sign": "test_linear_field_residual_is_face_quadrature_of_exact_flux",
    "dt_face_area": "test_dt_closed_form_on_a_cube",
    "rk_stage_two": "test_rk3_is_third_order_in_time",
    "wall_reflection": "test_closed_reflective_box_conserves_mass_and_energy",
}


def _run_mutant(tmp, name, old, new, src):
    assert src.count(old) == 1, f"mutation site of {name} not found exactly once"
    d = os.path.join(tmp, name)
    os.makedirs(d, exist_ok=True)
    cpp = os.path.join(d, "teno3_oracle.cpp")
    with open(cpp, "w") as fh:
        fh.write(src.replace(old, new))
    lib = os.path.join(d, "liboracle3.so")
    cmd = list(oracle_build.CMD)
    cmd[cmd.index("-o") + 1] = lib
    cmd[-1] = cpp
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ORACLE3_LIB=lib, OMP_NUM_THREADS="1")
    pins = os.path.join(ROOT, "tests", "test_oracle3_pins.py")
    r = subprocess.run([sys.executable, "-m", "pytest", pins + "::" + FIRST_PIN[name], "-x", "-q",
                        "-p", "no:cacheprovider", "-p", "no:randomly"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    if r.returncode == 1:
        return name, 1, (r.stdout.strip().splitlines() or [""])[-1]
    # the named pin missed it: the fast pins, then the convergence runs
    for sel in ("not convergence", "convergence"):
        r = subprocess.run([sys.executable, "-m", "pytest",
                            os.path.join(ROOT, "tests", "test_oracle3_pins.py"), "-x", "-q",
                            "-k", sel, "-p", "no:cacheprovider", "-p", "no:randomly"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
        last = (r.stdout.strip().splitlines() or [""])[-1]
        if r.returncode != 0:
            break
    return name, r.returncode, last


def test_every_mutant_fails_a_pin(tmp_path):
    src = open(oracle_build.SRC3).read()
    workers = max(1, min(6, (os.cpu_count() or 2) - 2))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda m: _run_mutant(str(tmp_path), *m, src), MUTANTS))
    survivors = [(n, last) for n, rc, last in results if rc == 0]
    errors = [(n, rc, last) for n, rc, last in results if rc not in (0, 1)]
    assert not errors, f"mutant runs that did not end in test failures: {errors}"
    assert not survivors, f"mutants no pin detects: {survivors}"
