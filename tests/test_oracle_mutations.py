"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake (a dropped term, a wrong sign, a transposed
operand or index) in a copy of the oracle's C source, builds it with gcc on the
CPU, and runs the pin suite against it in a subprocess; the suite must fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "efem_oracle.c")

MUTATIONS = {
    "tangent_last_term_transposed": ("+ c * Fi[J][k] * Fi[L][i]", "+ c * Fi[J][i] * Fi[L][k]"),
    "tangent_lambda_term_transposed": ("lam * Fi[J][i] * Fi[L][k]", "lam * Fi[J][k] * Fi[L][i]"),
    "tangent_dropped_identity": ("(i == k && J == L ? mu : 0.0)", "0.0"),
    "stress_transposed_inverse": ("Pm[i][J] = s->F[i][J] - s->Finv[J][i];",
                                  "Pm[i][J] = s->F[i][J] - s->Finv[i][J];"),
    "energy_log_sign": ("*dmu = 0.5 * s->I1m3 - s->lnJ;", "*dmu = 0.5 * s->I1m3 + s->lnJ;"),
    "gradient_uses_J_inverse_not_transpose": ("t += Ji[J][L] * r->dN[q][a][J]", "t += Ji[L][J] * r->dN[q][a][J]"),
    "jacobian_dropped_det_term": ("+ 0.5 * (trH * trH - trH2) + det3(H);", "+ 0.5 * (trH * trH - trH2);"),
    "coords_adjoint_transposed_H": ("t -= s.H[i][m] * P[i][L]", "t -= s.H[m][i] * P[i][L]"),
    "hex_gauss_point": ("const double g = 1.0 / sqrt(3.0);", "const double g = 0.5;"),
    "diag_wrong_index": ("A[i][J][i][L] * s.gN[a][J] * s.gN[a][L]", "A[i][J][i][J] * s.gN[a][J] * s.gN[a][L]"),
    "vjp_mu_transposed": ("gm += s.wdetJ * Pm[i][J] * gw;", "gm += s.wdetJ * Pm[J][i] * gw;"),
    "grad_material_swapped_parts": ("gm += s.wdetJ * pm;", "gm += s.wdetJ * pl;"),
    "linear_tangent_dropped_minor_symmetry": ("+ (i == L && J == k ? 1.0 : 0.0))", "+ 0.0)"),
    "linear_stress_factor": ("Pm[i][J] = 2.0 * s->eps[i][J];", "Pm[i][J] = s->eps[i][J];"),
    "linear_energy_lambda_half": ("*dlam = 0.5 * s->treps * s->treps;", "*dlam = s->treps * s->treps;"),
    "linear_strain_not_symmetrised": ("s->eps[i][j] = 0.5 * (H[i][j] + H[j][i]);", "s->eps[i][j] = H[i][j];"),
    "linear_lambda_term_off_diagonal": ("Pl[i][J] = i == J ? s->treps : 0.0;", "Pl[i][J] = s->treps;"),
    "tet_weight": ("r->w[0] = 1.0 / 6.0;", "r->w[0] = 1.0 / 3.0;"),
    "transport_rotation_orientation": ("const double b[3] = {omega[1] * xq[2] - omega[2] * xq[1],",
                                       "const double b[3] = {omega[2] * xq[1] - omega[1] * xq[2],"),
    "transport_matrix_test_trial_swapped": ("adv += b[L] * s.gN[bb][L];", "adv += b[L] * s.gN[a][L];"),
    "transport_matrix_reaction_dropped_trial": ("k[e] * r.N[q][bb] * r.N[q][a]", "k[e] * r.N[q][a]"),
    "transport_residual_dropped_diffusion": ("(D[e] * diff + val * r.N[q][a])", "(val * r.N[q][a])"),
    "transport_residual_value_not_interpolated": ("cq += r.N[q][a] * ce[a][sp];", "cq += ce[a][sp];"),
    "tet_centroid_value": ("r->N[0][a] = 0.25;", "r->N[0][a] = 1.0 / 3.0;"),
}
MUTATIONS.update({
    "tri_weight": ("r->w[0] = 0.5;", "r->w[0] = 1.0;"),
    "tri_thickness": ("Jm[2][2] += 1.0;", "Jm[2][2] += 2.0;"),
    "tri_shape_gradient": ("{{-1, -1, 0}, {1, 0, 0}, {0, 1, 0}}", "{{-1, -1, 0}, {1, 0, 0}, {0, 1, 1}}"),
})
PIN_FILES = ["test_oracle_pins.py", "test_oracle_transport.py"]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not found once: {old!r}"
    mutated = tmp_path / "mutated.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libmutated.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    str(mutated), "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ, EFEM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                         + [os.path.join(ROOT, "tests", f) for f in PIN_FILES],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode != 0, f"pins did not catch mutation {name}:\n{res.stdout[-2000:]}"


# Mistakes in the oracle's Python layer (the loaded Newton solve): planted in a
# copy of the oracle package placed in a scratch tree with the tests and the
# input generators, and run there against the real C oracle.
# name: (anchor, replacement, pin files that must catch it)
PY_MUTATIONS = {
    "load_residual_not_scaled_by_step": ("reshape(-1) - s * f)", "reshape(-1) - f)", ["test_oracle_load.py"]),
    "load_residual_sign": ("reshape(-1) - s * f)", "reshape(-1) + s * f)", ["test_oracle_load.py"]),
    "load_energy_not_scaled_by_step": ("- s * (f @ uu)", "- (f @ uu)", ["test_oracle_load.py"]),
    "load_energy_sign": ("- s * (f @ uu)", "+ s * (f @ uu)", ["test_oracle_load.py"]),
    "predictor_rhs_sign": ("* f - fem.hvp(u, dc).reshape(-1))", "* f + fem.hvp(u, dc).reshape(-1))",
                           ["test_oracle_newton.py"]),
    "predictor_not_applied": ("u_try = u + dc + free * df", "u_try = u + dc", ["test_oracle_newton.py"]),
    "forcing_held_at_eta_max": ("eta = opts.ew_gamma * (rn / rn_prev) ** opts.ew_alpha", "eta = opts.eta_max",
                                ["test_oracle_newton.py"]),
}


@pytest.mark.parametrize("name", sorted(PY_MUTATIONS))
def test_pins_catch_planted_mistake_in_solve(name, tmp_path):
    import shutil

    from oracle import build as _build
    old, new, pin_files = PY_MUTATIONS[name]
    for d in ("oracle", "tests", "paper_2602_12365_amd"):
        (tmp_path / d).mkdir()
        for f in os.listdir(os.path.join(ROOT, d)):
            if f.endswith(".py"):
                shutil.copy(os.path.join(ROOT, d, f), tmp_path / d / f)
    fem_py = tmp_path / "oracle" / "fem.py"
    src = fem_py.read_text()
    assert src.count(old) == 1, f"mutation anchor not found once: {old!r}"
    fem_py.write_text(src.replace(old, new))
    env = dict(os.environ, EFEM_ORACLE_LIB=_build.build(), OMP_NUM_THREADS="2")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"]
                         + [str(tmp_path / "tests" / f) for f in pin_files],
                         cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=300)
    assert "passed" in res.stdout or "failed" in res.stdout, res.stdout[-2000:] + res.stderr[-2000:]
    assert res.returncode != 0, f"pins did not catch mutation {name}:\n{res.stdout[-2000:]}"
