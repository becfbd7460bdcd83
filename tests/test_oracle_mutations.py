"""The pins catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's C source (a dropped term, a
flipped sign, a transposed derivative direction, a wrong stencil or quadrature
weight, a missing factor, a wrong exponent, a first-order closure), builds it with gcc and runs the pin file that should catch it against
that build (the oracle module loads the build HOSC_ORACLE_LIB names): the pins must
fail.  A control build of the unmodified source must pass the same files, so a
failure is the mistake's and not the harness's.  Everything runs on the CPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hosc_oracle.c")

# name: (text in the oracle, planted replacement, pin files that must catch it)
MUTANTS = {
    "time part of M18 dropped": (
        "double M18 = 0.5 * dt * ((C->L[c] - C->Lp[c]) / dt);", "double M18 = 0.0;",
        ["test_oracle_expanded_form.py"]),
    "convective sign in the compact bracket": (
        "s += hd2[d] / 12.0 * (D2(f, N, h, i, j, k, d) - C->V[d][c] * D1(f, N, h, i, j, k, d));",
        "s += hd2[d] / 12.0 * (D2(f, N, h, i, j, k, d) + C->V[d][c] * D1(f, N, h, i, j, k, d));",
        ["test_oracle_expanded_form.py"]),
    "convective sign in B": (
        "cd * (D2(x, N, h, i, j, k, d) - C->V[d][c] * D1(x, N, h, i, j, k, d))",
        "cd * (D2(x, N, h, i, j, k, d) + C->V[d][c] * D1(x, N, h, i, j, k, d))",
        ["test_oracle_expanded_form.py"]),
    "cross term M5 dropped": ("s -= M5 * (", "s -= 0.0 * M5 * (", ["test_oracle_closed_form.py"]),
    "derivative directions of p1 swapped": (
        "kk * D1(C->V[0], N, h, i, j, k, 1) + hh * D1(C->V[1], N, h, i, j, k, 0)",
        "kk * D1(C->V[0], N, h, i, j, k, 0) + hh * D1(C->V[1], N, h, i, j, k, 1)",
        ["test_oracle_expanded_form.py"]),
    "sign of the derivative term of alpha": (
        "(Vd * Vd - 2.0 * D1(C->V[d], N, h, i, j, k, d))", "(Vd * Vd + 2.0 * D1(C->V[d], N, h, i, j, k, d))",
        ["test_oracle_expanded_form.py"]),
    "sign of the pressure correction": (
        "S->p[ID(N, i, j, k)] -= P->lambda * div[ID(N, i, j, k)];",
        "S->p[ID(N, i, j, k)] += P->lambda * div[ID(N, i, j, k)];",
        ["test_oracle_pressure_iterations.py"]),
    "weight of the one-sided Nusselt stencil": (
        "- 36.0 * T[ID(N, 2, j, k)]", "- 35.0 * T[ID(N, 2, j, k)]", ["test_oracle_reductions.py"]),
    "viscosity missing from E_FF": (
        "double eff = P->phi * eta[c] * I2[c];", "double eff = P->phi * I2[c];", ["test_oracle_reductions.py"]),
    "sign of the buoyancy": (
        "+ P->Ra * Pr * (T[c] - P->theta_ref));", "- P->Ra * Pr * (T[c] - P->theta_ref));",
        ["test_oracle_physics.py::test_newtonian_reduction"]),
    "power-law exponent n - 1 instead of (n - 1)/2": (
        "double ex = 0.5 * (P->n_pl - 1.0);", "double ex = (P->n_pl - 1.0);", ["test_oracle_reductions.py"]),
    "factor 2 of the strain invariant's diagonal dropped": (
        "return 2.0 * (ux * ux + vy * vy + wz * wz) +", "return (ux * ux + vy * vy + wz * wz) +",
        ["test_oracle_physics.py::test_strain_invariant_is_twice_d_colon_d"]),
    "factor 2 of the viscous source's diagonal dropped": (
        "Pr * (2.0 * ux * ex + (uy + vx) * ey", "Pr * (ux * ex + (uy + vx) * ey",
        ["test_oracle_physics.py::test_viscous_source_is_the_stress_divergence_part"]),
    "first-order closure on a z wall": (
        "f[ID(N, i, j, 0)] = (4.0 * f[ID(N, i, j, 1)] - f[ID(N, i, j, 2)]) / 3.0;",
        "f[ID(N, i, j, 0)] = f[ID(N, i, j, 1)];", ["test_oracle_physics.py::test_symmetry_every_step"]),
    "middle Simpson weight": (
        "wq[q + 1] += 4.0 * h / 3.0;", "wq[q + 1] += 2.0 * h / 3.0;", ["test_oracle_reductions.py"]),
    "Bejan ratio taken from the friction part": (
        "double be = el > 0.0 ? eht / el : 1.0;", "double be = el > 0.0 ? (el - eht) / el : 1.0;",
        ["test_oracle_reductions.py"]),
    "relaxation weights the other way round": (
        "eta[c] = P->eta_relax * eta[c] + (1.0 - P->eta_relax) * S->etap[c];",
        "eta[c] = (1.0 - P->eta_relax) * eta[c] + P->eta_relax * S->etap[c];",
        ["test_oracle_eta_relax.py::test_relaxation_continuous_at_one"]),
    "source bracket without its time part": (
        "s += 0.5 * C->dt * ((f[c] - fp[c]) / C->dt);", "s += 0.0;", ["test_oracle_expanded_form.py"]),
    "cross term M7 dropped": ("s -= M7 * (", "s -= 0.0 * M7 * (", ["test_oracle_closed_form.py"]),
    "E_HT without its z component": (
        "double eht = tx * tx + ty * ty + tz * tz;", "double eht = tx * tx + ty * ty;", ["test_oracle_reductions.py"]),
    "cold-wall Nusselt sign": ("nc[j + (size_t)N * k] = -dc;", "nc[j + (size_t)N * k] = dc;",
                               ["test_oracle_reductions.py"]),
    "y term of the divergence dropped": (
        "double D = D1(trial[0], N, h, i, j, k, 0) + D1(trial[1], N, h, i, j, k, 1)",
        "double D = D1(trial[0], N, h, i, j, k, 0) + 0.0 * D1(trial[1], N, h, i, j, k, 1)",
        ["test_oracle_pressure_iterations.py"]),
    "first-order closure on every y and z wall": (
        "static void theta_yz_closure(double *f, int N)\n{\n",
        "static void theta_yz_closure(double *f, int N)\n{\n"
        "    for (int i = 1; i < N - 1; ++i) {\n"
        "        for (int j = 1; j < N - 1; ++j) {\n"
        "            f[ID(N, i, j, 0)] = f[ID(N, i, j, 1)];\n"
        "            f[ID(N, i, j, N - 1)] = f[ID(N, i, j, N - 2)];\n"
        "        }\n"
        "        for (int k = 0; k < N; ++k) {\n"
        "            f[ID(N, i, 0, k)] = f[ID(N, i, 1, k)];\n"
        "            f[ID(N, i, N - 1, k)] = f[ID(N, i, N - 2, k)];\n"
        "        }\n"
        "    }\n"
        "    return;\n",
        ["test_oracle_physics.py::test_theta_wall_closure_exact_on_quadratics"]),
    "first-order closure of p on every wall": (
        "static void pressure_closure(double *p, int N)\n{\n",
        "static void pressure_closure(double *p, int N)\n{\n"
        "    for (int k = 0; k < N; ++k)\n"
        "        for (int j = 0; j < N; ++j)\n"
        "            for (int i = 0; i < N; ++i) {\n"
        "                const int ii = i == 0 ? 1 : (i == N - 1 ? N - 2 : i);\n"
        "                const int jj = j == 0 ? 1 : (j == N - 1 ? N - 2 : j);\n"
        "                const int kk = k == 0 ? 1 : (k == N - 1 ? N - 2 : k);\n"
        "                p[ID(N, i, j, k)] = p[ID(N, ii, jj, kk)];\n"
        "            }\n"
        "    return;\n",
        ["test_oracle_physics.py::test_pressure_wall_closure_exact_on_quadratics"]),
    "level n-1 sources not copied at the first step": (
        "        memcpy(S->Eup, Eu, n3 * sizeof(double));\n", "",
        ["test_oracle_physics.py::test_first_step_takes_level_n_minus_1_equal_to_level_n"]),
    "level n-1 viscosity not copied at the first step": (
        "        memcpy(S->etap, eta, n3 * sizeof(double));\n", "",
        ["test_oracle_physics.py::test_first_step_takes_level_n_minus_1_equal_to_level_n"]),
    "x and y velocities swapped in the energy convection": (
        "Ct->V[0] = S->u; Ct->V[1] = S->v;", "Ct->V[0] = S->v; Ct->V[1] = S->u;", ["test_oracle_expanded_form.py"]),
    "momentum convection coefficient without L": (
        "cs->Gm[q] = S->u[q] * cs->Lm[q];", "cs->Gm[q] = S->u[q];", ["test_oracle_expanded_form.py"]),
    "energy equation with L = 1/Pr": ("cs->one[q] = 1.0;", "cs->one[q] = 1.0 / P->Pr;", ["test_oracle_expanded_form.py"]),
    "level n-1 momentum L taken from level n": (
        "cs->Lmp[q] = 1.0 / (P->Pr * S->etap[q]);", "cs->Lmp[q] = cs->Lm[q];", ["test_oracle_expanded_form.py"]),
    "first-order one-sided wall derivative": (
        "if (idx == 0) return (-3.0 * f[c] + 4.0 * f[c + s] - f[c + 2 * s]) / (2.0 * h);",
        "if (idx == 0) return (f[c + s] - f[c]) / h;", ["test_oracle_reductions.py"]),
    "viscosity missing from the pressure term of the momentum sources": (
        "Eu[c] = L * (-px + Pr * (2.0 * ux * ex + (uy + vx) * ey + (uz + wx) * ez));",
        "Eu[c] = -px / Pr + L * Pr * (2.0 * ux * ex + (uy + vx) * ey + (uz + wx) * ez);",
        ["test_oracle_physics.py::test_momentum_sources_times_pr_eta_are_the_unnormalised_right_side",
         "test_oracle_physics.py::test_one_momentum_step_follows_the_momentum_equations"]),
    "viscosity missing from the buoyancy": (
        "Ev[c] = L * (-py + Pr * ((uy + vx) * ex + 2.0 * vy * ey + (vz + wy) * ez) + P->Ra * Pr * (T[c] - P->theta_ref));",
        "Ev[c] = L * (-py + Pr * ((uy + vx) * ex + 2.0 * vy * ey + (vz + wy) * ez)) + P->Ra * (T[c] - P->theta_ref);",
        ["test_oracle_physics.py::test_momentum_sources_times_pr_eta_are_the_unnormalised_right_side",
         "test_oracle_physics.py::test_one_momentum_step_follows_the_momentum_equations"]),
    "largest local Nusselt number taken on the cold wall": (
        "if (-dh > numax_local) numax_local = -dh;", "if (-dc > numax_local) numax_local = -dc;",
        ["test_oracle_reductions.py"]),
    "steady residual divided by the old field": (
        "den += b[q] * b[q]; }", "den += a[q] * a[q]; }",
        ["test_oracle_physics.py::test_steady_residual_is_the_relative_change_of_each_field"]),
}


def _build(src_text, out_dir, name):
    c = os.path.join(out_dir, name + ".c")
    so = os.path.join(out_dir, name + ".so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", so, c, "-lm"], check=True,
                   capture_output=True)
    return so


def _pins(so, files, extra=()):
    env = dict(os.environ, HOSC_ORACLE_LIB=so, OMP_NUM_THREADS="4")
    p = subprocess.run([sys.executable, "-m", "pytest", *[os.path.join("tests", f) for f in files], "-q", "-m",
                        "not gpu", "-p", "no:cacheprovider", *extra], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return p.returncode, p.stdout


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def test_control_build_passes(source, tmp_path):
    so = _build(source, str(tmp_path), "control")
    files = sorted({f for _, _, fs in MUTANTS.values() for f in fs})
    rc, out = _pins(so, files, ("-k", "not steady_state_wall"))     # the slow steady-state pin is not needed here
    assert rc == 0, out[-2000:]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(source, tmp_path, name):
    old, new, files = MUTANTS[name]
    assert source.count(old) == 1, name
    so = _build(source.replace(old, new), str(tmp_path), "mutant")
    rc, out = _pins(so, files)
    assert rc == 1 and "failed" in out, (name, out[-2000:])
