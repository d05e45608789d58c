"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of ``oracle/lbm_oracle.c`` (a dropped
term, a wrong sign or index, a transposed operand, a shifted stencil, a wrong
digit in a printed table), builds it on the CPU, and runs the oracle pin tests
against it in a child process: at least one of them must fail.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.c")
PINS = ["tests/test_oracle_sets.py", "tests/test_oracle_collision.py", "tests/test_oracle_stream.py",
        "tests/test_oracle_step.py", "tests/test_oracle_adjoint.py", "tests/test_oracle_moments.py",
        "tests/test_oracle_glc.py", "tests/test_oracle_prandtl.py"]

MUTANTS = {
    "H2_drops_delta": ("double H2 = (xh[a] * xh[b] - kd(a, b)) / (cs * cs);",
                       "double H2 = (xh[a] * xh[b]) / (cs * cs);"),
    "H3_sign": ("double H3 = (xh[a] * xh[b] * xh[g] - (xh[a]", "double H3 = (xh[a] * xh[b] * xh[g] + (xh[a]"),
    "a4_drops_eta2": ("T0 * T0 * eta * eta * Dl);", "0.0 * Dl);"),
    "T_wrong_index": ("xh[a] * xh[d] * kd(b, g)", "xh[a] * xh[d] * kd(a, g)"),
    "a3_drops_term": ("kd(a, g) * u[b] + kd(b, g) * u[a]));", "kd(a, g) * u[b]));"),
    "even_stencil_shifted": ("first = j + fl - n / 2 + 1;", "first = j + fl - n / 2;"),
    "odd_tie_departure_side": ("else c = (llabs(fl) <= llabs(fl + 1)) ? fl : fl + 1;",
                               "else c = (llabs(fl) <= llabs(fl + 1)) ? fl + 1 : fl;"),
    "lagrange_sign": ("num *= (double)(j - nodes[m]) - s;", "num *= (double)(j - nodes[m]) + s;"),
    "bgk_times_tau": ("fout[k] = fin[k] - (fin[k] - eq[k]) / tau;", "fout[k] = fin[k] - (fin[k] - eq[k]) * tau;"),
    "momentum_axis": ("for (int a = 0; a < p->D; ++a) j[a] += p->t.xi[i][a] * fc[i];",
                      "for (int a = 0; a < p->D; ++a) j[a] += p->t.xi[i][0] * fc[i];"),
    "theta_drops_T0": ("e += z2 * fc[i] / p->T0 + fc[p->Q + i];", "e += z2 * fc[i] + fc[p->Q + i];"),
    "table_digit": ("{0.00462962962962958, 2.403092127540177, 0.8892242114059369, -1.5602655313772367}",
                    "{0.00462962962962958, 2.413092127540177, 0.8892242114059369, -1.5602655313772367}"),
    "d2q19_weight": ("push_signs(t, 0.00953510698543825, r3, 2);", "push_signs(t, 0.00935510698543825, r3, 2);"),
    "scale_inverted": ("double lam = p->cs / p->t.cs_tab;", "double lam = p->t.cs_tab / p->cs;"),
    "wrap_off_by_one": ("return (r < 0) ? r + N : r;", "return (r < 0) ? r + N - 1 : r;"),
    "geq_factor": ("out[p->Q + i] = theta * (2.0 * p->Cv - p->D) * out[i];",
                   "out[p->Q + i] = theta * (2.0 * p->Cv) * out[i];"),
    "tau_pressure_inverted": ("tau = 0.5 + (p->c.tau - 0.5) / (rho * theta);",
                              "tau = 0.5 + (p->c.tau - 0.5) * (rho * theta);"),
    "transpose_drops_z_weight": ("li[cell_index(&p, m)] += L[0][kx] * L[1][ky] * L[2][kz] * mi[e];",
                                 "li[cell_index(&p, m)] += L[0][kx] * L[1][ky] * mi[e];"),
    "init_transpose_real_part": ("s += cimag(eq[k]) / ORC_CSTEP * lam0[(int64_t)k * NC + e];",
                                 "s += cimag(eq[k]) / ORC_CSTEP * lam0[(int64_t)k * NC + e] * 0.999;"),
    "d1q5_weight": ("wt[k] = 120.0 / (25.0 * he4 * he4);", "wt[k] = 120.0 / (24.0 * he4 * he4);"),
    "ke_drops_half": ("ke += 0.5 * u2;", "ke += u2;"),
    "first_step_g_reads_f": ("* creal(eq[a * p.Q + i]);", "* creal(eq[i]);"),
    "min_rho_sense": ("if (rr < rmin) rmin = rr;", "if (rr > rmin) rmin = rr;"),
    "min_theta_of_rho": ("if (t < tmin) tmin = t;", "if (rr < tmin) tmin = rr;"),
    "energy_drops_g": ("((p.A == 2) ? creal(fc[p.Q + i]) : 0.0)", "0.0"),
    "momentum_unweighted": ("mom[a] += rr * creal(uu[a]);", "mom[a] += creal(uu[a]);"),
    "glc_points_uniform": ("return 0.5 * (1.0 - cos(pi * (double)m / (double)pp));", "return (double)m / (double)pp;"),
    "glc_shift_sign": ("const double r = glc_point((int)k, pp) - s / (double)pp;",
                       "const double r = glc_point((int)k, pp) + s / (double)pp;"),
    "glc_cell_ceil": ("const double d = floor(r);", "const double d = ceil(r);"),
    "glc_shift_in_nodes": ("- s / (double)pp;", "- s;"),
    "qe_lattice_frame": ("      zeta[a] = p->t.xi[i][a] - u[a];", "      zeta[a] = p->t.xi[i][a];"),
    "qe_f_basis_factor": ("(X - (D + 2.0)) / (2.0 * (D + 2.0));", "(X - (D + 2.0)) / (2.0 * (D + 4.0));"),
    "qe_g_flux_dropped": ("qe[Q + i] = eq[Q + i] + p->t.w[i] * pg;", "qe[Q + i] = eq[Q + i];"),
    "qe_tau_q_inverted": ("const double complex tau_q = 0.5 + (tau - 0.5) / p->c.prandtl;",
                          "const double complex tau_q = 0.5 + (tau - 0.5) * p->c.prandtl;"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found: " + name
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "mutant.so"
    from oracle import oracle as O

    subprocess.check_call(["gcc", *O.GCC_FLAGS, "-o", str(so), str(mut), "-lm"])
    env = dict(os.environ, ORACLE_LIB=str(so), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "mutant %s survived the pins:\n%s" % (name, r.stdout[-2000:])
