"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake (a dropped term, a wrong sign, a
wrong index, a transposed operand, a wrong weight) in a temporary copy of
``oracle/ppml_oracle.c``, compiles it, and runs the pin suite on it in a
child process.  The case passes when at least one pin fails -- i.e. the pins
would have caught that mistake in the oracle.
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ppml_oracle.c")

# (id, text in the oracle, replacement)
MUTANTS = [
    ("avg_left_jump_sign", "    double d = qR - qL;\n    double w = 1.0 - (2.0 * z) / 3.0;\n    return qR",
     "    double d = qL - qR;\n    double w = 1.0 - (2.0 * z) / 3.0;\n    return qR"),
    ("avg_right_q6_sign", "return qL + (0.5 * z) * (d + q6 * w);", "return qL + (0.5 * z) * (d - q6 * w);"),
    ("avg_left_weight", "    return qR - (0.5 * z) * (d - q6 * w);", "    return qR - z * (d - q6 * w);"),
    ("avg_right_curvature_term", "double w = 1.0 - (2.0 * z) / 3.0;\n    return qL",
     "double w = 1.0 - z / 3.0;\n    return qL"),
    ("limiter_factor", "b = 2.0 * fabs(dplus)", "b = fabs(dplus)"),
    ("limiter_index", "double dminus = q[j] - q[j - 1];", "double dminus = q[j + 1] - q[j - 1];"),
    ("limiter_no_extremum_test", "if (dplus * dminus > 0.0) {", "if (1) {"),
    ("interface_coeff", "- (dm[j + 1] - dm[j]) / 6.0;", "- (dm[j + 1] - dm[j]) / 3.0;"),
    ("interface_slope_index", "- (dm[j + 1] - dm[j]) / 6.0;", "- (dm[j + 1] - dm[j - 1]) / 6.0;"),
    ("steepen_left_operand", "l = 3.0 * c - 2.0 * r;", "l = 3.0 * c - 2.0 * l;"),
    ("steepen_swapped", "if (d * s6 > d * d)", "if (d * s6 < d * d)"),
    ("flatten_test", "if ((r - c) * (c - l) <= 0.0) {", "if ((r - c) * (c - l) >= 0.0) {"),
    ("q6_sum", "q6[j] = 6.0 * (c - 0.5 * (l + r));", "q6[j] = 6.0 * (c - 0.5 * (l - r));"),
    ("riemann_V_sign", "+ (pm - pp) / (2.0 * Z);", "+ (pp - pm) / (2.0 * Z);"),
    ("riemann_P_sign", "(0.5 * Z) * (vm - vp);", "(0.5 * Z) * (vp - vm);"),
    ("riemann_V_impedance", "+ (pm - pp) / (2.0 * Z);", "+ (pm - pp) / (2.0);"),
    ("lambda_no_gamma", "double lam = sqrt(gam * C / A);", "double lam = sqrt(C / A);"),
    ("impedance_no_B", "double Z = sqrt(gam * A * C) / B;", "double Z = sqrt(gam * A * C);"),
    ("roe_weights_transposed", "double A = qr[j] * sL + qr[j + 1] * sR;", "double A = qr[j] * sR + qr[j + 1] * sL;"),
    ("euler_state_index", "double vp = og_avg_right(b.qL[0][j + 1], b.qR[0][j + 1], b.q6[0][j + 1], z);",
     "double vp = og_avg_right(b.qL[0][j], b.qR[0][j], b.q6[0][j], z);"),
    ("euler_work_term", "(Pi[j] * Vi[j] - Pi[j - 1] * Vi[j - 1]) / h;", "(Pi[j] * Vi[j] - Pi[j - 1] * Vi[j]) / h;"),
    ("eps_equation_gamma", "((tau * (gam - 1.0)) * U[F_E][q])", "((tau * gam) * U[F_E][q])"),
    ("force_sign", "g->W[F_MX + a][q] - (tau * r) * gr[a];", "g->W[F_MX + a][q] + (tau * r) * gr[a];"),
    ("force_log_q", "gr[2] = a * (Z / q2);", "gr[2] = a * Z;"),
    ("lagr_weights_transposed", "double v = (vt[j] * sq[j] + vt[j + 1] * sq[j + 1]) / (sq[j] + sq[j + 1]);",
     "double v = (vt[j] * sq[j + 1] + vt[j + 1] * sq[j]) / (sq[j] + sq[j + 1]);"),
    ("lagr_downwind", "if (v >= 0.0) fs = og_avg_left", "if (v < 0.0) fs = og_avg_left"),
    ("lagr_z_signed", "double z = fabs(v) * tau / h;", "double z = v * tau / h;"),
    ("transverse_3d_weights", "return 0.0625 * corners + 0.125 * edges + 0.25 * V[q];",
     "return 0.0625 * corners + 0.0625 * edges + 0.5 * V[q];"),
    ("transverse_3d_index", "double corners = V[q + s1 + s2] + V[q + s1 - s2]",
     "double corners = V[q + s1 + s1] + V[q + s1 - s2]"),
    ("transverse_2d_weights", "return 0.25 * (V[q + s1] + V[q - s1]) + 0.5 * V[q];",
     "return 0.5 * (V[q + s1] + V[q - s1]) + 0.0 * V[q];"),
    ("kinetic_factor", "double kin = (mx * mx + my * my + mz * mz) / (2.0 * r);",
     "double kin = (mx * mx + my * my + mz * mz) / r;"),
    ("vacuum_speed", "double sc = sqrt(2.0 * (E - eps)) / w;", "double sc = sqrt(E - eps) / w;"),
    ("periodic_wrap", "if (bc_lo == BC_PERIODIC) return G + ((((i - G) % n) + n) % n);",
     "if (bc_lo == BC_PERIODIC) return G + ((((i - G + 1) % n) + n) % n);"),
    ("outflow_copy", "if (bc_hi == BC_OUTFLOW) return G + n - 1;", "if (bc_hi == BC_OUTFLOW) return G + n - 2;"),
    ("reflect_mirror", "return 2 * G - 1 - i; /* mirror */", "return 2 * G - i; /* mirror */"),
    ("cfl_sum", "return g->cfl * h / (vm + cm);", "return g->cfl * h / cm;"),
    ("cfl_h_max", "if (g->h[a] < h) h = g->h[a];", "if (g->h[a] > h) h = g->h[a];"),
    ("pressure_eos", ": (gam - 1.0) * U[F_E][q];", ": gam * U[F_E][q];"),
    ("euler_h", "g->acc[a][q] = (Pi[j] - Pi[j - 1]) / h;", "g->acc[a][q] = (Pi[j] - Pi[j - 1]);"),
    ("inflow_side", "const double *st = g->inflow[2 * a + (i >= G + n ? 1 : 0)];",
     "const double *st = g->inflow[2 * a + (i >= G + n ? 0 : 1)];"),
    ("inflow_energy", "st[F_ET] = e + ke;", "st[F_ET] = e;"),
    ("multipole_no_half", "/ (2.0 * r2 * r);", "/ (r2 * r);"),
    ("multipole_cross_sign", "2.0 * (x * y * mom[4] + x * z * mom[5] + y * z * mom[6])",
     "2.0 * (x * y * mom[4] - x * z * mom[5] + y * z * mom[6])"),
    ("moment_Iy_axes", "mom[2] += (x * x + z * z) * m;", "mom[2] += (x * x + y * y) * m;"),
    ("poisson_eigen_sign", "double lam = -6.0 * (1.0 - prod);", "double lam = 6.0 * (1.0 - prod);"),
    ("poisson_eigen_period", "double sy = sin(M_PI * (double)(j + 1) / (2.0 * (double)(n1 + 1)));",
     "double sy = sin(M_PI * (double)(j + 1) / (2.0 * (double)(n1)));"),
    ("poisson_norm_axis", "* (2.0 / (double)(n1 + 1)) *", "* (2.0 / (double)(n0 + 1)) *"),
    ("stencil_edge_weight", "(nd == 2 ? 1.0 / 9.0 : 1.0 / 36.0)", "(nd == 2 ? 1.0 / 36.0 : 1.0 / 9.0)"),
    ("sine_table_period", "S[(j - 1) * n + (k - 1)] = sin(M_PI * (double)(j * k) / (double)(n + 1));",
     "S[(j - 1) * n + (k - 1)] = sin(M_PI * (double)(j * k) / (double)(n));"),
    ("poisson_rhs_h", "4.0 * M_PI * G * h * h *", "4.0 * M_PI * G * h *"),
    ("gravity_gradient_h", "double h2 = 2.0 * g->h[0];", "double h2 = g->h[0];"),
    ("gravity_gradient_axis", "gr[1] = (g->phi[pidx(g, i, j + 1, k)] - g->phi[pidx(g, i, j - 1, k)]) / h2;",
     "gr[1] = (g->phi[pidx(g, i + 1, j, k)] - g->phi[pidx(g, i - 1, j, k)]) / h2;"),
    ("halo_mass_sign", "(u - atan(u));", "(u + atan(u));"),
    ("halo_r0_power", "g->pot[0] * (r0 * r0 * r0) *", "g->pot[0] * (r0 * r0) *"),
    ("halo_truncation", "double u = (r < g->pot[2] ? r : g->pot[2]) / r0;", "double u = r / r0;"),
    ("iso_pressure", "qp[m] = g->iso ? (g->cs * g->cs) * r", "qp[m] = g->iso ? g->cs * r"),
    ("iso_riemann_gamma", "const double gam = g->iso ? 1.0 : g->gamma;", "const double gam = g->gamma;"),
    ("iso_cfl_speed", "double c = sqrt((g->iso ? 1.0 : g->gamma) * p / r);", "double c = sqrt(g->gamma * p / r);"),
    ("iso_cfl_pressure", "double p = g->iso ? (g->cs * g->cs) * r :", "double p = g->iso ? g->cs * r :"),
    ("totals_skip_row", "for (long j = 0; j < g->n[1]; j++)\n                for (long i = 0; i < g->n[0]; i++) s +=",
     "for (long j = 0; j + 1 < g->n[1]; j++)\n                for (long i = 0; i < g->n[0]; i++) s +="),
    ("totals_ghost_offset", "s += g->U[f][gidx(g, i + g->g[0], j + g->g[1], k + g->g[2])];",
     "s += g->U[f][gidx(g, i + g->g[0] - 1, j + g->g[1], k + g->g[2])];"),
]

RUNNER = r"""
import sys, traceback
sys.path[:0] = [{root!r}, {tests!r}]
import pin_suite, oracle
lib = oracle.load_library({lib!r})
for pin in pin_suite.ALL_PINS:
    try:
        if pin.__name__ == "pin_aksenov":
            pin(lib, small_cfl=False)
        else:
            pin(lib)
    except Exception as exc:  # the pin caught the planted mistake
        print("CAUGHT", pin.__name__, type(exc).__name__)
        sys.exit(0)
print("SURVIVED")
"""


@pytest.mark.parametrize("mid,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(mid, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {mid}"
    mutated = src.replace(old, new, 1)
    assert mutated != src
    c = tmp_path / "mutant.c"
    c.write_text(mutated)
    lib = str(tmp_path / "libmutant.so")
    oracle.build(str(c), lib)
    code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    # a crash of the child (e.g. a NaN-driven fault) also counts as caught
    assert "SURVIVED" not in out, f"mutant {mid} passed every pin:\n{out[-2000:]}"
