"""Planted mistakes in the oracle must be caught by its pins.

Each mutant is a copy of ``oracle/adot_oracle.c`` with one plausible slip (a
dropped term, a wrong sign, index or operand order) compiled on the CPU into a
temporary library; ``oracle_battery.py`` runs the fast pins against it in a
subprocess.  The unmodified oracle must pass the same battery.
"""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "adot_oracle.c")

MUTANTS = {
    "k1_drops_factor_3": ("3.0 + Fr * Fr + 3.0 * p->xi * dqs_dq", "3.0 + Fr * Fr + p->xi * dqs_dq"),
    "k2_sign_of_cubic": ("-2.0 * Fr * Fr * Fr + 18.0", "2.0 * Fr * Fr * Fr + 18.0"),
    "k2_times_c": ("27.0 * p->xi * dqs_dh / c", "27.0 * p->xi * dqs_dh * c"),
    "k2_drops_one": ("18.0 * Fr * (1.0 + p->xi * dqs_dq)", "18.0 * Fr * (p->xi * dqs_dq)"),
    "lambda1_angle": ("cos(phi / 3.0 - OR_PI / 3.0)", "cos(phi / 3.0 - OR_PI / 6.0)"),
    "lambda3_sign": ("2.0 / 3.0 * Fr + 2.0 / 3.0 * sqrt(k1)", "2.0 / 3.0 * Fr - 2.0 / 3.0 * sqrt(k1)"),
    "phi_not_divided": ("cos(phi / 3.0));", "cos(phi));"),
    "acos_arg_sqrt": ("k2 / sqrt(4.0 * k1 * k1 * k1)", "k2 / sqrt(4.0 * k1 * k1)"),
    "R_row3_sign": ("(u - lam[m]) * (u - lam[m]) / c2 - 1.0", "(u - lam[m]) * (u - lam[m]) / c2 + 1.0"),
    "R_row2": ("R[1 * 3 + m] = lam[m];", "R[1 * 3 + m] = u - lam[m];"),
    "Rinv_col2_sign": ("(2.0 * u - lj - lk) / den", "(2.0 * u - lj + lk) / den"),
    "Rinv_col1": ("(c2 - u * u + lj * lk) / den", "(c2 + lj * lk) / den"),
    "Rinv_perm": ("int k = (i < 2) ? i + 2 : i - 1;", "int k = (i < 2) ? i + 1 : i - 1;"),
    "abs_without_abs": ("R[r * 3 + m] * fabs(lam[m])", "R[r * 3 + m] * lam[m]"),
    "abs_transposed_operand": ("RL[r * 3 + m] * Rinv[m * 3 + cc]", "RL[r * 3 + m] * Rinv[cc * 3 + m]"),
    "flux_c2_plus_u2": ("A[3] = c2 - u * u;", "A[3] = c2 + u * u;"),
    "flux_no_bed_term": ("A[5] = c2;", "A[5] = 0.0;"),
    "flux_no_xi": ("A[6] = p->xi * dqs_dh;", "A[6] = dqs_dh;"),
    "grass_dh_sign": ("*dqs_dh = -3.0 * qs / h;", "*dqs_dh = 3.0 * qs / h;"),
    "grass_dq_no_h": ("*dqs_dq = 3.0 * Ag * u * u / h;", "*dqs_dq = 3.0 * Ag * u * u;"),
    "fluct_no_half": ("Dm[r] = 0.5 * Sm[r];", "Dm[r] = Sm[r];"),
    "fluct_node_is_weight": ("Psi[r] = Wm[r] + s[k] * dW[r];", "Psi[r] = Wm[r] + w[k] * dW[r];"),
    "fluct_minus_swapped": ("(A[r * 3 + cc] - absA[r * 3 + cc])", "(absA[r * 3 + cc] - A[r * 3 + cc])"),
    "gauss_weight_unscaled": ("w[G - 1 - i] = 0.5 * wi;", "w[G - 1 - i] = wi;"),
    "update_edge_index": ("c->Dm[0 * E + i + 1] + c->Dp[0 * E + i]", "c->Dm[0 * E + i] + c->Dp[0 * E + i + 1]"),
    "update_sign": ("c->hn[i] = c->h[i] - r *", "c->hn[i] = c->h[i] + r *"),
    "update_z_uses_q_row": ("c->Dm[2 * E + i + 1] + c->Dp[2 * E + i]", "c->Dm[1 * E + i + 1] + c->Dp[2 * E + i]"),
    "dt_without_cfl": ("double dt = ch->cfl * ch->dx / amax;", "double dt = ch->dx / amax;"),
    "amax_ignores_lambda3": ("if (fabs(lam[2]) > a) a = fabs(lam[2]);", ""),
    "grass_thr_no_threshold": ("double ex = fabs(u) - p->par[0];", "double ex = fabs(u);"),
    "power_exponent": ("pow(fabs(u), beta - 1.0)", "pow(fabs(u), beta)"),
    "mpm_h_exponent": ("*dqs_dh = sign_of(q) * dqs_dtheta * (-7.0 / 3.0) * theta / h;",
                       "*dqs_dh = sign_of(q) * dqs_dtheta * (-10.0 / 3.0) * theta / h;"),
    "mpm_q_factor": ("*dqs_dq = dqs_dtheta * 2.0 * theta / fabs(q);",
                     "*dqs_dq = dqs_dtheta * theta / fabs(q);"),
    "vanrijn_exponent": ("pow(T, 1.1)", "pow(T, 2.1)"),
    "vanrijn_dstar_nu": ("cbrt(p->g * (Sg - 1.0) / (nu * nu))", "cbrt(p->g * (Sg - 1.0) / nu)"),
    "friction_sign": ("c->dt * (-c->p.g * c->h[i] * friction_slope", "c->dt * (c->p.g * c->h[i] * friction_slope"),
    "friction_h_power": ("return q * fabs(q) / (ks * ks * pow(h, 10.0 / 3.0));",
                         "return q * fabs(q) / (ks * ks * pow(h, 7.0 / 3.0));"),
    "fixed_depth_ghost": ("case OR_BC_FIXED_DEPTH: gr[0] = ch->h_out;", "case OR_BC_FIXED_DEPTH: gr[0] = h[N - 1];"),
    "inflow_qh_ghost_depth": ("case OR_BC_INFLOW_QH: gl[0] = ch->h_in;", "case OR_BC_INFLOW_QH: gl[0] = h[0];"),
    "dirichlet_drift_sign": ("gl[2] = ch->dir_l[2] + t * ch->dir_l[3];", "gl[2] = ch->dir_l[2] - t * ch->dir_l[3];"),
    "periodic_ghost_wrong_end": ("case OR_BC_PERIODIC: gl[0] = h[N - 1]; gl[1] = q[N - 1]; gl[2] = z[N - 1];",
                                 "case OR_BC_PERIODIC: gl[0] = h[0]; gl[1] = q[0]; gl[2] = z[0];"),
}


def _build(src_text, out_path):
    cpath = out_path[:-3] + ".c"
    with open(cpath, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", *oracle._CFLAGS, "-o", out_path, cpath, "-lm"])


def _battery(lib_path):
    r = subprocess.run([sys.executable, os.path.join(HERE, "oracle_battery.py"), lib_path],
                       capture_output=True, text=True, timeout=300)
    return r.returncode, r.stdout + r.stderr


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def test_unmodified_oracle_passes_battery(source, tmp_path):
    lib = str(tmp_path / "liboracle_ref.so")
    _build(source, lib)
    rc, out = _battery(lib)
    assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(source, name, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) >= 1, f"mutation site for {name} not found"
    mutated = source.replace(old, new, 1)
    lib = str(tmp_path / f"liboracle_{name}.so")
    _build(mutated, lib)
    rc, out = _battery(lib)
    assert rc != 0, f"mutant {name} survived the pins: {out}"
