"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of ``oracle/oif_oracle.c`` (on the CPU,
never in the product code), builds it, and runs the oracle pin suite against
that library in a subprocess; the suite must fail.  A mutation that survives
means some part of the oracle is not pinned.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oif_oracle.c")
PIN_FILES = ["tests/test_oracle_mesh.py", "tests/test_oracle_lb.py", "tests/test_oracle_coupling.py",
             "tests/test_oracle_conservative.py", "tests/test_oracle_boundaries.py",
             "tests/test_oracle_mrt_verlet.py", "tests/test_oracle_repulsion.py"]

MUTATIONS = {
    "pair_first_setting": ("            r = &s->pair[k];\n    return r;",
                           "            if (!r) r = &s->pair[k];\n    return r;"),
    "wall_first_setting": ("if (s->wall[k].type_a == s->o_type[o]) ss = &s->wall[k];",
                           "if (s->wall[k].type_a == s->o_type[o] && !ss) ss = &s->wall[k];"),
    "pair_order_matters": ("(s->pair[k].type_a == ta && s->pair[k].type_b == tb) ||\n            (s->pair[k].type_a == tb && s->pair[k].type_b == ta)",
                           "(s->pair[k].type_a == ta && s->pair[k].type_b == tb)"),
    "kappa_exponent": ("(lambda + pow(lambda, -3.0))", "(lambda + pow(lambda, -2.0))"),
    "stretch_sign": ("double f = ks * kap * (L - L0[e]) / L0[e];",
                     "double f = ks * kap * (L0[e] - L) / L0[e];"),
    "stretch_denominator": ("double f = ks * kap * (L - L0[e]) / L0[e];",
                            "double f = ks * kap * (L - L0[e]) / L;"),
    "bend_wing_normal": ("F[3 * D + c] += f * n2[c];", "F[3 * D + c] += f * n1[c];"),
    "bend_split": ("F[3 * B + c] -= 0.5 * f * (n1[c] + n2[c]);",
                   "F[3 * B + c] -= f * (n1[c] + n2[c]);"),
    "dihedral_sign": ("return M_PI + atan2(dot3(m, e), dot3(n1, n2));",
                      "return M_PI - atan2(dot3(m, e), dot3(n1, n2));"),
    "local_area_denominator": ("double coef = -kal * (S - S0[t]) / S;",
                               "double coef = -kal * (S - S0[t]) / S0[t];"),
    "global_area_denominator": ("double coef = -kag * (Sg - Sg0) / Sg;",
                                "double coef = -kag * (Sg - Sg0) / Sg0;"),
    "volume_force_inward": ("coef * S * (-n_in[c]) / 3.0", "coef * S * (n_in[c]) / 3.0"),
    "volume_force_split": ("coef * S * (-n_in[c]) / 3.0", "coef * S * (-n_in[c]) / 2.0"),
    "volume_sign": ("V += -dot3(at, bc) / 6.0;", "V += dot3(at, bc) / 6.0;"),
    "equilibrium_coefficient": ("4.5 * eu * eu", "4.0 * eu * eu"),
    "guo_prefactor": ("src *= (1.0 - 0.5 / tau) * w;", "src *= w;"),
    "guo_second_order_term": ("(3.0 * (e[c] - u[c]) + 9.0 * eu * e[c])",
                              "(3.0 * (e[c] - u[c]))"),
    "lb_velocity_half_force": ("u[c] = (j[c] + 0.5 * F[c]) / rho;", "u[c] = j[c] / rho;"),
    "bounce_back_direction": ("nout[opposite(i) * N + p] = ns;", "nout[i * N + p] = ns;"),
    "stream_direction": ("int xd = wrap(x + EV[i][0], L->nx);", "int xd = wrap(x - EV[i][0], L->nx);"),
    "weight_table": ("return 1.0 / 36.0;", "return 1.0 / 32.0;"),
    "drag_sign": ("drag[c] = L->xi * (V[c] - uj[c]);", "drag[c] = L->xi * (uj[c] - V[c]);"),
    "interp_uniform": ("uj[c] += w[k] * u[c * N + idx[k]];", "uj[c] += 0.125 * u[c * N + idx[k]];"),
    "spread_uniform": ("G[c * N + idx[k]] += w[k] * drag[c];",
                       "G[c * N + idx[k]] += 0.125 * drag[c];"),
    "node_offset": ("double s = X[c] - 0.5;", "double s = X[c];"),
    "interp_full_force": ("for (int c = 0; c < 3; ++c) u[c * N + p] = (j[c] + 0.5 * F[c]) / r;",
                          "for (int c = 0; c < 3; ++c) u[c * N + p] = (j[c] + F[c]) / r;"),
    "mass_ignored": ("V[3 * j + c] += Ft / m;", "V[3 * j + c] += Ft;"),
    "bend_gradient_feet_swapped": ("double gB = -(1.0 - aA) * gA - (1.0 - aD) * gD;",
                                   "double gB = -aA * gA - aD * gD;"),
    "bend_gradient_wing_height": ("double gA = -n1[c] / hA, gD = -n2[c] / hD;",
                                  "double gA = -n1[c] / hA, gD = -n2[c] / hA;"),
    "bend_gradient_no_hbar": ("double dEdt = kb * hbar[e] * (theta - theta0[e]) / theta0[e];",
                              "double dEdt = kb * (theta - theta0[e]) / theta0[e];"),
    "wing_height_sum": ("hbar[e] = (tri_area(x, t1) + tri_area(x, t2)) / norm3(bc);",
                        "hbar[e] = (tri_area(x, t1) + tri_area(x, t2)) / (2.0 * norm3(bc));"),
    "balanced_rms_divisor": ("ms += dot3(w[s], w[s]) / 3.0;", "ms += dot3(w[s], w[s]) / 2.0;"),
    "balanced_unit_vectors": ("double l = balanced ? sqrt(ms) : norm3(w[s]);", "double l = norm3(w[s]);"),
    "moving_wall_sign": ("nout[opposite(i) * N + p] = ns - 6.0 * w * L->rho0 * euw;",
                         "nout[opposite(i) * N + p] = ns + 6.0 * w * L->rho0 * euw;"),
    "moving_wall_factor": ("nout[opposite(i) * N + p] = ns - 6.0 * w * L->rho0 * euw;",
                           "nout[opposite(i) * N + p] = ns - 3.0 * w * L->rho0 * euw;"),
    "obstacle_bounce_direction": ("nout[opposite(i) * N + p] = ns - 6.0 * w * L->rho0 * euw;",
                                  "nout[i * N + p] = ns - 6.0 * w * L->rho0 * euw;"),
    "rhomboid_open_faces": ("s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0 && u >= 0.0 && u <= 1.0",
                            "s > 0.0 && s < 1.0 && t > 0.0 && t < 1.0 && u > 0.0 && u < 1.0"),
    "wall_closed_half_space": ("dot3(r, normal) / len - dist < 0.0)", "dot3(r, normal) / len - dist <= 0.0)"),
    "solid_velocity_ignored": ("for (int c = 0; c < 3; ++c) u[c * N + p] = L->wall_u[3 * L->solid[p] + c];",
                               "for (int c = 0; c < 3; ++c) u[c * N + p] = 0.0;"),
    "spread_into_solid": ("if (L->solid && L->solid[idx[k]]) continue;", "if (0) continue;"),
    "solid_nodes_updated": ("if (L->solid && L->solid[p]) {  /* obstacle node: not updated */", "if (0) {"),
    "drift_before_kick": ("V[3 * j + c] += Ft / m;\n                        X[3 * j + c] += V[3 * j + c];",
                          "X[3 * j + c] += V[3 * j + c];\n                        V[3 * j + c] += Ft / m;"),
    "mrt_bulk_shear_swapped": ("double g = (k == 4) ? L->gamma_bulk : L->gamma_shear;",
                               "double g = (k == 4) ? L->gamma_shear : L->gamma_bulk;"),
    "mrt_force_factor": ("0.5 * (1.0 + g) * phi[k]", "0.5 * phi[k]"),
    "mrt_ghost_parity": ("for (int k = 10; k <= 15; ++k) ms[k] = L->gamma_odd * m[k];",
                         "for (int k = 10; k <= 15; ++k) ms[k] = L->gamma_even * m[k];"),
    "mrt_momentum_no_force": ("ms[1 + c] = m[1 + c] + F[c];", "ms[1 + c] = m[1 + c];"),
    "mrt_basis_not_orthogonal": ("case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;",
                                 "case 16: return 3.0 * c2 * c2 - 5.0 * c2 + 1.0;"),
    "mrt_equilibrium_without_uu": ("Pi[a][b] = rho * u[a] * u[b] + (a == b ? rho / 3.0 : 0.0);",
                                   "Pi[a][b] = (a == b ? rho / 3.0 : 0.0);"),
    "verlet_full_first_kick": ("V[3 * j + c] += 0.5 * s->Fprev[3 * j + c] / m;",
                               "V[3 * j + c] += s->Fprev[3 * j + c] / m;"),
    "verlet_force_not_carried": ("s->Fprev[3 * j + c] = Ft;", "s->Fprev[3 * j + c] = 0.0;"),
    "verlet_full_second_kick": ("V[3 * j + c] += 0.5 * Ft / m;", "V[3 * j + c] += Ft / m;"),
    "soft_sphere_exponent": ("pow(e, -(ss->n + 1.0))", "pow(e, -ss->n)"),
    "soft_sphere_offset_ignored": ("double e = d - ss->offset;", "double e = d;"),
    "pair_no_minimum_image": ("if (periodic[c]) r[c] -= box[c] * floor(r[c] / box[c] + 0.5);",
                              "if (0) r[c] -= box[c] * floor(r[c] / box[c] + 0.5);"),
    "pair_third_law": ("F[3 * k + c] -= f[c];", "F[3 * k + c] += f[c];"),
    "rhomboid_edges_skipped": ("for (int k = 0; k < 3; ++k)            /* edges along E[k] */",
                               "for (int k = 0; k < 0; ++k)            /* edges along E[k] */"),
    "zwall_direction": ("double up[3] = {0, 0, 1}, down[3] = {0, 0, -1};",
                        "double up[3] = {0, 0, -1}, down[3] = {0, 0, 1};"),
    "touched_double_count": ("            if (!mark[idx[k]]) {", "            if (1) {"),
    "repulsion_not_applied": (" + s->o_fext[3 * o + c] + s->Frep[3 * j + c];", " + s->o_fext[3 * o + c];"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    mutated = src.replace(old, new)
    cfile = tmp_path / "oif_oracle.c"
    cfile.write_text(mutated)
    (tmp_path / "oif_oracle.h").write_text(open(SRC[:-2] + ".h").read())
    so = tmp_path / "liboif_oracle_mut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                    "-ffp-contract=off", "-o", str(so), str(cfile), "-lm"], check=True)
    env = dict(os.environ, OIF_ORACLE_LIB=str(so), PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PIN_FILES], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"
