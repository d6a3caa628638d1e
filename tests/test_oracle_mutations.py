"""The oracle's pins have teeth: each plausible mistake planted in a copy of
the oracle source (a sign, an index, a dropped term, a swapped operand) must
make at least one pin test fail.  Everything here runs on the CPU; the
mutated libraries live in a temporary directory."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mb_oracle.c")
PACK_SRC = os.path.join(ROOT, "oracle", "pack_oracle.c")
# the adjoint pins run first: they take under a second, and their comparison
# of the tangent step with differences of the forward step also trips on most
# mistakes in the forward step
PINS = ["tests/test_oracle_adjoint.py", "tests/test_oracle_rng.py", "tests/test_oracle_yee.py",
        "tests/test_oracle_bloch.py", "tests/test_oracle_monitors.py"]

# (name, original text, mutated text)
MUTATIONS = [
    ("faraday_sign", "s->Hn[c][x] = H3[c][x] - S * c3[c];", "s->Hn[c][x] = H3[c][x] + S * c3[c];"),
    ("curl_index", "double cx = (Ez[xj] - Ez[x])", "double cx = (Ez[xi] - Ez[x])"),
    ("curl_operand_order", "double cz = (Ey[xi] - Ey[x]) - (Ex[xj] - Ex[x]);",
     "double cz = (Ex[xj] - Ex[x]) - (Ey[xi] - Ey[x]);"),
    ("ampere_index", "curl = (Hz[x] - Hz[at(s, i, j - 1, k)])", "curl = (Hz[x] - Hz[at(s, i - 1, j, k)])"),
    ("ampere_polarisation_sign", "s->f[c][x] = s->Eold[c][x] + ie * (S * curl - dP);", "s->f[c][x] = s->Eold[c][x] + ie * (S * curl + dP);"),
    ("ampere_missing_inv_eps", "s->Eold[c][x] + ie * (S * curl - dP)", "s->Eold[c][x] + (S * curl - dP)"),
    ("lorentz_history", "c[ORC_C_B] * Pprev", "c[ORC_C_B] * P"),
    ("lorentz_inversion_sign", "double dN = s->f[12 + c][x] - s->f[15 + c][x];",
     "double dN = s->f[15 + c][x] - s->f[12 + c][x];"),
    ("lorentz_damping", "c[ORC_C_A] = rnd(s, (2.0 - wa * wa * dt * dt) / D);",
     "c[ORC_C_A] = rnd(s, (2.0 - wa * wa * dt * dt));"),
    ("rate_work_sign", "c[ORC_C_DT10] * n1 - W;", "c[ORC_C_DT10] * n1 + W;"),
    ("rate_dropped_decay", "N[3] = n3 + c[ORC_C_DTWP] * n0 - c[ORC_C_DT32] * n3;",
     "N[3] = n3 + c[ORC_C_DTWP] * n0;"),
    ("rate_work_factor", "double W = c[ORC_C_BETA] * Ebar * dP;", "double W = c[ORC_C_BETA] * Ebar * Ebar * dP;"),
    ("energy_missing_eps", "acc += e * s->f[c][x] * s->f[c][x];", "acc += s->f[c][x] * s->f[c][x];"),
    ("mur_new_neighbour", "E[xb] = Eo[x1] + m * (E[x1] - Eo[xb]);", "E[xb] = Eo[x1] + m * (Eo[x1] - Eo[xb]);"),
    ("mur_coefficient_sign", "return rnd(s, (sp - 1.0) / (sp + 1.0));", "return rnd(s, (1.0 - sp) / (sp + 1.0));"),
    ("dft_sign", "s->spec[o + 1] += e * sin(ph);", "s->spec[o + 1] -= e * sin(ph);"),
    ("dft_time_index", "const double tn = (double)(s->step + 1) * dt;", "const double tn = (double)(s->step) * dt;"),
    ("source_phase", "s->src_amp * sin(s->src_ws * t)", "s->src_amp * cos(s->src_ws * t)"),
    ("philox_weyl", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE86u;"),
    ("philox_word_order", "uint32_t y1 = lo1;", "uint32_t y1 = lo0;"),
    ("rate_work_factor_only", "double W = c[ORC_C_BETA] * Ebar * dP;", "double W = 0.5 * c[ORC_C_BETA] * Ebar * dP;"),
    ("layer_loss_sign", "s->Hn[c][x] = layer_ca(s, a) * H3[c][x]", "s->Hn[c][x] = layer_ca(s, -a) * H3[c][x]"),
    ("layer_e_scale", "layer_cb(s, a) * (ie * (S * curl - dP));", "(ie * (S * curl - dP));"),
    ("layer_h_half_position", "const int half = is_h ? (ax != c) : (ax == c);",
     "const int half = is_h ? (ax == c) : (ax == c);"),
    ("layer_high_side_grading", "if (x > n - L) v += pow((x - (n - L)) / L, (double)s->p.absorb_order);",
     "if (x > n - L) v += pow((n - x) / L, (double)s->p.absorb_order);"),
    ("prepump_fixed_point", "N[2] = rnd(s, dwp * n0 / d21);", "N[2] = rnd(s, dwp * n0 / d32);"),
    ("adjoint_curl_transpose_sign", "htot[cc][x] = w[3 + cc][x] + S * curl_plus(s, u, cc, i, j, k);",
     "htot[cc][x] = w[3 + cc][x] - S * curl_plus(s, u, cc, i, j, k);"),
    ("adjoint_missing_work_term", "e_adj += c[ORC_C_CK] * dN * pn + Wh * c[ORC_C_BETA] * 0.5 * dPf;",
     "e_adj += c[ORC_C_CK] * dN * pn;"),
    ("adjoint_history_coefficient", "z[9 + cc][x] = c[ORC_C_B] * pn;", "z[9 + cc][x] = c[ORC_C_A] * pn;"),
    ("adjoint_eps_derivative", "g_eps[cell] += etot[cc][x] * cb * rhs * (-ie * ie);",
     "g_eps[cell] += etot[cc][x] * cb * rhs * (-ie);"),
    ("adjoint_initial_populations", "r[0] = r0; r[3] = dwp * r0 / d32;", "r[0] = r0; r[3] = dwp * r0 / d21;"),
    ("adjoint_noise_amplitude", "*g_na += c[ORC_C_CK] * s->p.E_sp * xi[cc] * pn;",
     "*g_na += c[ORC_C_CK] * xi[cc] * pn;"),
    ("adjoint_layer_scale", "vh[cc][x] = layer_cb(s, a) * htot[cc][x];", "vh[cc][x] = htot[cc][x];"),
    ("tangent_inversion_term", "c[ORC_C_CK] * dN * v[cc][x];", "c[ORC_C_CK] * dN * v[cc][x] * 0.5;"),
]

# mistakes in the packing oracle, caught by its own pins
PACK_PINS = ["tests/test_oracle_pack.py"]
PACK_MUTATIONS = [
    ("pack_pair_sign", "const double q = (sig - r) / r;", "const double q = (r - sig) / r;"),
    ("pack_contact_distance", "const double sig = s * (0.5 * (d[i] + d[j]));", "const double sig = s * d[i];"),
    ("pack_unscaled_contact", "const double sig = s * (0.5 * (d[i] + d[j]));", "const double sig = 0.5 * (d[i] + d[j]);"),
    ("pack_pair_index", "const double rz = x[3 * i + 2] - x[3 * j + 2];\n            const double r2",
     "const double rz = x[3 * i + 2] - x[3 * (j + 1) % n + 2];\n            const double r2"),
    ("pack_upper_wall_sign", "if (hi > 0.0) fa[a] -= hi;", "if (hi > 0.0) fa[a] += hi;"),
    ("pack_wall_radius", "const double ri = s * (0.5 * d[i]);\n        double fa", "const double ri = s * d[i];\n        double fa"),
    ("pack_schedule_end", "const int steps = m < stages ? iters : final_iters;", "const int steps = m <= stages ? iters : final_iters;"),
    ("pack_schedule_scale", "s0 + (1.0 - s0) * (double)m / (double)stages", "s0 + (1.0 - s0) * (double)(m + 1) / (double)stages"),
    ("pack_gauss_seidel", "for (int k = 0; k < 3 * n; ++k) x[k] += eta * f[k];",
     "for (int k = 0; k < 3 * n; ++k) x[k] += eta * f[k] * (k < 3 ? 2.0 : 1.0);"),
]


CASES = [(m, SRC, PINS) for m in MUTATIONS] + [(m, PACK_SRC, PACK_PINS) for m in PACK_MUTATIONS]


@pytest.mark.parametrize("mutation,path,pins", CASES, ids=[c[0][0] for c in CASES])
def test_planted_mistake_is_caught(tmp_path, mutation, path, pins):
    name, orig, mut = mutation
    srcs = []
    for f in (SRC, PACK_SRC):
        text = open(f).read()
        if f == path:
            assert text.count(orig) == 1, f"mutation anchor for {name} not unique"
            text = text.replace(orig, mut)
        out = tmp_path / os.path.basename(f)
        out.write_text(text)
        srcs.append(str(out))
    (tmp_path / "mb_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "mb_oracle.h")).read())
    lib = tmp_path / "libbad.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                    "-o", str(lib), *srcs, "-lm"], check=True)
    env = dict(os.environ, MB_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *pins], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"
