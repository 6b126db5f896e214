"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (a reading
of the paper flipped, a sign or an index changed), builds it with gcc in a
temporary folder, and runs the pins in a child process against that build
(``STEV_ORACLE_LIB``); the Python Levenberg-Marquardt oracle is mutated in a
copy of ``oracle/`` and ``tests/`` in a temporary folder.  The case passes
when at least one of the named pins fails.  Nothing here touches the
committed oracle or any GPU code.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "stev_oracle.c")

# (name, exact text in stev_oracle.c, replacement, pins expected to catch it)
MUTATIONS = [
    # Eq 8: the ring stores the damped rate rOF q h instead of the undamped q h
    ("ring_stores_damped_rate",
     "ring[j * W + (int)((it - 1) % W)] = q[j] * h;",
     "ring[j * W + (int)((it - 1) % W)] = rOF[j] * q[j] * h;",
     "damped_trajectory"),
    # Eqs 15-16: the low set taken from T_mid up
    ("range_select_swapped",
     "(T < m->T_mid[k]) ? &m->nasa_lo[7 * k] : &m->nasa_hi[7 * k]",
     "(T >= m->T_mid[k]) ? &m->nasa_lo[7 * k] : &m->nasa_hi[7 * k]",
     "range_select or thermo"),
    # Eq 10: the high band widened down to bin 3
    ("band_from_bin_3",
     "int k_lo = (W + 3) / 4, k_hi = W / 2;",
     "int k_lo = 3, k_hi = W / 2;",
     "high_band"),
    # Eq 30: (RT / 1 atm)^dN in place of (1 atm / RT)^dN
    ("delta_n_inverted",
     "double K = pow(ORC_PATM / (ORC_R * T), dN) * exp(-dG_RT);\n      double kr = kf / K;\n      double prod_r",
     "double K = pow((ORC_R * T) / ORC_PATM, dN) * exp(-dG_RT);\n      double kr = kf / K;\n      double prod_r",
     "t10_two or t8"),
    # Eq 2: the 90 % rule applied below 1e-20 and the unit value above
    ("eq2_branches_swapped",
     "double ystar = (Y[k] < 1.0e-20) ? 1.0 : 0.9 * Y[k];",
     "double ystar = (Y[k] < 1.0e-20) ? 0.9 * Y[k] : 1.0;",
     "t3"),
    # Eq 13: no cap at 1
    ("rof_uncapped",
     "double r = fmin(rof * rof_star, 1.0);",
     "double r = rof * rof_star;",
     "t7 or damped_trajectory"),
    # Eq 12: rOF update before the ring is full
    ("rof_before_full_ring",
     "if (it >= W) {",
     "if (it >= 1) {",
     "t7 or damped_trajectory"),
    # Sec 3: the sigmoid's exponent with the wrong sign
    ("ann_sigmoid_sign",
     "a[u] = 1.0 / (1.0 + exp(-(w1[u] * x[i] + b1[u])));",
     "a[u] = 1.0 / (1.0 + exp(w1[u] * x[i] + b1[u]));",
     "ann_forward"),
    # Sec 3: the output weights read column-major
    ("ann_output_transposed",
     "v += W2[(size_t)o * H + u] * a[u];",
     "v += W2[(size_t)u * n_out + o] * a[u];",
     "ann_forward"),
    # Sec 3: h/R from the network not divided by T
    ("ann_h_not_over_T",
     "h_RT[k] = y[n_s + k] / T;",
     "h_RT[k] = y[n_s + k];",
     "ann_thermo_mode"),
    # Eq 1: every species' rate of change limits the step, not only consumption
    ("eq1_any_sign",
     "double rstar = fmax(-dYdt[k], 1.0e-30);",
     "double rstar = fmax(fabs(dYdt[k]), 1.0e-30);",
     "t3 or t1 or t8"),
    # Eq 4: no cap at delta_max of the flow step
    ("eq4_cap_dropped",
     "double h = fmin(tstar, dtmax);",
     "double h = tstar;",
     "t4 or t1"),
    # Eq 5 without the clamp to the end of the flow step
    ("no_end_clamp",
     "return fmin(h, tf - t);",
     "return h;",
     "last_step"),
    # Eq 13 without its lower bound on rOF
    ("rof_floor_dropped",
     "return fmax(r, p->rof_min);",
     "return r;",
     "t7_rof_sequences"),
    # the energy equation with the wrong sign
    ("energy_sign",
     "*dTdt = -T * sum_hw / (rho * cpmix_R);",
     "*dTdt = T * sum_hw / (rho * cpmix_R);",
     "energy_equation"),
    # Eqs 6-7: gamma left out of the rate-law concentrations
    ("gamma_dropped_from_rates",
     "C[k] = rho * orc_ystarstar(Y[k], p->alpha) / m->W[k];\n  }\n  if (m->mlp_prm",
     "C[k] = rho * Y[k] / m->W[k];\n  }\n  if (m->mlp_prm",
     "t9 or t11"),
    # cm-mol-s to SI: one power of 1e-6 too many
    ("arrhenius_units",
     "double A_SI = m->A[j] * pow(1e-6, m_f - 1.0);\n    double kf = A_SI * pow(T, m->b[j]) * exp(-m->Ea[j] / (ORC_R * T));\n    double prod_f",
     "double A_SI = m->A[j] * pow(1e-6, m_f);\n    double kf = A_SI * pow(T, m->b[j]) * exp(-m->Ea[j] / (ORC_R * T));\n    double prod_f",
     "unit_conversion or t1"),
    # Eq 16: h/RT with a3 T^2 / 2 in place of a3 T^2 / 3
    ("enthalpy_coefficient",
     "a[2] * T2 / 3.0 + a[3] * T3 / 4.0 +\n           a[4] * T4 / 5.0 + a[5] / T;",
     "a[2] * T2 / 2.0 + a[3] * T3 / 4.0 +\n           a[4] * T4 / 5.0 + a[5] / T;",
     "thermo_identities"),
    # s/R without the a7 constant (the reverse rates' K then loses it)
    ("entropy_constant_dropped",
     "a[4] * T4 / 4.0 + a[6];",
     "a[4] * T4 / 4.0;",
     "t8 or thermo_identities"),
    # Eq 25: d(C^o)/dY without the gamma factor's (Y + 2 alpha) / (alpha + Y)
    ("jacobian_gamma_factor_dropped",
     "return pow(rho / W, o) * o * pow(Y, 2.0 * o - 1.0) * (Y + 2.0 * alpha) *\n         pow(alpha + Y, -(1.0 + o));",
     "return pow(rho / W, o) * o * pow(Y, 2.0 * o - 1.0) * pow(alpha + Y, -o);",
     "jacobian"),
    # Sec 3 network training: tanh' taken as 1 - a instead of 1 - a^2
    ("mlp_tanh_derivative",
     "d2[v] = s * (1.0 - a2[v] * a2[v]);",
     "d2[v] = s * (1.0 - a2[v]);",
     "mlp_gradient"),
    # back-propagation through the transposed hidden weights
    ("mlp_backward_transposed",
     "for (int u = 0; u < H; ++u) s += W2[u * H + v] * d2[u];",
     "for (int u = 0; u < H; ++u) s += W2[v * H + u] * d2[u];",
     "mlp_gradient"),
    # Adam without the first-moment bias correction
    ("adam_no_bias_correction",
     "double mhat = m1[i] / c1;",
     "double mhat = m1[i];",
     "adam"),
    # Eq 25: the reverse rate's derivative with the wrong sign
    ("jacobian_reverse_sign",
     "double dq = forward ? kf * d : -kr * d;",
     "double dq = forward ? kf * d : kr * d;",
     "jacobian or eq25"),
    # Eq 25: the Jacobian of the undamped rates (rOF ignored)
    ("jacobian_ignores_damping",
     "double damp = m->rev[j] ? rOF[j] : 1.0;\n    /* d q_eff",
     "double damp = 1.0;\n    /* d q_eff",
     "jacobian or eq25"),
    # Eq 25: the column sum norm in place of the row sum norm
    ("jacobian_one_norm",
     "for (int c = 0; c < n_s; ++c) row += fabs(A[(size_t)i * n_s + c]);",
     "for (int c = 0; c < n_s; ++c) row += fabs(A[(size_t)c * n_s + i]);",
     "jacobian or eq25"),
    # Eq 25: W of the differentiated species in place of the row species
    ("jacobian_wrong_molar_mass",
     "A[(size_t)ki * n_s + kc] += m->W[ki] / rho * m->nu[i] * damp * dq;",
     "A[(size_t)ki * n_s + kc] += m->W[kc] / rho * m->nu[i] * damp * dq;",
     "jacobian or eq25"),
]


SRC_C3M = os.path.join(ROOT, "oracle", "c3m_oracle.c")

# the same for the multiphase oracle, caught by tests/test_oracle_c3m.py
C3M_MUTATIONS = [
    # Eq 42 evaluated at the gas temperature
    ("pyro_at_gas_temperature",
     "exp(-c->Ea_pyro / T_s);",
     "exp(-c->Ea_pyro / T_g);",
     "arrhenius and PYRO"),
    # Eq 46: theta_1 on phi instead of vartheta
    ("anneal_theta1_on_phi",
     "g[1] * th + g[0];",
     "g[1] * phi + g[0];",
     "anneal"),
    # Eq 54 without its gamma(X_H2)
    ("hox_gamma_dropped",
     "pos(X_g[G_H2]) * gam(X_g[G_O2], a) * gam(X_g[G_H2], a);",
     "pos(X_g[G_H2]) * gam(X_g[G_O2], a);",
     "gamma_factor_of_gas"),
    # Eq 51: film temperature weighted to the gas
    ("film_temperature_skewed",
     "const double T_film = 0.5 * T_g + 0.5 * T_s;",
     "const double T_film = 0.75 * T_g + 0.25 * T_s;",
     "arrhenius and COX"),
    # Eqs 1-3 over the gas fractions only
    ("step_rule_gas_only",
     "double h = orc_step_size(p, NX, X, dX, t, tf);",
     "double h = orc_step_size(p, NG, X, dX, t, tf);",
     "step_rule"),
    # Eq 38: half the oxygen of CO oxidation dropped
    ("coox_oxygen_dropped",
     "nu[R_COOX][G_O2] = -0.5;",
     "nu[R_COOX][G_O2] = -1.0;",
     "conserved"),
    # Eq 14 damping applied to a reaction that has no ring
    ("damping_on_hox",
     "double r_eff = (j == R_WGS) ? rof * r[j] : r[j];",
     "double r_eff = (j == R_WGS || j == R_HOX) ? rof * r[j] : r[j];",
     "damping_applies"),
    # Eq 43: the forward and reverse WGS constants swapped
    ("wgs_constants_swapped",
     "(c->Kf_wgs * pos(X_g[G_CO])",
     "(c->Kr_wgs * pos(X_g[G_CO])",
     "wgs_closed_form"),
    # Eq 47: the H2 inhibition term added instead of dividing
    ("stg_inhibition_sign",
     "(1.0 + c->Fp_stg * (MW_g",
     "(1.0 - c->Fp_stg * (MW_g",
     "pressure_orders"),
    # Eq 50: the O2 partial-pressure order 0.5 instead of 0.73
    ("cox_order",
     "pos(X_g[G_O2]) / 31.9988, 0.73)",
     "pos(X_g[G_O2]) / 31.9988, 0.5)",
     "pressure_orders"),
    # Eq 55: the gas density to the power of the O2 order
    ("meox_density_power",
     "ep_g * pow(rho_g, 1.5) *\n              pow(pos(X_g[G_O2]), 1.3)",
     "ep_g * pow(rho_g, 1.3) *\n              pow(pos(X_g[G_O2]), 1.3)",
     "gas_density_orders"),
    # Eq 8 on WGS: the ring stores the damped rate rOF r h
    ("c3m_ring_stores_damped_rate",
     "ring[(int)((it - 1) % W)] = r[R_WGS] * h;",
     "ring[(int)((it - 1) % W)] = rof * r[R_WGS] * h;",
     "wgs_damped_trajectory"),
    # Eq 12 on WGS: rOF updated before the ring holds 13 samples
    ("c3m_rof_before_full_ring",
     "      if (it >= W) {\n        orc_dft_mag(ring, W, D);",
     "      if (it >= 1) {\n        orc_dft_mag(ring, W, D);",
     "wgs_ring_damping_sequence or wgs_damped_trajectory"),
    # solids volume fraction taken as the bulk density
    ("eps_s_not_divided",
     "const double ep_s = ROP_s / rho_s;\n  const double ep_g",
     "const double ep_s = ROP_s;\n  const double ep_g",
     "solid_geometry"),
]


def _build(src_text, out_dir, c3m_text=None):
    c = os.path.join(out_dir, "stev_oracle.c")
    with open(c, "w") as f:
        f.write(src_text)
    if c3m_text is not None:
        with open(os.path.join(out_dir, "c3m_oracle.c"), "w") as f:
            f.write(c3m_text)
    shutil.copy(os.path.join(ROOT, "oracle", "stev_oracle.h"), out_dir)
    c3m = os.path.join(out_dir, "c3m_oracle.c")
    if not os.path.exists(c3m):
        shutil.copy(os.path.join(ROOT, "oracle", "c3m_oracle.c"), out_dir)
    lib = os.path.join(out_dir, "liboracle_mut.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-fPIC", "-shared", "-o", lib, c, c3m, "-lm"])
    return lib


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, pins):
    with open(SRC) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation site for {name} not unique/found"
    lib = _build(text.replace(old, new), str(tmp_path))
    env = dict(os.environ, STEV_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and "failed" in r.stdout, (
        f"pins '{pins}' did not catch {name}:\n{r.stdout[-2000:]}")


@pytest.mark.parametrize("name,old,new,pins", C3M_MUTATIONS, ids=[m[0] for m in C3M_MUTATIONS])
def test_c3m_pins_catch_planted_mistake(tmp_path, name, old, new, pins):
    with open(SRC_C3M) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation site for {name} not unique/found"
    with open(SRC) as f:
        base = f.read()
    lib = _build(base, str(tmp_path), text.replace(old, new))
    env = dict(os.environ, STEV_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_c3m.py"), "-k", pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and "failed" in r.stdout, (
        f"pins '{pins}' did not catch {name}:\n{r.stdout[-2000:]}")


SRC_LMA = os.path.join(ROOT, "oracle", "ann_lma.py")

# the same for the Levenberg-Marquardt oracle of the paper's network (Python):
# the mutated module runs from a copy of oracle/ and tests/ in a temporary
# folder, caught by tests/test_oracle_lma.py
LMA_MUTATIONS = [
    # the sigmoid's derivative taken as a instead of a (1 - a)
    ("lma_sigmoid_derivative",
     "ds = a * (1.0 - a)",
     "ds = a",
     "central_differences"),
    # the residual with the wrong sign (J^T r then points uphill)
    ("lma_residual_sign",
     "r = forward(prm, H, n_out, xs) - target[s0:s0 + chunk]",
     "r = target[s0:s0 + chunk] - forward(prm, H, n_out, xs)",
     "least_squares_step"),
    # Levenberg's identity in place of the scaled diagonal
    ("lma_damping_identity",
     "return dg + mu * np.mean(dg)",
     "return np.ones_like(dg)",
     "damping"),
    # lambda raised after an accepted step as well as after a rejected one
    ("lma_lambda_never_lowered",
     "lam /= down",
     "lam *= down",
     "fits_a_known"),
]


@pytest.mark.parametrize("name,old,new,pins", LMA_MUTATIONS, ids=[m[0] for m in LMA_MUTATIONS])
def test_lma_pins_catch_planted_mistake(tmp_path, name, old, new, pins):
    with open(SRC_LMA) as f:
        text = f.read()
    assert text.count(old) == 1, f"mutation site for {name} not unique/found"
    skip = shutil.ignore_patterns("__pycache__", "*.so", "*.tmp")
    shutil.copytree(os.path.join(ROOT, "oracle"), str(tmp_path / "oracle"), ignore=skip)
    shutil.copytree(os.path.join(ROOT, "tests"), str(tmp_path / "tests"), ignore=skip)
    (tmp_path / "oracle" / "ann_lma.py").write_text(text.replace(old, new))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        str(tmp_path / "tests" / "test_oracle_lma.py"), "-k", pins],
                       cwd=str(tmp_path), capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and "failed" in r.stdout, (
        f"pins '{pins}' did not catch {name}:\n{r.stdout[-2000:]}")
