"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of oracle/oracle.c (a flipped sign, a
dropped term, a wrong index or stride, a transposed operand), builds it, and
runs the pin suite against the copy in a subprocess: the suite must fail.
Mistakes are planted in the oracle, on the CPU, never in GPU code.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "ac_c1_sign": ("rhs[i] = (lap[i] + c1 * p) - c2 * (p * p * p);", "rhs[i] = (lap[i] - c1 * p) - c2 * (p * p * p);"),
    "ac_drop_cubic": ("rhs[i] = (lap[i] + c1 * p) - c2 * (p * p * p);", "rhs[i] = (lap[i] + c1 * p);"),
    "ch_lap_sign": ("mu[i] = (c2 * (c * c * c) - c1 * c) - lap[i];", "mu[i] = (c2 * (c * c * c) - c1 * c) + lap[i];"),
    "ch_square_not_cube": ("mu[i] = (c2 * (c * c * c) - c1 * c) - lap[i];", "mu[i] = (c2 * (c * c) - c1 * c) - lap[i];"),
    "gs_reaction_sign": ("rhs[i] = (Du * lap[i] - uvv) + F * (1.0 - u[i]);", "rhs[i] = (Du * lap[i] + uvv) + F * (1.0 - u[i]);"),
    "gs_drop_k": ("rhs[N + i] = (Dv * lapv[i] + uvv) - (F + k) * v[i];", "rhs[N + i] = (Dv * lapv[i] + uvv) - F * v[i];"),
    "gs_feed_wrong_field": ("F * (1.0 - u[i])", "F * (1.0 - v[i])"),
    "gs_v_uses_u_laplacian": ("(Dv * lapv[i] + uvv)", "(Dv * lap[i] + uvv)"),
    "lap_wrong_minus_index": ("u[site(n, x - dp[0], y - dp[1], z - dp[2])]", "u[site(n, x - dp[0], y + dp[1], z - dp[2])]"),
    "lap_dx_not_squared": ("1.0 / (dx * dx)", "1.0 / dx"),
    "lap_transposed_stride": ("wrap(x, n[0]) + n[0] * (wrap(y, n[1]) + n[1] * wrap(z, n[2]))",
                              "wrap(x, n[0]) + n[1] * (wrap(y, n[1]) + n[0] * wrap(z, n[2]))"),
    "lap_skip_last_j": ("for (int j = 1; j <= r; ++j) {\n                        int64_t dp",
                        "for (int j = 1; j < r; ++j) {\n                        int64_t dp"),
    "euler_sign": ("fields[i] = fields[i] + dt * rhs[i];", "fields[i] = fields[i] - dt * rhs[i];"),
    "energy_quartic_coeff": ("(0.25 * c2)", "(0.5 * c2)"),
    "energy_drop_gradient": ("((-0.5 * v) * lap[i] + (0.25 * c2)", "((-0.0 * v) * lap[i] + (0.25 * c2)"),
    "exact_sum_drop_error": ("if (lo != 0.0) part[k++] = lo;", "(void)lo;"),
    "mc_coupling_sign": ("- 2.0 * p * rho[i];", "+ 2.0 * p * rho[i];"),
    "mc_coupling_factor": ("- 2.0 * p * rho[i];", "- p * rho[i];"),
    "mc_drop_c3": ("g[i] = rho[i] + c3 * (phi[i] * phi[i]);", "g[i] = rho[i];"),
    "mc_phi_not_squared": ("g[i] = rho[i] + c3 * (phi[i] * phi[i]);", "g[i] = rho[i] + c3 * phi[i];"),
    "mc_rho_laplacian_of_rho_only": ("orc_laplacian(ndim, n, dx, r, w, g, rhs + N);",
                                     "orc_laplacian(ndim, n, dx, r, w, rho, rhs + N);"),
    "chd_mixed_factor": ("out[i] = out[i] + 2.0 * tt[i];", "out[i] = out[i] + tt[i];"),
    "chd_mixed_same_axis": ("orc_axis(a, n, inv_dx2, r, w, t, tt);", "orc_axis(b, n, inv_dx2, r, w, t, tt);"),
    "chd_dx_cubed": ("1.0 / (dx * dx * dx * dx)", "1.0 / (dx * dx * dx)"),
    "chd_biharmonic_sign": ("rhs[i] = rhs[i] - b[i];", "rhs[i] = rhs[i] + b[i];"),
    "chd_d4_skip_last_j": ("for (int j = 1; j <= r; ++j) {\n                    int64_t dp",
                           "for (int j = 1; j < r; ++j) {\n                    int64_t dp"),
    "chd_drop_c1": ("g[i] = c2 * (c * c * c) - c1 * c;", "g[i] = c2 * (c * c * c);"),
    "mh_div_sign": ("rhs[i] = rhs[i] - c3 * d[i];", "rhs[i] = rhs[i] + c3 * d[i];"),
    "mh_grad_sign": ("ra[i] = ra[i] + c3 * (m[i] * d[i]);", "ra[i] = ra[i] - c3 * (m[i] * d[i]);"),
    "mh_d1_direction": ("acc = acc + (w1[k] * inv_dx) * (up - um);", "acc = acc + (w1[k] * inv_dx) * (um - up);"),
    "mh_div_of_j_only": ("t[i] = m[i] * ja[i];", "t[i] = ja[i];"),
    "mh_grad_of_m_not_mu": ("orc_d1(a, n, dx, r, w1, mu, d);", "orc_d1(a, n, dx, r, w1, m, d);"),
    "mh_j_laplacian_of_m": ("orc_laplacian(ndim, n, dx, r, w, ja, ra);", "orc_laplacian(ndim, n, dx, r, w, m, ra);"),
    "chd_mixed_includes_diagonal": ("for (int b = a + 1; b < ndim; ++b) {", "for (int b = a; b < ndim; ++b) {"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor not found: " + name
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared", "-o",
                    str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, PF_ORACLE_MUTANT_LIB=str(lib), OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, "pin suite passed with planted mistake " + name


SPECTRAL = os.path.join(ROOT, "oracle", "spectral.py")
SPECTRAL_MUTANTS = {
    "sp_ac_sign": ("uh = (uh + dt * nh) / (1.0 + dt * K2)", "uh = (uh - dt * nh) / (1.0 + dt * K2)"),
    "sp_ch_k2_not_k4": ("(1.0 + dt * K2 * K2)", "(1.0 + dt * K2)"),
    "sp_ch_drop_k2": ("uh = (uh - dt * K2 * nh)", "uh = (uh - dt * nh)"),
    "sp_k_without_2pi": ("kx = 2 * np.pi * np.fft.rfftfreq(nx, d=dx)", "kx = np.fft.rfftfreq(nx, d=dx)"),
    "sp_drop_ky": ("K2 += ky[None, :, None] ** 2", "K2 += 0.0 * ky[None, :, None] ** 2"),
    "sp_ch_c1_sign": ("return c2 * (u * u * u) - c1 * u", "return c2 * (u * u * u) + c1 * u"),
    "sp_dx_ignored_in_y": ("np.fft.fftfreq(ny, d=dx)", "np.fft.fftfreq(ny, d=1.0)"),
    "sp_dt_max_ch": ("else 2.0 / (c1 * c1)", "else 4.0 / (c1 * c1)"),
    "sp_dt_max_ac": ("return 1.0 / c1 if kind == AC", "return 2.0 / c1 if kind == AC"),
}


@pytest.mark.parametrize("name", sorted(SPECTRAL_MUTANTS))
def test_spectral_pins_catch_planted_mistake(name, tmp_path):
    old, new = SPECTRAL_MUTANTS[name]
    src = open(SPECTRAL).read()
    assert src.count(old) >= 1, "mutation anchor not found: " + name
    mut = tmp_path / "spectral_mutant.py"
    mut.write_text(src.replace(old, new))
    env = dict(os.environ, PF_ORACLE_SPECTRAL_MUTANT=str(mut), OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_spectral.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, "spectral pins passed with planted mistake " + name


STABILITY = os.path.join(ROOT, "oracle", "stability.py")
STABILITY_MUTANTS = {
    "dtmax_gs_min_for_max": ("rho = max(params[0], params[1]) * lam", "rho = min(params[0], params[1]) * lam"),
    "dtmax_gs_drop_lam": ("rho = max(params[0], params[1]) * lam", "rho = max(params[0], params[1])"),
    "dtmax_gs_drop_one": ("+ params[2] + params[3] + 1.0", "+ params[2] + params[3]"),
    "dtmax_gs_lam_squared": ("rho = max(params[0], params[1]) * lam", "rho = max(params[0], params[1]) * lam * lam"),
    "dtmax_ac_drop_c1": ("rho = lam + 2 * abs(params[0])", "rho = lam"),
    "dtmax_ac_c1_factor": ("rho = lam + 2 * abs(params[0])", "rho = lam + abs(params[0])"),
    "dtmax_ch_drop_c1": ("        rho = lam * lam + 2 * abs(params[0]) * lam\n    else:",
                         "        rho = lam * lam\n    else:"),
    "dtmax_ch_c1_factor": ("        rho = lam * lam + 2 * abs(params[0]) * lam\n    else:",
                           "        rho = lam * lam + abs(params[0]) * lam\n    else:"),
    "dtmax_ch_c1_without_lam": ("        rho = lam * lam + 2 * abs(params[0]) * lam\n    else:",
                                "        rho = lam * lam + 2 * abs(params[0])\n    else:"),
    "dtmax_mh_min_for_max": ("rho = max(lam * lam + 2 * abs(params[0]) * lam, lam)",
                             "rho = min(lam * lam + 2 * abs(params[0]) * lam, lam)"),
    "dtmax_mh_drop_c1": ("rho = max(lam * lam + 2 * abs(params[0]) * lam, lam)", "rho = max(lam * lam, lam)"),
    "dtmax_mh_drop_diffusion": ("rho = max(lam * lam + 2 * abs(params[0]) * lam, lam)",
                                "rho = lam * lam + 2 * abs(params[0]) * lam"),
    "dtmax_mc_as_ch": ("    elif kind in (AC, MC):", "    elif kind == AC:"),
    "dtmax_ndim_ignored": ("lam = abs(float(sigma)) * ndim / (dx * dx)", "lam = abs(float(sigma)) / (dx * dx)"),
    "dtmax_dx_not_squared": ("lam = abs(float(sigma)) * ndim / (dx * dx)", "lam = abs(float(sigma)) * ndim / dx"),
}


@pytest.mark.parametrize("name", sorted(STABILITY_MUTANTS))
def test_stability_pins_catch_planted_mistake(name, tmp_path):
    """Mistakes planted in the explicit-stability limit (oracle/stability.py)
    fail the dt_max pins of tests/test_oracle_pins.py."""
    old, new = STABILITY_MUTANTS[name]
    src = open(STABILITY).read()
    assert src.count(old) == 1, "mutation anchor not found once: " + name
    mut = tmp_path / "stability_mutant.py"
    mut.write_text(src.replace(old, new))
    env = dict(os.environ, PF_ORACLE_STABILITY_MUTANT=str(mut), OMP_NUM_THREADS="1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          "-k", "dt_max or unstable", os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, "stability pins passed with planted mistake " + name
