"""The pins catch plausible mistakes in the oracle.

Each mutant below plants one mistake (a flipped sign, a wrong index or range, a dropped
factor, a swapped operand) into a copy of the oracle source, on the CPU.  The copy is
compiled and the fast pins are run against it; every mutant must fail at least one pin.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_kw as KW
import test_oracle_multid as MD
import test_oracle_muscl3 as M3
import test_oracle_pins as P
import test_oracle_step_cells as SC
import test_oracle_tau_field as TF
import test_oracle_tauhat as TH
import test_oracle_weno5 as W5

SRC = oracle.SRC

MUTANTS = {
    "half-line tail sign": ("M->u[R_POS][1] = U * M->u[R_POS][0] + tail;",
                            "M->u[R_POS][1] = U * M->u[R_POS][0] - tail;"),
    "moment recurrence factor": ("M->u[r][n + 1] = U * M->u[r][n] + n * h * M->u[r][n - 1];",
                                 "M->u[r][n + 1] = U * M->u[r][n] + (n + 1) * h * M->u[r][n - 1];"),
    "internal xi^4 moment": ("M->xi[2] = gas->K * (gas->K + 2.0) * h * h;", "M->xi[2] = gas->K * gas->K * h * h;"),
    "interface state half lines swapped": (
        "W0[m] = gl.rho * p_expect(&pm, &Ml, R_POS) + gr.rho * p_expect(&pm, &Mr, R_NEG);",
        "W0[m] = gl.rho * p_expect(&pm, &Ml, R_NEG) + gr.rho * p_expect(&pm, &Mr, R_POS);"),
    "compatibility sign": ("        r[m] = -p_expect(&prod, &Ml, R_ALL);\n        for (int t = 0; t < ntan; ++t) r[m] -= og_tan_moment(dim, b_l",
                           "        r[m] = p_expect(&prod, &Ml, R_ALL);\n        for (int t = 0; t < ntan; ++t) r[m] -= og_tan_moment(dim, b_l"),
    "time weight gam1": ("g1 = 2.0 * s - x * (1.0 + E);", "g1 = 2.0 * s - x * (1.0 - E);"),
    "time weight c5 sign": ("k->c5 = -s / g0;", "k->c5 = s / g0;"),
    "turbulent tau without strain": ("tau += (kf / wf) / ((p0 / rho0) * sqrt(1.0 + eta * eta));",
                                     "tau += (kf / wf) / ((p0 / rho0) * sqrt(1.0 + eta));"),
    "Prandtl factor": ("F[nv - 1] += (1.0 / gas->prandtl - 1.0) * q;", "F[nv - 1] += (gas->prandtl - 1.0) * q;"),
    "heat flux frame": ("p_term(&lin1, -g0.U[0], 0, 0, 0, 0);", "p_term(&lin1, g0.U[0], 0, 0, 0, 0);"),
    "minmod picks the larger": ("return (p > 0.0 ? 1.0 : -1.0) * fmin(fabs(p), fabs(q));",
                                "return (p > 0.0 ? 1.0 : -1.0) * fmax(fabs(p), fabs(q));"),
    "equilibrium slope distance": ("r[m] = (W0[m] - Wi[m]) / (g0.rho * dxl);", "r[m] = (W0[m] - Wi[m]) / (g0.rho * dxr);"),
    "Abar time weight": ("ADD_TERM(g0.rho * kw.g[2], 0, R_ALL, p_lin(dim, Ab, &terms[nt].poly));",
                         "ADD_TERM(g0.rho * kw.g[1], 0, R_ALL, p_lin(dim, Ab, &terms[nt].poly));"),
    "wall mirrors normal momentum only": ("if (bc == OG_WALL && m >= 1 && m <= dim) v = -v;",
                                          "if (bc == OG_WALL && m == 1) v = -v;"),
    "update sign": ("Wn[m * N + s] = W[m * N + s] - og_flux_out(gr, F, fn, m, idx);",
                    "Wn[m * N + s] = W[m * N + s] + og_flux_out(gr, F, fn, m, idx);"),
    "flux difference faces swapped": ("acc += (F[d][m * nf + hi] - F[d][m * nf + lo])",
                                      "acc += (F[d][m * nf + lo] - F[d][m * nf + hi])"),
    "strain not symmetrised": ("double sab = 0.5 * (grad[a][b] + grad[b][a]);", "double sab = grad[a][b];"),
    "viscous CFL term": ("r += 2.0 * nu * r2;", "r += nu * r2;"),
    "periodic ghost face coordinates": ("gr->xfe[d][2 - m] = xf[0] - (xf[n] - xf[n - m]);",
                                        "gr->xfe[d][2 - m] = xf[0] - (xf[m] - xf[0]);"),
    "k-omega convection downwind": ("*Fk = Frho * (Frho >= 0.0 ? kl : kr)", "*Fk = Frho * (Frho >= 0.0 ? kr : kl)"),
    "k-omega diffusion sign": ("*Fk = Frho * (Frho >= 0.0 ? kl : kr) - dt", "*Fk = Frho * (Frho >= 0.0 ? kl : kr) + dt"),
    "omega diffusion coefficient": ("(mu + KW_SIGMA * nut) * (wr - wl)", "(mu + KW_SIGMA_STAR * nut) * (wr - wl)"),
    "eddy diffusivity from one side": ("const double nut = 0.5 * (rl * kl / wl + rr * kr / wr);",
                                       "const double nut = rl * kl / wl;"),
    "k sink coefficient": ("rkn[s] = (ak + dt * Qk) / (1.0 + dt * KW_BETA_STAR * om[s]);",
                           "rkn[s] = (ak + dt * Qk) / (1.0 + dt * KW_BETA * om[s]);"),
    "k flux difference sign": ("double ak = rk[s] - og_flux_out(gr, Fk, fn, 0, idx);",
                               "double ak = rk[s] + og_flux_out(gr, Fk, fn, 0, idx);"),
    "eddy viscosity without strain limiter": ("const double mut = rho * kc / (wc * root);",
                                              "const double mut = rho * kc / wc;"),
    "omega production without limiter": ("*Qw = KW_ALPHA * rho * (shear / root", "*Qw = KW_ALPHA * rho * (shear"),
    "cross diffusion regardless of sign": ("if (cross > 0.0) *Qw +=", "if (cross != 0.0) *Qw +="),
    "material derivative sign": ("drho = g0.U[0] * grho - gmom;", "drho = g0.U[0] * grho + gmom;"),
    "tau_hat from the cell density": ("const double eps_hat = tau * fabs(drho) / g0.rho;",
                                      "const double eps_hat = tau * fabs(drho) / Wi[0];"),
    "decay time inverted": ("og_time_weights(tau, dt * eps_hat, dt, &kw)", "og_time_weights(tau, dt / eps_hat, dt, &kw)"),
    "slope term of gam1": ("k->g[1] = -tau * gam0 + I1;", "k->g[1] = -tau * gam0 - I1;"),
    "slope term of gam4": ("k->g[4] = -tau * I0 - I1;", "k->g[4] = -tau * I0 + I1;"),
    "series of t e^{-t/tau_e}": ("h -= sg * (n - 1) * term;", "h -= sg * n * term;"),
    "hydrodynamic limit keeps the upwind part": ("I0 = 0.0; I1 = 0.0; gam0 = dt;", "I0 = dt; I1 = 0.0; gam0 = 0.0;"),
    "kappa-scheme weights swapped": ("return 0.5 * (1.0 - kappa) * og_minmod(away, b * toward) + 0.5 * (1.0 + kappa) * og_minmod(toward, b * away);",
                                     "return 0.5 * (1.0 + kappa) * og_minmod(away, b * toward) + 0.5 * (1.0 - kappa) * og_minmod(toward, b * away);"),
    "kappa-scheme limiter bound": ("b = (3.0 - kappa) / (1.0 - kappa);", "b = (1.0 + kappa) / (1.0 - kappa);"),
    "third-order right face value from the wrong cell": ("*wr = w[2] - og_muscl3(d2, d1) * (xc[2] - xf);",
                                                          "*wr = w[2] - og_muscl3(d1, d2) * (xc[2] - xf);"),
    "interface tangential slope from one side": ("r[m] = 0.5 * (tsl[t * 5 + m] + tsr[t * 5 + m]) / g0.rho;",
                                                 "r[m] = tsl[t * 5 + m] / g0.rho;"),
    "tangential terms of A with the wrong sign": ("r[m] -= og_tan_moment(dim, b_l[t], t, m, &Ml, R_ALL, 0);",
                                                  "r[m] += og_tan_moment(dim, b_l[t], t, m, &Ml, R_ALL, 0);"),
    "tangential Abar term dropped": ("x1 += og_tan_moment(dim, b_0[t], t, m, &M0, R_ALL, 0);",
                                     "x1 += 0.0 * og_tan_moment(dim, b_0[t], t, m, &M0, R_ALL, 0);"),
    "tangential flux term on the normal velocity": (
        "ADD_TERM(g0.rho * kw.g[1], 0, R_ALL, (p_lin(dim, b_0[t], &terms[nt].poly), p_tpow(&terms[nt].poly, t)));",
        "ADD_TERM(g0.rho * kw.g[1], 0, R_ALL, (p_lin(dim, b_0[t], &terms[nt].poly), p_upow(&terms[nt].poly, 1)));"),
    "one-sided tangential slope": ("out[(t - 1) * 5 + m] = og_minmod(dm, dp);", "out[(t - 1) * 5 + m] = dp;"),
    "WENO candidate coefficient": ("const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;",
                                   "const double q0 = (2.0 * a - 7.0 * b + 10.0 * c) / 6.0;"),
    "WENO linear weight": ("const double al0 = 0.1 / ((eps + beta0) * (eps + beta0));",
                           "const double al0 = 0.3 / ((eps + beta0) * (eps + beta0));"),
    "WENO smoothness coefficient": ("const double beta1 = 13.0 / 12.0 * s1 * s1 + 0.25 * t1 * t1;",
                                    "const double beta1 = 13.0 / 12.0 * s1 * s1 + 0.5 * t1 * t1;"),
    "WENO weight exponent": ("const double al2 = 0.3 / ((eps + beta2) * (eps + beta2));",
                             "const double al2 = 0.3 / (eps + beta2);"),
    "WENO epsilon": ("const double eps = 1e-6;", "const double eps = 1e-40;"),
    "WENO right value not mirrored": ("*wr = og_weno5(w[4], w[3], w[2], w[1], w[0]);",
                                      "*wr = og_weno5(w[-1], w[0], w[1], w[2], w[3]);"),
    "sampled-cell flux difference sign": ("acc[m] -= (Fhi[m] - Flo[m]) / gr.dx[d][idx[d] + 2];",
                                          "acc[m] -= (Flo[m] - Fhi[m]) / gr.dx[d][idx[d] + 2];"),
    "tau field reports the rarefaction": ("        diag_out[1] = info[40];", "        diag_out[1] = info[50];"),
    "sampled-cell width of the wrong cell": ("acc[m] -= (Fhi[m] - Flo[m]) / gr.dx[d][idx[d] + 2];",
                                             "acc[m] -= (Fhi[m] - Flo[m]) / gr.dx[d][idx[d] + 3];"),
}


def _sod_quick():
    import exact_riemann as ER
    from inputs import cases as C
    case = C.sod_tube(100, ny=2, t_end=0.2)
    r = oracle.run(case, 100000, nthreads=4)
    x = 0.5 * (case.xf[0][1:] + case.xf[0][:-1])
    ex = ER.sample((1, 0, 1), (0.125, 0, 0.1), x, 0.2)
    assert float(np.mean(np.abs(r["W"][0, 0, 0] - ex[0]))) < 0.02


PINS = [
    lambda: P.test_p1_moments_vs_mpmath(0.7, 0.35),
    lambda: P.test_kogan_weights_vs_time_quadrature(1.7),
    lambda: P.test_kogan_weights_vs_time_quadrature(0.1),
    lambda: P.test_p2_moment_solve(2),
    lambda: P.test_p5_continuous_data_navier_stokes(2),
    lambda: P.test_p5_prandtl_correction_heat_flux(2),
    lambda: P.test_p6_euler_limit(2),
    lambda: P.test_p7_collisionless_limit_kfvs(2),
    lambda: P.test_p8_symmetries(2),
    lambda: P.test_p11_turbulent_tau(),
    lambda: P.test_ghost_fill_rules(),
    lambda: P.test_cfl_dt_uniform(),
    lambda: P.test_strain_rate_linear_field(),
    lambda: P.test_p4_free_stream(2, None),
    lambda: P.test_p10_conservation_periodic(),
    lambda: P.test_p9_periodic_seam_invariance(),
    lambda: P.test_coefficient_definitions_by_quadrature(2),
    lambda: P.test_p16_flux_bruteforce(2, 1.0),
    _sod_quick,
    lambda: KW.test_homogeneous_decay_follows_the_point_implicit_recurrence(2),
    lambda: KW.test_uniform_k_stays_uniform_in_a_density_wave(),
    lambda: KW.test_rho_k_and_rho_omega_conserved_up_to_their_sources("mixing"),
    lambda: KW.test_convection_is_upwind(),
    lambda: KW.test_production_of_a_linear_shear(),
    lambda: KW.test_cross_diffusion_only_where_gradients_align(-1.0),
    lambda: KW.test_cross_diffusion_only_where_gradients_align(1.0),
    lambda: KW.test_diffusion_rate_of_a_sine_mode("k"),
    lambda: KW.test_diffusion_rate_of_a_sine_mode("omega"),
    lambda: KW.test_mirror_symmetry(),
    lambda: [TH.test_time_weights_by_quadrature(x, r) for x in (0.3, 2.0) for r in (0.1, 7.0)],
    lambda: TH.test_hydrodynamic_limit(),
    lambda: TH.test_eps_hat_of_a_velocity_gradient(2),
    lambda: TH.test_eps_hat_of_density_and_velocity_gradients(),
    lambda: TH.test_continuous_data_navier_stokes_flux_in_tauhat_mode(2),
    lambda: [M3.test_quadratic_face_values_are_exact_on_a_uniform_grid(s) for s in range(3)],
    lambda: M3.test_no_new_extrema_on_a_uniform_grid(),
    lambda: M3.test_quadratic_with_slopes_three_times_apart(),
    lambda: MD.test_continuous_data_full_navier_stokes_flux(2),
    lambda: MD.test_continuous_data_full_navier_stokes_flux(3),
    lambda: MD.test_transposed_data_give_the_transposed_solution(),
    lambda: MD.test_mirror_in_the_tangential_direction(),
    lambda: MD.test_free_stream_and_conservation_with_the_expansion(),
    lambda: W5.test_quadratics_are_exact(0),
    lambda: W5.test_closed_forms_match_the_definition(1.0),
    lambda: W5.test_epsilon_matters_for_nearly_linear_data(),
    lambda: W5.test_mirror_and_minmod_gradients(),
    lambda: SC.step_cells_matches_run("2d_mixed_bc"),
    lambda: SC.step_cells_matches_run("3d_mixed_bc"),
    lambda: TF.test_tau_field_of_a_uniform_flow(2),
]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutation site not unique or missing: {name}"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-o", str(so), str(src), "-lm"])
    oracle.use_library(str(so))
    caught = None
    try:
        for i, pin in enumerate(PINS):
            try:
                pin()
            except (AssertionError, oracle.OracleError, FloatingPointError, ValueError):
                caught = i
                break
    finally:
        oracle.use_library(None)
    assert caught is not None, f"no pin caught the planted mistake: {name}"
