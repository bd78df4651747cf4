"""The oracle's pins must catch plausible mistakes.

Each mutant below plants one typical error (a dropped term, a flipped sign, a
wrong neighbour, an x/y mix-up, a wrong donor) into a temporary copy of the
oracle's C source, compiles it on the CPU, and runs the pin suite
(test_oracle_pins.py, test_oracle_variants.py, test_oracle_forcing.py) against
it in a subprocess.  Every mutant must make at
least one pin fail; the unmodified source must pass.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "csph_oracle.c")

MUTANTS = {
    "w_drops_sqrt2": ("return sqrt(2.0) * H / sqrt(", "return H / sqrt("),
    "minmod_is_maxmod": ("if (a > 0.0) return a < b ? a : b;", "if (a > 0.0) return a > b ? a : b;"),
    "hll_diffusion_sign": ("+ SL * SR * (UR[k] - UL[k])", "- SL * SR * (UR[k] - UL[k])"),
    "hll_davis_speed": ("fmin(unL - cL, unR - cR)", "fmin(unL - cL, unR + cR)"),
    "pressure_sign_x": ("Sx[c] = -(Pe - Pw) / dx", "Sx[c] = (Pe - Pw) / dx"),
    "bed_slope_term_dropped_x": ("Sx[c] = -(Pe - Pw) / dx + (g / (2.0 * dx)) * (HsLe * HsLe - HsRw * HsRw);",
                                 "Sx[c] = -(Pe - Pw) / dx;"),
    "force_y_uses_x_terms": ("(g / (2.0 * dx)) * (HsLn * HsLn - HsRs * HsRs)",
                             "(g / (2.0 * dx)) * (HsLe * HsLe - HsRw * HsRw)"),
    "force_y_wrong_neighbour": ("size_t n = c + nx;", "size_t n = c + 1;"),
    "manning_exponent": ("(Hf * cbrt(Hf))", "(Hf * sqrt(Hf))"),
    "predictor_full_step": ("(qx[c] + 0.5 * dt * (Sx[c] + Fx))", "(qx[c] + dt * (Sx[c] + Fx))"),
    "half_depth_multiplies": ("Hh[c] = H[c] / (Jx * Jy);", "Hh[c] = H[c] * (Jx * Jy);"),
    "transport_velocity_drops_vn": ("utx[c] = 0.5 * (u[c] + uLx[c]);", "utx[c] = uLx[c];"),
    "y_face_transposed_operand": ("double tL = FACEV(uty, sy[2], cL, +1), tR = FACEV(uty, sy[2], cR, -1);",
                                  "double tL = FACEV(utx, sy[2], cL, +1), tR = FACEV(uty, sy[2], cR, -1);"),
    "slope_ghost_normal_flag": ("const int fx_nx[5] = {0, 0, 1, 1, 0}", "const int fx_nx[5] = {0, 0, 1, 0, 0}"),
    "wall_flux_sign_east": ("side > 0 ? Hs * n * (u + fabs(u) + c)",
                            "side > 0 ? Hs * n * (u - fabs(u) + c)"),
    "limiter_minmod_is_maxmod": ("        m = fmin(A, B);", "        m = fmax(A, B);"),
    "limiter_mc_drops_half": ("0.5 * (A + B)", "(A + B)"),
    "limiter_superbee_is_min": ("m = fmax(fmin(2.0 * A, B), fmin(A, 2.0 * B));",
                                "m = fmin(fmin(2.0 * A, B), fmin(A, 2.0 * B));"),
    "slope_ignores_limiter_choice": ("orc_limiter(p->limiter, a0 - am, ap - a0)",
                                     "orc_limiter(ORC_LIM_MINMOD, a0 - am, ap - a0)"),
    "trr_celerity_sign": ("0.25 * (unL - unR)", "0.25 * (unR - unL)"),
    "trr_velocity_sign": ("*ustar = 0.5 * (unL + unR) + cL - cR;", "*ustar = 0.5 * (unL + unR) + cR - cL;"),
    "trr_speed_uses_left_head_twice": ("*SR = fmax(unR + cR, us + cs);", "*SR = fmax(unL + cL, us + cs);"),
    "trr_wall_ghost_not_mirrored": ("orc_hll_v(p->hll_speeds, p->g, Hs, n, t, u, Hs, -n, t, -u, f);",
                                    "orc_hll_v(p->hll_speeds, p->g, Hs, n, t, u, Hs, n, t, u, f);"),
    "coriolis_sign": ("*Fy = -p->coriolis * qxc", "*Fy = p->coriolis * qxc"),
    "coriolis_corrector_uses_qn": ("forcing(p, Hh[c], QPx[c], QPy[c], &Fx, &Fy);",
                                   "forcing(p, Hh[c], qx[c], qy[c], &Fx, &Fy);"),
    "wind_drops_depth_ramp": ("double chi = fmin(1.0, Hd / p->h_sed);", "double chi = 1.0;"),
    "wind_drops_speed_factor": ("p->wind_coef * Wm * p->wind_x * chi", "p->wind_coef * p->wind_x * chi"),
    "rain_dropped": (" + dt * src[c] + dt * p->rain;", " + dt * src[c];"),
    "absorption_explicit": ("double Ha = Hn / a;", "double Ha = Hn * (2.0 - a);"),
    "absorption_keeps_momentum": ("                qxn /= a;\n                qyn /= a;\n", ""),
    "open_boundary_blocks_mass": ("fl[0] = tL * HsL;\n                    fl[1] = tL * HsL * nL;\n                    fl[2] = tL * HsL * sL;\n                    fj = fmax(J0x[c], 0.0);",
                                  "fl[1] = tL * HsL * nL;\n                    fl[2] = tL * HsL * sL;\n                    fj = fmax(J0x[c], 0.0);"),
    "theta_wrong_donor": ("if (FH[f] > 0.0 && k - 1 >= 0) th = theta[(size_t)j * nx + k - 1];",
                          "if (FH[f] > 0.0 && k < nx) th = theta[(size_t)j * nx + k];"),
    "inflow_source_dropped": ("+ dt * src[c] + dt * p->rain;", "+ dt * p->rain;"),
    "exner_drops_porosity": ("double bn = b[c] - dt / (om * dx) *", "double bn = b[c] - dt / dx *"),
    "bed_slope_diffusion_sign": ("fj = fmax(J0x[cL], 0.0) + fmin(J0x[cR], 0.0) - CJ * mag",
                                 "fj = fmax(J0x[cL], 0.0) + fmin(J0x[cR], 0.0) + CJ * mag"),
    "bedload_downwind": ("fj = fmax(J0x[cL], 0.0) + fmin(J0x[cR], 0.0)",
                         "fj = fmax(J0x[cR], 0.0) + fmin(J0x[cL], 0.0)"),
    "eq4_drops_s_minus_one": ("((p->s_rel - 1.0) * sqrt(p->g * H) * d50)", "(p->s_rel * sqrt(p->g * H) * d50)"),
    "eq7_vp_term": ("h / (2.0 * vp)", "h / vp"),
    "eq7_D_term": ("h * h / (2.0 * D)", "h * h / D"),
    "shamov_exponent": ("cbrt(d50) * sqrt(cbrt(H))", "cbrt(d50) * cbrt(H)"),
    "hydrograph_at_step_start": ("orc_hydrograph(in, t + 0.5 * dt)", "orc_hydrograph(in, t)"),
    "hydrograph_at_step_end": ("orc_hydrograph(in, t + 0.5 * dt)", "orc_hydrograph(in, t + dt)"),
    "hydrograph_sigma_factor": ("exp(-d * d / (2.0 * s * s))", "exp(-d * d / (s * s))"),
    "force2_ignored": ("if (p->force_order == 2) forces_second", "if (p->force_order == 3) forces_second"),
    "force2_central_term_sign": ("- g * Hd[c] * sZx[c] / dx;", "+ g * Hd[c] * sZx[c] / dx;"),
    "force2_drops_central_term_y": ("(HsLn * HsLn - HsRs * HsRs)\n                    - g * Hd[c] * sZy[c] / dx;",
                                    "(HsLn * HsLn - HsRs * HsRs);"),
    "force2_own_side_wrong_half": ("zL = Z[c] + 0.5 * sZx[c];", "zL = Z[c] - 0.5 * sZx[c];"),
    "force2_neighbour_side_wrong_half": ("zR = Z[e] - 0.5 * sZx[e];", "zR = Z[e] + 0.5 * sZx[e];"),
    "force2_face_bed_from_cell_bed": ("bf = fmax(zL - hL, zR - hR);\n            HsL = fmax(0.0, zL - bf);\n            HsR = fmax(0.0, zR - bf);\n            Pe",
                                      "bf = fmax(b[c], zR - hR);\n            HsL = fmax(0.0, zL - bf);\n            HsR = fmax(0.0, zR - bf);\n            Pe"),
    "force2_depth_slope_is_surface_slope": ("sHx[c] = orc_limiter(p->limiter, Hd[c] - Hd[w], Hd[e] - Hd[c]);",
                                            "sHx[c] = sZx[c];"),
}


def _run_pins(lib):
    env = dict(os.environ, CSPH_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_variants.py"),
                        os.path.join(ROOT, "tests", "test_oracle_forcing.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


@pytest.mark.slow
def test_every_mutant_is_caught(oracle_mod):
    src = open(SRC).read()
    with tempfile.TemporaryDirectory() as d:
        jobs = {}
        for name, (old, new) in MUTANTS.items():
            assert src.count(old) >= 1, f"mutant {name}: pattern not found"
            msrc = os.path.join(d, f"{name}.c")
            with open(msrc, "w") as f:
                f.write(src.replace(old, new, 1))
            jobs[name] = oracle_mod.compile_source(msrc, os.path.join(d, f"{name}.so"))
        with ThreadPoolExecutor(max_workers=4) as ex:
            results = dict(zip(jobs, ex.map(_run_pins, jobs.values())))
    survivors = [n for n, (rc, _) in results.items() if rc == 0]
    assert not survivors, f"mutants not caught by any pin: {survivors}"
