/* Drives the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (host code only; tests/test_oracle_runtime.py compiles it with gcc):
 * every stage on small grids with walls and open sides, per-cell soil, an
 * inflow, bed sources, rain, absorption, Coriolis, wind, every limiter and
 * wave-speed estimate and both force orders.  Prints "ok" when every step
 * returned ORC_OK and the volumes are finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/csph_oracle.c"

static int run_case(int nx, int ny, int limiter, int speeds, int force_order, int sed_law)
{
    orc_params p = {0};
    p.nx = nx; p.ny = ny; p.dx = 2.0;
    p.bc[0] = 0; p.bc[1] = 1; p.bc[2] = 0; p.bc[3] = 1;
    p.g = 9.81; p.cfl = 0.3; p.eps = 1e-5; p.h_sed = 1e-2; p.dt_max = 1.0; p.dt_min = 1e-9;
    p.s_rel = 2.65; p.C_J = 2.0; p.C_Sh = 5.0; p.A_G = 1e-3; p.m_exp = 2.0;
    p.sed_law = sed_law; p.limiter = limiter; p.hll_speeds = speeds; p.force_order = force_order;
    p.rain = 1e-5; p.coriolis = 1e-4; p.wind_x = 6.0; p.wind_y = -2.0; p.wind_coef = 1.3e-6;
    const size_t n = (size_t)nx * ny;
    double *H = calloc(n, sizeof(double)), *qx = calloc(n, sizeof(double));
    double *qy = calloc(n, sizeof(double)), *b = calloc(n, sizeof(double));
    double *nM = malloc(n * sizeof(double)), *d50 = malloc(n * sizeof(double));
    double *psi = malloc(n * sizeof(double)), *qb = calloc(n, sizeof(double));
    double *beta = malloc(n * sizeof(double));
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            b[c] = 0.5 * sin(0.3 * i) * cos(0.2 * j) + 0.01 * i;
            H[c] = i < nx / 3 ? fmax(0.0, 2.0 - b[c]) : 0.0;
            nM[c] = 0.02 + 0.01 * ((i + j) % 3);
            d50[c] = 5e-4 + 1e-4 * (j % 4);
            psi[c] = 0.35 + 0.02 * (i % 3);
            beta[c] = 1e-3 * ((i * 7 + j) % 5);
        }
    qb[(size_t)(ny / 2) * nx + nx / 2] = 2e-6;
    int32_t idx[3] = {0, nx, 2 * nx};
    double w[3] = {0.25, 0.5, 0.25};
    orc_inputs in = {nM, d50, psi, qb, 3, idx, w, 5.0, 20.0, 4.0, 2.0, beta};
    orc_step_info info;
    double t = 0.0;
    int rc = ORC_OK;
    for (int s = 0; s < 40 && rc == ORC_OK; ++s) {
        rc = orc_step(&p, &in, H, qx, qy, b, t, 0.0, &info);
        t += info.dt;
    }
    double Vw = 0.0, Vs = 0.0;
    if (rc == ORC_OK) orc_volumes(&p, &in, H, b, &Vw, &Vs);
    if (rc == ORC_OK && !(isfinite(Vw) && isfinite(Vs))) rc = -100;
    double Sx[64 * 64], Sy[64 * 64];
    if (rc == ORC_OK && n <= 64 * 64) rc = orc_force(&p, H, b, Sx, Sy);
    free(H); free(qx); free(qy); free(b); free(nM); free(d50); free(psi); free(qb); free(beta);
    return rc;
}

int main(void)
{
    for (int lim = 0; lim < 3; ++lim)
        for (int sp = 0; sp < 2; ++sp)
            for (int fo = 1; fo <= 2; ++fo)
                for (int law = 1; law <= 2; ++law) {
                    int rc = run_case(23 + lim, 17 + sp, lim, sp, fo, law);
                    if (rc) {
                        printf("case %d %d %d %d: rc %d\n", lim, sp, fo, law, rc);
                        return 1;
                    }
                }
    printf("ok\n");
    return 0;
}
