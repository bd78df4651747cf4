/*
 * csph_oracle_f32.c -- the oracle's algorithm (csph_oracle.c, included below
 * unchanged) evaluated in IEEE float32 arithmetic, behind the same double
 * interface as orc_step.
 *
 * TEST INFRASTRUCTURE ONLY, and never a reference value: it measures how far
 * rounding at float32 precision alone moves the FP64 answer at each cell (the
 * conditioning of the problem there).  A cell where this float32 evaluation
 * already differs from the FP64 oracle by a tenth of a field's tolerance
 * cannot be held to that tolerance by any float32 implementation of the
 * step; the parity tests count and report such cells instead of asserting
 * the flat bound on them.  Compiled with -fsingle-precision-constant, so every
 * literal is a float and every operation rounds to float32 (math functions
 * round their double result to float).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* the double interface (the layouts of csph_oracle.c's structs) */
typedef struct {
    int32_t nx, ny;
    double dx;
    int32_t bc[4];
    double g, cfl, eps, h_sed, dt_max, dt_min, s_rel, C_J, C_Sh, A_G, m_exp;
    int32_t sed_law, limiter, hll_speeds;
    double rain, coriolis, wind_x, wind_y, wind_coef;
    int32_t force_order;
} f32_params_d;
typedef struct {
    const double *nM, *d50, *psi, *qb;
    int32_t n_inflow;
    const int32_t *inflow_idx;
    const double *inflow_w;
    double Q_base, Q_peak, t_peak, t_sigma;
    const double *beta;
} f32_inputs_d;
typedef struct {
    double dt, vp, vs, D;
    int32_t binding;
    double out_w, in_w, out_s, in_s, rain_in, absorbed;
} f32_info_d;

/* every name the oracle exports gets an _f32 suffix inside this unit */
#define double float
#define orc_step orc_step_f32
#define orc_cfl orc_cfl_f32
#define orc_volumes orc_volumes_f32
#define orc_w orc_w_f32
#define orc_minmod orc_minmod_f32
#define orc_limiter orc_limiter_f32
#define orc_j0 orc_j0_f32
#define orc_hll orc_hll_f32
#define orc_hll_v orc_hll_v_f32
#define orc_wave_speeds orc_wave_speeds_f32
#define orc_trr_star orc_trr_star_f32
#define orc_hydrograph orc_hydrograph_f32
#define orc_threads orc_threads_f32
#define orc_set_threads orc_set_threads_f32
#define orc_force orc_force_f32
#include "csph_oracle.c"
#undef double

static float *to_f32(const double *a, size_t n)
{
    if (!a) return NULL;
    float *f = malloc(n * sizeof(float));
    for (size_t i = 0; i < n; ++i) f[i] = (float)a[i];
    return f;
}

void orcf_set_threads(int n) { orc_set_threads_f32(n); }

/* One step of the oracle in float32: the double state is rounded to float,
 * stepped, and written back. */
int orcf_step(const f32_params_d *pd, const f32_inputs_d *id, double *H, double *qx, double *qy,
              double *b, double t, double dt_fixed, f32_info_d *info)
{
    orc_params p;
    p.nx = pd->nx; p.ny = pd->ny; p.dx = (float)pd->dx;
    for (int k = 0; k < 4; ++k) p.bc[k] = pd->bc[k];
    p.g = (float)pd->g; p.cfl = (float)pd->cfl; p.eps = (float)pd->eps; p.h_sed = (float)pd->h_sed;
    p.dt_max = (float)pd->dt_max; p.dt_min = (float)pd->dt_min; p.s_rel = (float)pd->s_rel;
    p.C_J = (float)pd->C_J; p.C_Sh = (float)pd->C_Sh; p.A_G = (float)pd->A_G;
    p.m_exp = (float)pd->m_exp; p.sed_law = pd->sed_law; p.limiter = pd->limiter;
    p.hll_speeds = pd->hll_speeds;
    p.rain = (float)pd->rain; p.coriolis = (float)pd->coriolis; p.wind_x = (float)pd->wind_x;
    p.wind_y = (float)pd->wind_y; p.wind_coef = (float)pd->wind_coef;
    p.force_order = pd->force_order;
    const size_t n = (size_t)p.nx * p.ny;
    orc_inputs in;
    in.nM = to_f32(id->nM, n); in.d50 = to_f32(id->d50, n); in.psi = to_f32(id->psi, n);
    in.qb = to_f32(id->qb, n);
    in.n_inflow = id->n_inflow; in.inflow_idx = id->inflow_idx;
    in.inflow_w = to_f32(id->inflow_w, (size_t)(id->n_inflow > 0 ? id->n_inflow : 0));
    in.Q_base = (float)id->Q_base; in.Q_peak = (float)id->Q_peak;
    in.t_peak = (float)id->t_peak; in.t_sigma = (float)id->t_sigma;
    in.beta = to_f32(id->beta, n);
    float *Hf = to_f32(H, n), *uf = to_f32(qx, n), *vf = to_f32(qy, n), *bf = to_f32(b, n);
    orc_step_info si;
    int rc = orc_step_f32(&p, &in, Hf, uf, vf, bf, (float)t, (float)dt_fixed, &si);
    for (size_t i = 0; i < n; ++i) {
        H[i] = Hf[i]; qx[i] = uf[i]; qy[i] = vf[i]; b[i] = bf[i];
    }
    info->dt = si.dt; info->vp = si.vp; info->vs = si.vs; info->D = si.D;
    info->binding = si.binding; info->out_w = si.out_w; info->in_w = si.in_w;
    info->out_s = si.out_s; info->in_s = si.in_s;
    info->rain_in = si.rain_in; info->absorbed = si.absorbed;
    free(Hf); free(uf); free(vf); free(bf);
    free((void *)in.nM); free((void *)in.d50); free((void *)in.psi); free((void *)in.qb);
    free((void *)in.inflow_w); free((void *)in.beta);
    return rc;
}
