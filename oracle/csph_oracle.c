/*
 * csph_oracle.c -- plain FP64 CPU oracle of one CSPH-TVD time step for the
 * coupled Saint-Venant (shallow water) + Exner (bed evolution) system of
 * Khrapov & Khoperskov, "Application of GPUs for self-consistent modelling of
 * shallow water dynamics and sediment transport", Lobachevskii J. Math. 41(8)
 * (2020) 1475-1484.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU path is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.  It
 * shares no code, header, table or constant with the HIP library.
 *
 * What is fixed by the paper and what is a reading
 * ------------------------------------------------
 * The paper prints the PDEs (Exner Eq. 1, slope-corrected bedload Eq. 2, Grass
 * law Eq. 3, coefficient Eq. 4, Shamov critical velocity Eq. 5, the vector
 * form Eq. 6), the time-step rule Eq. 7, and the kernel sequence K1..K8 of
 * Section 3 (forces at t_n, dt, predictor to t_{n+1/2}, forces at t_{n+1/2},
 * corrector, Euler-stage fluxes by piecewise-linear reconstruction + TVD
 * limiter + HLL, update).  It does not print the discretisation itself, so
 * the step below is one concrete reading of that sequence, with each choice
 * named where it is made (O1..O9).  The layout of the computation is the
 * simplest one: every stage loops over all cells (or all faces) of the grid,
 * writes whole-grid arrays, and the next stage reads them.  Faces are computed
 * once into face arrays and both neighbouring cells read the same value, so
 * the scheme is exactly conservative up to rounding.
 *
 * Parity pins (tests/test_oracle_*.py): lake at rest over uneven bed with
 * emerged islands, Stoker and Ritter dam breaks against the exact Riemann
 * solutions, water and sediment volume conservation, balance with open
 * boundaries and inflow, friction-only decay against its ODE, slope-diffusion
 * decay of a bed mode against its closed form, a hand-stepped 3-cell grid,
 * transpose / mirror / y-invariance symmetries, and the first time step.
 * Parity unpinned: the authors' own CSPH-TVD program (only this reading of it
 * exists here), the intended exponent of Eq. 4, and Eq. 7 omitting C_J.
 *
 * Layout: arrays are row-major [ny][nx], x fastest.  Sides are indexed
 * W=0, E=1, S=2, N=3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_BC_WALL 0
#define ORC_BC_OPEN 1

#define ORC_SED_NONE 0
#define ORC_SED_GRASS 1
#define ORC_SED_EQ4 2

#define ORC_LIM_MINMOD 0
#define ORC_LIM_MC 1
#define ORC_LIM_SUPERBEE 2

#define ORC_SPEEDS_DAVIS 0
#define ORC_SPEEDS_TWO_RAREFACTION 1

typedef struct {
    int32_t nx, ny;
    double dx;        /* cell size (uniform, dx = dy); "h" in Eq. 7 */
    int32_t bc[4];    /* W, E, S, N: 0 = wall (mirror), 1 = open (zero gradient) */
    double g;         /* gravity */
    double cfl;       /* Courant number K of Eq. 7 */
    double eps;       /* desingularisation depth */
    double h_sed;     /* no bedload at or below this depth */
    double dt_max, dt_min;
    double s_rel;     /* s = rho_s / rho of Eq. 4 */
    double C_J;       /* slope coefficient of Eq. 2 */
    double C_Sh;      /* Shamov coefficient of Eq. 5 */
    double A_G, m_exp;/* Grass law coefficient and exponent of Eq. 3 */
    int32_t sed_law;  /* 0 none, 1 Grass (A_G, m_exp), 2 Eq. 4 coefficient (m = 4) */
    int32_t limiter;  /* TVD limiter of the Euler stage: 0 minmod, 1 MC, 2 superbee */
    int32_t hll_speeds; /* HLL wave speeds: 0 Davis, 1 two-rarefaction (Toro) */
    /* Forcing named by Eq. 6's sigma and f without a formula (readings):    */
    double rain;      /* rainfall rate, m/s, on every cell (mass only)       */
    double coriolis;  /* Coriolis parameter f_c = 2 Omega sin(latitude), 1/s */
    double wind_x, wind_y; /* wind velocity W at 10 m, m/s                   */
    double wind_coef; /* C_w = (rho_air / rho_water) C_D, dimensionless      */
    int32_t force_order; /* Lagrangian force: 1 on cell values, 2 on states  */
                         /* reconstructed with the TVD limiter (O4)          */
} orc_params;

typedef struct {
    const double *nM;   /* Manning coefficient per cell            [ny*nx] */
    const double *d50;  /* median grain size per cell, m           [ny*nx] */
    const double *psi;  /* bed porosity per cell                   [ny*nx] */
    const double *qb;   /* q_b^+ - q_b^- per cell, m/s, or NULL    [ny*nx] */
    int32_t n_inflow;            /* number of inflow cells */
    const int32_t *inflow_idx;   /* flat cell index of each inflow cell */
    const double *inflow_w;      /* weight of each inflow cell (sum 1) */
    double Q_base, Q_peak, t_peak, t_sigma;  /* hydrograph, m^3/s */
    const double *beta; /* absorption (infiltration) coefficient, 1/s, or NULL [ny*nx] */
} orc_inputs;

typedef struct {
    double dt;          /* step actually taken */
    double vp, vs, D;   /* the three maxima of Eq. 7 at t_n */
    int32_t binding;    /* 0: h/(2 vp), 1: h/vs, 2: h^2/(2D), 3: dt_max, 4: fixed */
    double out_w;       /* water volume leaving through the boundary this step */
    double in_w;        /* water volume added by inflow this step */
    double out_s;       /* sediment volume (1-psi) b dx^2 leaving this step */
    double in_s;        /* sediment volume added by q_b this step */
    double rain_in;     /* water volume added by rainfall this step */
    double absorbed;    /* water volume absorbed (infiltrated) this step */
} orc_step_info;

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads an OpenMP loop of the oracle runs on. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the thread count of the oracle's OpenMP loops (timing at one thread). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_NONFINITE = -3, ORC_ERR_DT = -4, ORC_ERR_CFL = -6 };

/* ---------------------------------------------------------------------- */
/* O1  Velocity from momentum.  A cell's velocity is q * w(H), with w the   */
/* desingularised reciprocal depth of Kurganov & Petrova (2007): 1/H when   */
/* H >= eps, else sqrt(2) H / sqrt(H^4 + eps^4), which is continuous at     */
/* H = eps and vanishes at H = 0.                                           */
/* ---------------------------------------------------------------------- */
double orc_w(double H, double eps)
{
    if (H >= eps) return 1.0 / H;
    return sqrt(2.0) * H / sqrt(H * H * H * H + eps * eps * eps * eps);
}

/* minmod limiter (the TVD limiter of the Euler stage, Section 3). */
double orc_minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    if (a > 0.0) return a < b ? a : b;
    return a > b ? a : b;
}

/* The TVD limiters the Euler stage offers (Section 3 names TVD limiters      */
/* without fixing one): the limited slope of a cell from its backward and   */
/* forward differences a and b.  Zero unless a and b share a sign; else,    */
/* with A = |a|, B = |b| and the sign of a:                                  */
/*   minmod:   min(A, B)                                                    */
/*   MC (monotonised central, van Leer 1977): min(2A, 2B, (A + B)/2)         */
/*   superbee (Roe 1985): max(min(2A, B), min(A, 2B))                       */
double orc_limiter(int kind, double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    double A = fabs(a), B = fabs(b), m;
    if (kind == ORC_LIM_MC) {
        m = fmin(fmin(2.0 * A, 2.0 * B), 0.5 * (A + B));
    } else if (kind == ORC_LIM_SUPERBEE) {
        m = fmax(fmin(2.0 * A, B), fmin(A, 2.0 * B));
    } else {
        m = fmin(A, B);
    }
    return a > 0.0 ? m : -m;
}

/* ---------------------------------------------------------------------- */
/* O2  Zero-slope bedload J0 of one cell, Eqs. 3-5.  Bedload exists only    */
/* where the depth exceeds h_sed and the speed exceeds the Shamov critical  */
/* velocity v_k = C_Sh d50^(1/3) H^(1/6) (Eq. 5).  Then J0 = A |v|^m v with */
/* A = A_G, m = m_exp for the Grass law (Eq. 3), or A from Eq. 4,           */
/* A = 0.05 nM^3 / ((s-1) sqrt(g H) d50), with m = 4.                       */
/* ---------------------------------------------------------------------- */
void orc_j0(const orc_params *p, double H, double u, double v, double nM, double d50,
            double *jx, double *jy)
{
    *jx = 0.0;
    *jy = 0.0;
    if (p->sed_law == ORC_SED_NONE) return;
    if (!(H > p->h_sed)) return;
    double speed = sqrt(u * u + v * v);
    double vk = p->C_Sh * cbrt(d50) * sqrt(cbrt(H));  /* d50^(1/3) H^(1/6) */
    if (!(speed > vk)) return;
    double A, m;
    if (p->sed_law == ORC_SED_GRASS) {
        A = p->A_G;
        m = p->m_exp;
    } else {
        A = 0.05 * nM * nM * nM / ((p->s_rel - 1.0) * sqrt(p->g * H) * d50);
        m = 4.0;
    }
    double f = (m == 4.0) ? A * (speed * speed) * (speed * speed) : A * pow(speed, m);
    *jx = f * u;
    *jy = f * v;
}

/* Star state of the two-rarefaction approximation of the shallow-water    */
/* Riemann problem (Toro, Shock-capturing methods for free-surface shallow  */
/* flows, 2001): celerity c* = (cL + cR)/2 + (uL - uR)/4 and velocity       */
/* u* = (uL + uR)/2 + cL - cR, exact when both waves are rarefactions.  A   */
/* negative c* (the waves would open a dry middle) is taken as 0.           */
void orc_trr_star(double g, double HsL, double unL, double HsR, double unR, double *ustar,
                  double *cstar)
{
    double cL = sqrt(g * HsL), cR = sqrt(g * HsR);
    *ustar = 0.5 * (unL + unR) + cL - cR;
    *cstar = fmax(0.0, 0.5 * (cL + cR) + 0.25 * (unL - unR));
}

/* HLL wave-speed estimates from the side depths and transport velocities:  */
/* Davis, SL = min(uL - cL, uR - cR), SR = max(uL + cL, uR + cR); or the    */
/* two-rarefaction estimate, SL = min(uL - cL, u* - c*), SR = max(uR + cR,  */
/* u* + c*), with the star state above (no separate dry-bed forms: the      */
/* estimate stays continuous in the side states).                          */
void orc_wave_speeds(int kind, double g, double HsL, double unL, double HsR, double unR,
                     double *SL, double *SR)
{
    double cL = sqrt(g * HsL), cR = sqrt(g * HsR);
    if (kind == ORC_SPEEDS_TWO_RAREFACTION) {
        double us, cs;
        orc_trr_star(g, HsL, unL, HsR, unR, &us, &cs);
        *SL = fmin(unL - cL, us - cs);
        *SR = fmax(unR + cR, us + cs);
    } else {
        *SL = fmin(unL - cL, unR - cR);
        *SR = fmax(unL + cL, unR + cR);
    }
}

/* HLL flux of the remap (Euler stage, Section 3).  Side states are the     */
/* hydrostatic face depth Hs, the Lagrangian velocity (uLn normal, uLt      */
/* tangential) and the transport velocity un.  Conserved U = (Hs, Hs uLn,   */
/* Hs uLt), physical flux un * U, wave speeds of the chosen estimate.       */
/* Output f[0..2] = (mass, normal momentum, tangential momentum).           */
void orc_hll_v(int speeds, double g,
               double HsL, double uLnL, double uLtL, double unL,
               double HsR, double uLnR, double uLtR, double unR, double f[3])
{
    double UL[3] = {HsL, HsL * uLnL, HsL * uLtL};
    double UR[3] = {HsR, HsR * uLnR, HsR * uLtR};
    double FL[3], FR[3];
    for (int k = 0; k < 3; ++k) {
        FL[k] = unL * UL[k];
        FR[k] = unR * UR[k];
    }
    double SL, SR;
    orc_wave_speeds(speeds, g, HsL, unL, HsR, unR, &SL, &SR);
    for (int k = 0; k < 3; ++k) {
        if (SL >= 0.0) f[k] = FL[k];
        else if (SR <= 0.0) f[k] = FR[k];
        else if (SR - SL <= 0.0) f[k] = 0.0;
        else f[k] = (SR * FL[k] - SL * FR[k] + SL * SR * (UR[k] - UL[k])) / (SR - SL);
    }
}

/* The same with Davis speeds. */
void orc_hll(double g,
             double HsL, double uLnL, double uLtL, double unL,
             double HsR, double uLnR, double uLtR, double unR, double f[3])
{
    orc_hll_v(ORC_SPEEDS_DAVIS, g, HsL, uLnL, uLtL, unL, HsR, uLnR, uLtR, unR, f);
}

/* Hydrostatic face depths (Audusse et al. 2004) of a face between side     */
/* states with free surfaces zL, zR and depths HL, HR: the face bed is the  */
/* higher of the two side beds z - H, and each side depth is its surface    */
/* above that bed, never negative.                                          */
static void face_depths(double zL, double HL, double zR, double HR, double *HsL, double *HsR)
{
    double bL = zL - HL, bR = zR - HR;
    double bf = bL > bR ? bL : bR;
    *HsL = fmax(0.0, zL - bf);
    *HsR = fmax(0.0, zR - bf);
}

/* Hydrograph of the inflow cells: Q(t) = Q_base + Q_peak exp(-(t-tp)^2 / (2 s^2)). */
double orc_hydrograph(const orc_inputs *in, double t)
{
    double d = t - in->t_peak;
    double s = in->t_sigma;
    double pk = (s > 0.0) ? in->Q_peak * exp(-d * d / (2.0 * s * s)) : 0.0;
    return in->Q_base + pk;
}

/* ---------------------------------------------------------------------- */
/* O4  Lagrangian force per unit area on every cell column for a depth      */
/* field Hd over bed b: the pressure + bed-slope row of Phi in Eq. 6,       */
/* -g H grad(H + b), in hydrostatic-face form.  At each face the face bed   */
/* is max(b_L, b_R); each side depth is Hs = max(0, Hd + b - b_face); the   */
/* face pressure is P = (g/2) HsL HsR.  On cell i (x direction):            */
/*   Sx_i = -(P_{i+1/2} - P_{i-1/2})/dx                                     */
/*          + (g/(2 dx)) [ (HsL_{i+1/2})^2 - (HsR_{i-1/2})^2 ].             */
/* A boundary face sees a ghost copy of its cell (face bed = the cell's own */
/* bed), so there Hs = Hd and P = (g/2) Hd^2; it is evaluated through the   */
/* same expression as an interior face between two equal cells, so a       */
/* problem that is uniform along y stays exactly uniform.                   */
/* At rest over any bed (constant Hd + b where wet, dry banks               */
/* above it) every face has HsL = HsR and S = 0.                            */
/* ---------------------------------------------------------------------- */
static void forces_first(const orc_params *p, const double *Hd, const double *b, double *Sx,
                         double *Sy)
{
    const int nx = p->nx, ny = p->ny;
    const double g = p->g, dx = p->dx;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            double HsL, HsR, Pe, Pw, Pn, Ps, HsLe, HsRw, HsLn, HsRs;
            /* east face: cell is the left side */
            if (i + 1 < nx) {
                size_t e = c + 1;
                double bf = fmax(b[c], b[e]);
                HsL = fmax(0.0, Hd[c] + b[c] - bf);
                HsR = fmax(0.0, Hd[e] + b[e] - bf);
            } else {
                HsL = HsR = fmax(0.0, Hd[c] + b[c] - b[c]);
            }
            Pe = 0.5 * g * HsL * HsR;
            HsLe = HsL;
            /* west face: cell is the right side */
            if (i > 0) {
                size_t w = c - 1;
                double bf = fmax(b[w], b[c]);
                HsL = fmax(0.0, Hd[w] + b[w] - bf);
                HsR = fmax(0.0, Hd[c] + b[c] - bf);
            } else {
                HsL = HsR = fmax(0.0, Hd[c] + b[c] - b[c]);
            }
            Pw = 0.5 * g * HsL * HsR;
            HsRw = HsR;
            Sx[c] = -(Pe - Pw) / dx + (g / (2.0 * dx)) * (HsLe * HsLe - HsRw * HsRw);
            /* north face */
            if (j + 1 < ny) {
                size_t n = c + nx;
                double bf = fmax(b[c], b[n]);
                HsL = fmax(0.0, Hd[c] + b[c] - bf);
                HsR = fmax(0.0, Hd[n] + b[n] - bf);
            } else {
                HsL = HsR = fmax(0.0, Hd[c] + b[c] - b[c]);
            }
            Pn = 0.5 * g * HsL * HsR;
            HsLn = HsL;
            /* south face */
            if (j > 0) {
                size_t s = c - nx;
                double bf = fmax(b[s], b[c]);
                HsL = fmax(0.0, Hd[s] + b[s] - bf);
                HsR = fmax(0.0, Hd[c] + b[c] - bf);
            } else {
                HsL = HsR = fmax(0.0, Hd[c] + b[c] - b[c]);
            }
            Ps = 0.5 * g * HsL * HsR;
            HsRs = HsR;
            Sy[c] = -(Pn - Ps) / dx + (g / (2.0 * dx)) * (HsLn * HsLn - HsRs * HsRs);
        }
    }
}

/* ---------------------------------------------------------------------- */
/* O4, second-order form (force_order = 2; a reading: the paper names TVD   */
/* reconstruction only for the Euler stage).  The same hydrostatic-face     */
/* force, on side states reconstructed with the run's TVD limiter: a cell   */
/* with surface zeta = Hd + b and limited slopes s_zeta, s_H (per direction,*/
/* ghost cells copy their neighbour, so boundary cells have zero slope)     */
/* offers the face on its east (north) side zeta + s_zeta/2, Hd + s_H/2,    */
/* and on its west (south) side zeta - s_zeta/2, Hd - s_H/2, with the bed   */
/* side b_s = zeta_s - H_s.  At a face: b_face = max of the two side beds,  */
/* each side depth Hs = max(0, zeta_s - b_face), P = (g/2) HsL HsR.  On     */
/* cell i (x direction), with Audusse et al. (2004)'s centred term for the  */
/* bed slope inside the cell:                                               */
/*   Sx_i = -(P_{i+1/2} - P_{i-1/2})/dx                                     */
/*          + (g/(2 dx)) [ (HsL_{i+1/2})^2 - (HsR_{i-1/2})^2 ]              */
/*          - g Hd_i s_zeta_i / dx.                                         */
/* (The last term is what remains of Audusse's corrections                  */
/* g/2 (h_side^2 - Hs^2) and -g (h_w + h_e)/2 (b_e - b_w) once the side    */
/* depths h_e + h_w = 2 Hd_i and surfaces zeta_e - zeta_w = s_zeta_i are    */
/* used.)  With s = 0 it is the first-order form; at rest (zeta constant    */
/* where wet) every wet cell has s_zeta = 0 and every face balances.        */
/* ---------------------------------------------------------------------- */
static void forces_second(const orc_params *p, const double *Hd, const double *b, double *Sx,
                          double *Sy)
{
    const int nx = p->nx, ny = p->ny;
    const double g = p->g, dx = p->dx;
    const size_t n = (size_t)nx * ny;
    double *Z = (double *)malloc(n * sizeof(double));
    double *sZx = (double *)malloc(n * sizeof(double)), *sHx = (double *)malloc(n * sizeof(double));
    double *sZy = (double *)malloc(n * sizeof(double)), *sHy = (double *)malloc(n * sizeof(double));
    for (size_t c = 0; c < n; ++c) Z[c] = Hd[c] + b[c];
    /* limited slopes; the ghost of a boundary cell is the cell itself */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            size_t w = i > 0 ? c - 1 : c, e = i + 1 < nx ? c + 1 : c;
            size_t s = j > 0 ? c - nx : c, nn = j + 1 < ny ? c + nx : c;
            sZx[c] = orc_limiter(p->limiter, Z[c] - Z[w], Z[e] - Z[c]);
            sHx[c] = orc_limiter(p->limiter, Hd[c] - Hd[w], Hd[e] - Hd[c]);
            sZy[c] = orc_limiter(p->limiter, Z[c] - Z[s], Z[nn] - Z[c]);
            sHy[c] = orc_limiter(p->limiter, Hd[c] - Hd[s], Hd[nn] - Hd[c]);
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            double zL, hL, zR, hR, bf, HsL, HsR, Pe, Pw, Pn, Ps, HsLe, HsRw, HsLn, HsRs;
            /* east face: this cell's east side against the east cell's west side */
            zL = Z[c] + 0.5 * sZx[c];
            hL = Hd[c] + 0.5 * sHx[c];
            if (i + 1 < nx) {
                size_t e = c + 1;
                zR = Z[e] - 0.5 * sZx[e];
                hR = Hd[e] - 0.5 * sHx[e];
            } else {
                zR = zL;
                hR = hL;
            }
            bf = fmax(zL - hL, zR - hR);
            HsL = fmax(0.0, zL - bf);
            HsR = fmax(0.0, zR - bf);
            Pe = 0.5 * g * HsL * HsR;
            HsLe = HsL;
            /* west face: the west cell's east side against this cell's west side */
            zR = Z[c] - 0.5 * sZx[c];
            hR = Hd[c] - 0.5 * sHx[c];
            if (i > 0) {
                size_t w = c - 1;
                zL = Z[w] + 0.5 * sZx[w];
                hL = Hd[w] + 0.5 * sHx[w];
            } else {
                zL = zR;
                hL = hR;
            }
            bf = fmax(zL - hL, zR - hR);
            HsL = fmax(0.0, zL - bf);
            HsR = fmax(0.0, zR - bf);
            Pw = 0.5 * g * HsL * HsR;
            HsRw = HsR;
            Sx[c] = -(Pe - Pw) / dx + (g / (2.0 * dx)) * (HsLe * HsLe - HsRw * HsRw)
                    - g * Hd[c] * sZx[c] / dx;
            /* north face */
            zL = Z[c] + 0.5 * sZy[c];
            hL = Hd[c] + 0.5 * sHy[c];
            if (j + 1 < ny) {
                size_t nn = c + nx;
                zR = Z[nn] - 0.5 * sZy[nn];
                hR = Hd[nn] - 0.5 * sHy[nn];
            } else {
                zR = zL;
                hR = hL;
            }
            bf = fmax(zL - hL, zR - hR);
            HsL = fmax(0.0, zL - bf);
            HsR = fmax(0.0, zR - bf);
            Pn = 0.5 * g * HsL * HsR;
            HsLn = HsL;
            /* south face */
            zR = Z[c] - 0.5 * sZy[c];
            hR = Hd[c] - 0.5 * sHy[c];
            if (j > 0) {
                size_t s = c - nx;
                zL = Z[s] + 0.5 * sZy[s];
                hL = Hd[s] + 0.5 * sHy[s];
            } else {
                zL = zR;
                hL = hR;
            }
            bf = fmax(zL - hL, zR - hR);
            HsL = fmax(0.0, zL - bf);
            HsR = fmax(0.0, zR - bf);
            Ps = 0.5 * g * HsL * HsR;
            HsRs = HsR;
            Sy[c] = -(Pn - Ps) / dx + (g / (2.0 * dx)) * (HsLn * HsLn - HsRs * HsRs)
                    - g * Hd[c] * sZy[c] / dx;
        }
    }
    free(Z); free(sZx); free(sHx); free(sZy); free(sHy);
}

static void forces(const orc_params *p, const double *Hd, const double *b, double *Sx, double *Sy)
{
    if (p->force_order == 2) forces_second(p, Hd, b, Sx, Sy);
    else forces_first(p, Hd, b, Sx, Sy);
}

/* The O4 force alone on a state (the first- or second-order form of the    */
/* run's parameters), for pins of its consistency.                          */
int orc_force(const orc_params *p, const double *Hd, const double *b, double *Sx, double *Sy)
{
    if (!p || !Hd || !b || !Sx || !Sy || p->nx < 1 || p->ny < 1) return ORC_ERR_ARG;
    forces(p, Hd, b, Sx, Sy);
    return ORC_OK;
}

/* External forces per unit area on the momentum q of a column of depth    */
/* Hd (the Earth-rotation and wind parts of f in Eq. 6, readings):          */
/*   Coriolis  f_c (q_y, -q_x), turning the flow to the right for f_c > 0;  */
/*   wind      C_w |W| W chi(Hd), chi = min(1, Hd / h_sed): the stress acts */
/*             on water at least h_sed deep and fades to zero on a drying   */
/*             cell (continuous at Hd = 0).                                  */
static void forcing(const orc_params *p, double Hd, double qxc, double qyc, double *Fx, double *Fy)
{
    double Wm = sqrt(p->wind_x * p->wind_x + p->wind_y * p->wind_y);
    double chi = fmin(1.0, Hd / p->h_sed);
    *Fx = p->coriolis * qyc + p->wind_coef * Wm * p->wind_x * chi;
    *Fy = -p->coriolis * qxc + p->wind_coef * Wm * p->wind_y * chi;
}

/* Manning friction rate gamma = g nM^2 |v| / max(H, eps)^(4/3), applied    */
/* semi-implicitly (the bottom-friction part of f in Eq. 6).                */
static double friction_rate(const orc_params *p, double nM, double speed, double H)
{
    double Hf = H > p->eps ? H : p->eps;
    return p->g * nM * nM * speed / (Hf * cbrt(Hf));  /* Hf^(4/3) */
}

/* ---------------------------------------------------------------------- */
/* O3  Time step of Eq. 7 on the state at t_n:                              */
/*   tau = K min( h/(2 vp), h/vs, h^2/(2 D) ),                              */
/*   vp = max|v|, vs = max(|v| + sqrt(g H)), D = max |J0| / (1 - psi),      */
/* over all cells; a term with a zero denominator is infinite; the result   */
/* is capped at dt_max.                                                     */
/* ---------------------------------------------------------------------- */
int orc_cfl(const orc_params *p, const orc_inputs *in, const double *H, const double *qx,
            const double *qy, double *dt, double *vp_o, double *vs_o, double *D_o, int32_t *binding)
{
    const size_t n = (size_t)p->nx * p->ny;
    double vp = 0.0, vs = 0.0, D = 0.0;
    int bad = 0;
    /* maxima are independent of the order they are taken in */
#pragma omp parallel for schedule(static) reduction(max : vp, vs, D) reduction(| : bad)
    for (size_t c = 0; c < n; ++c) {
        double w = orc_w(H[c], p->eps);
        double u = qx[c] * w, v = qy[c] * w;
        double sp = sqrt(u * u + v * v);
        double cs = sqrt(p->g * (H[c] > 0.0 ? H[c] : 0.0));
        double jx, jy;
        orc_j0(p, H[c], u, v, in->nM[c], in->d50[c], &jx, &jy);
        double Dc = sqrt(jx * jx + jy * jy) / (1.0 - in->psi[c]);
        if (!isfinite(sp) || !isfinite(Dc) || !isfinite(H[c])) bad = 1;
        if (sp > vp) vp = sp;
        if (sp + cs > vs) vs = sp + cs;
        if (Dc > D) D = Dc;
    }
    double h = p->dx;
    double t0 = vp > 0.0 ? h / (2.0 * vp) : INFINITY;
    double t1 = vs > 0.0 ? h / vs : INFINITY;
    double t2 = D > 0.0 ? h * h / (2.0 * D) : INFINITY;
    double m = t0;
    int which = 0;
    if (t1 < m) { m = t1; which = 1; }
    if (t2 < m) { m = t2; which = 2; }
    double d = p->cfl * m;
    if (!(d < p->dt_max)) { d = p->dt_max; which = 3; }
    *dt = d;
    if (vp_o) *vp_o = vp;
    if (vs_o) *vs_o = vs;
    if (D_o) *D_o = D;
    if (binding) *binding = which;
    if (bad) return ORC_ERR_NONFINITE;
    return ORC_OK;
}

/* Normal-momentum flux through a wall face: the HLL flux against the      */
/* mirrored ghost of the interior face state (depth Hs, Lagrangian velocity */
/* normal n and tangential t, transport velocity u).  It carries no mass    */
/* and no tangential momentum.  With Davis speeds this is                   */
/* Hs n (u + |u| + c) for an interior cell on the minus side (E/N wall,     */
/* side = +1) and Hs n (u - |u| - c) on the plus side (W/S wall).           */
static double wall_flux_n(const orc_params *p, double Hs, double n, double t, double u, int side)
{
    if (p->hll_speeds == ORC_SPEEDS_DAVIS) {
        double c = sqrt(p->g * Hs);
        return side > 0 ? Hs * n * (u + fabs(u) + c) : Hs * n * (u - fabs(u) - c);
    }
    double f[3];
    if (side > 0)
        orc_hll_v(p->hll_speeds, p->g, Hs, n, t, u, Hs, -n, t, -u, f);
    else
        orc_hll_v(p->hll_speeds, p->g, Hs, -n, t, -u, Hs, n, t, u, f);
    return f[1];
}

/* Ghost rule: value of a per-cell field at cell (i,j) when (i,j) may sit   */
/* one cell outside the grid.  A wall mirrors (the normal velocity          */
/* component flips sign, everything else is copied); an open side copies.   */
/* `normal_x` / `normal_y` say whether the field is the x / y component of  */
/* a velocity.                                                              */
static double ghost(const orc_params *p, const double *a, int i, int j, int normal_x, int normal_y)
{
    const int nx = p->nx, ny = p->ny;
    int ci = i, cj = j;
    double sgn = 1.0;
    if (i < 0) { ci = 0; if (p->bc[0] == ORC_BC_WALL && normal_x) sgn = -1.0; }
    if (i >= nx) { ci = nx - 1; if (p->bc[1] == ORC_BC_WALL && normal_x) sgn = -1.0; }
    if (j < 0) { cj = 0; if (p->bc[2] == ORC_BC_WALL && normal_y) sgn = -1.0; }
    if (j >= ny) { cj = ny - 1; if (p->bc[3] == ORC_BC_WALL && normal_y) sgn = -1.0; }
    return sgn * a[(size_t)cj * nx + ci];
}

/* Limited slope of field a at cell (i,j) along x (dir 0) or y (dir 1),    */
/* with the run's TVD limiter.                                              */
static double slope(const orc_params *p, const double *a, int i, int j, int dir, int nxf, int nyf)
{
    double am, a0, ap;
    a0 = a[(size_t)j * p->nx + i];
    if (dir == 0) {
        am = ghost(p, a, i - 1, j, nxf, nyf);
        ap = ghost(p, a, i + 1, j, nxf, nyf);
    } else {
        am = ghost(p, a, i, j - 1, nxf, nyf);
        ap = ghost(p, a, i, j + 1, nxf, nyf);
    }
    return orc_limiter(p->limiter, a0 - am, ap - a0);
}

/* ---------------------------------------------------------------------- */
/* One CSPH-TVD step.  Arrays H, qx, qy, b are updated in place from t_n to */
/* t_{n+1}.  dt_fixed <= 0 selects the Eq. 7 step; dt_fixed > 0 takes that  */
/* step and fails with ORC_ERR_CFL if it exceeds the Eq. 7 step.            */
/* ---------------------------------------------------------------------- */
int orc_step(const orc_params *p, const orc_inputs *in, double *H, double *qx, double *qy,
             double *b, double t, double dt_fixed, orc_step_info *info)
{
    const int nx = p->nx, ny = p->ny;
    if (nx < 1 || ny < 1 || !(p->dx > 0.0)) return ORC_ERR_ARG;
    const size_t n = (size_t)nx * ny;
    const double g = p->g, dx = p->dx, eps = p->eps;

    memset(info, 0, sizeof(*info));

    /* O3 (K3): time step from the state at t_n. */
    double dt, vp, vs, D;
    int32_t binding;
    int rc = orc_cfl(p, in, H, qx, qy, &dt, &vp, &vs, &D, &binding);
    info->vp = vp;
    info->vs = vs;
    info->D = D;
    if (rc != ORC_OK) return rc;
    if (dt_fixed > 0.0) {
        if (dt_fixed > dt) return ORC_ERR_CFL;
        dt = dt_fixed;
        binding = 4;
    }
    if (dt < p->dt_min) return ORC_ERR_DT;
    info->dt = dt;
    info->binding = binding;

    double *u = malloc(n * sizeof(double)), *v = malloc(n * sizeof(double));
    double *Sx = malloc(n * sizeof(double)), *Sy = malloc(n * sizeof(double));
    double *up = malloc(n * sizeof(double)), *vpv = malloc(n * sizeof(double));
    double *Hh = malloc(n * sizeof(double));
    double *QPx = malloc(n * sizeof(double)), *QPy = malloc(n * sizeof(double));
    double *QLx = malloc(n * sizeof(double)), *QLy = malloc(n * sizeof(double));
    double *uLx = malloc(n * sizeof(double)), *uLy = malloc(n * sizeof(double));
    double *utx = malloc(n * sizeof(double)), *uty = malloc(n * sizeof(double));
    double *zeta = malloc(n * sizeof(double));
    double *J0x = malloc(n * sizeof(double)), *J0y = malloc(n * sizeof(double));
    double *theta = malloc(n * sizeof(double));
    /* x faces: (nx+1) per row, face k sits west of cell k; y faces likewise. */
    const size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);
    double *FH = malloc(nfx * sizeof(double)), *Fqx = malloc(nfx * sizeof(double));
    double *Fqy = malloc(nfx * sizeof(double)), *FJ = malloc(nfx * sizeof(double));
    double *GH = malloc(nfy * sizeof(double)), *Gqx = malloc(nfy * sizeof(double));
    double *Gqy = malloc(nfy * sizeof(double)), *GJ = malloc(nfy * sizeof(double));

    /* O1 + O2 (K2): velocities and bedload at t_n. */
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < n; ++c) {
        double w = orc_w(H[c], eps);
        u[c] = qx[c] * w;
        v[c] = qy[c] * w;
        orc_j0(p, H[c], u[c], v[c], in->nM[c], in->d50[c], &J0x[c], &J0y[c]);
    }

    /* O4 + O5 (K2, K4): forces at t_n; predictor momentum and velocity;    */
    /* half-step depth from the deformation of each column's area under the */
    /* face-mean velocities at t_n over dt/2.                               */
    forces(p, H, b, Sx, Sy);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            double sp = sqrt(u[c] * u[c] + v[c] * v[c]);
            double gam = friction_rate(p, in->nM[c], sp, H[c]);
            double w = orc_w(H[c], eps);
            double Fx, Fy;
            forcing(p, H[c], qx[c], qy[c], &Fx, &Fy);
            double qpx = (qx[c] + 0.5 * dt * (Sx[c] + Fx)) / (1.0 + 0.5 * dt * gam);
            double qpy = (qy[c] + 0.5 * dt * (Sy[c] + Fy)) / (1.0 + 0.5 * dt * gam);
            QPx[c] = qpx;
            QPy[c] = qpy;
            up[c] = qpx * w;
            vpv[c] = qpy * w;
            /* face-mean velocities: interior mean; wall 0; open = the cell's own */
            double ue, uw, vn, vs_;
            if (i + 1 < nx) ue = 0.5 * (u[c] + u[c + 1]);
            else ue = (p->bc[1] == ORC_BC_WALL) ? 0.0 : u[c];
            if (i > 0) uw = 0.5 * (u[c - 1] + u[c]);
            else uw = (p->bc[0] == ORC_BC_WALL) ? 0.0 : u[c];
            if (j + 1 < ny) vn = 0.5 * (v[c] + v[c + nx]);
            else vn = (p->bc[3] == ORC_BC_WALL) ? 0.0 : v[c];
            if (j > 0) vs_ = 0.5 * (v[c - nx] + v[c]);
            else vs_ = (p->bc[2] == ORC_BC_WALL) ? 0.0 : v[c];
            double Jx = 1.0 + (dt / (2.0 * dx)) * (ue - uw);
            double Jy = 1.0 + (dt / (2.0 * dx)) * (vn - vs_);
            Hh[c] = H[c] / (Jx * Jy);
        }
    }

    /* O6 (K5, K6): forces at t_{n+1/2} on the half-step depths (bed b^n),  */
    /* corrector momentum Q^L, Lagrangian velocity u^L and the transport    */
    /* velocity u~ = (v^n + u^L)/2 that carries the remap.                  */
    forces(p, Hh, b, Sx, Sy);
#pragma omp parallel for schedule(static)
    for (size_t c = 0; c < n; ++c) {
        double spp = sqrt(up[c] * up[c] + vpv[c] * vpv[c]);
        double gam = friction_rate(p, in->nM[c], spp, Hh[c]);
        double Fx, Fy;  /* forcing at t_{n+1/2}: half-step depth, predictor momentum */
        forcing(p, Hh[c], QPx[c], QPy[c], &Fx, &Fy);
        QLx[c] = (qx[c] + dt * (Sx[c] + Fx)) / (1.0 + dt * gam);
        QLy[c] = (qy[c] + dt * (Sy[c] + Fy)) / (1.0 + dt * gam);
        double w = orc_w(H[c], eps);
        uLx[c] = QLx[c] * w;
        uLy[c] = QLy[c] * w;
        utx[c] = 0.5 * (u[c] + uLx[c]);
        uty[c] = 0.5 * (v[c] + uLy[c]);
        zeta[c] = H[c] + b[c];
    }

    /* O7 (K7): Euler-stage raw fluxes on every face.  Per direction, the   */
    /* free surface zeta, the depth H, the normal transport velocity and    */
    /* both Lagrangian velocity components are reconstructed piecewise      */
    /* linearly with minmod slopes; face depths are hydrostatic; the water  */
    /* flux is HLL; the bedload flux is the flux-split donor cell of J0     */
    /* plus the slope term of Eq. 2, -C_J |J0| grad b, with |J0| averaged.  */
    /* Slopes first: sx[k] / sy[k] hold the limited slope of field k of     */
    /* each cell along x / y (fields: zeta, H, normal transport velocity,   */
    /* normal and tangential Lagrangian velocity; ghosts per the BC).       */
    const double CJ = p->C_J;
    double *sx[5], *sy[5];
    for (int k = 0; k < 5; ++k) {
        sx[k] = malloc(n * sizeof(double));
        sy[k] = malloc(n * sizeof(double));
    }
    const double *fx[5] = {zeta, H, utx, uLx, uLy};  /* along x: normal = x */
    const int fx_nx[5] = {0, 0, 1, 1, 0}, fx_ny[5] = {0, 0, 0, 0, 1};
    const double *fy[5] = {zeta, H, uty, uLy, uLx};  /* along y: normal = y */
    const int fy_nx[5] = {0, 0, 0, 0, 1}, fy_ny[5] = {0, 0, 1, 1, 0};
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            for (int k = 0; k < 5; ++k) {
                sx[k][c] = slope(p, fx[k], i, j, 0, fx_nx[k], fx_ny[k]);
                sy[k][c] = slope(p, fy[k], i, j, 1, fy_nx[k], fy_ny[k]);
            }
        }
    }
    /* face values of cell c on its plus (+0.5 slope) or minus (-0.5) side */
#define FACEV(arr, sl, c, side) ((arr)[c] + 0.5 * (side) * (sl)[c])
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int k = 0; k <= nx; ++k) {
            size_t f = (size_t)j * (nx + 1) + k;
            int iL = k - 1, iR = k;  /* cells west / east of face k */
            double fl[3] = {0.0, 0.0, 0.0}, fj = 0.0;
            if (iL >= 0 && iR < nx) {
                size_t cL = (size_t)j * nx + iL, cR = cL + 1;
                double zL = FACEV(zeta, sx[0], cL, +1), zR = FACEV(zeta, sx[0], cR, -1);
                double hL = FACEV(H, sx[1], cL, +1), hR = FACEV(H, sx[1], cR, -1);
                double tL = FACEV(utx, sx[2], cL, +1), tR = FACEV(utx, sx[2], cR, -1);
                double nL = FACEV(uLx, sx[3], cL, +1), nR = FACEV(uLx, sx[3], cR, -1);
                double sL = FACEV(uLy, sx[4], cL, +1), sR = FACEV(uLy, sx[4], cR, -1);
                double HsL, HsR;
                face_depths(zL, hL, zR, hR, &HsL, &HsR);
                orc_hll_v(p->hll_speeds, g, HsL, nL, sL, tL, HsR, nR, sR, tR, fl);
                double mag = 0.5 * (sqrt(J0x[cL] * J0x[cL] + J0y[cL] * J0y[cL]) +
                                    sqrt(J0x[cR] * J0x[cR] + J0y[cR] * J0y[cR]));
                fj = fmax(J0x[cL], 0.0) + fmin(J0x[cR], 0.0) - CJ * mag * (b[cR] - b[cL]) / dx;
            } else if (iR == nx) {  /* east boundary, interior cell on the left */
                size_t c = (size_t)j * nx + nx - 1;
                double zL = FACEV(zeta, sx[0], c, +1), hL = FACEV(H, sx[1], c, +1);
                double tL = FACEV(utx, sx[2], c, +1), nL = FACEV(uLx, sx[3], c, +1);
                double sL = FACEV(uLy, sx[4], c, +1);
                double HsL, HsR;
                face_depths(zL, hL, zL, hL, &HsL, &HsR);
                if (p->bc[1] == ORC_BC_WALL) {
                    fl[1] = wall_flux_n(p, HsL, nL, sL, tL, +1);
                } else {
                    fl[0] = tL * HsL;
                    fl[1] = tL * HsL * nL;
                    fl[2] = tL * HsL * sL;
                    fj = fmax(J0x[c], 0.0);
                }
            } else {  /* west boundary, interior cell on the right */
                size_t c = (size_t)j * nx;
                double zR = FACEV(zeta, sx[0], c, -1), hR = FACEV(H, sx[1], c, -1);
                double tR = FACEV(utx, sx[2], c, -1), nR = FACEV(uLx, sx[3], c, -1);
                double sR = FACEV(uLy, sx[4], c, -1);
                double HsL, HsR;
                face_depths(zR, hR, zR, hR, &HsL, &HsR);
                if (p->bc[0] == ORC_BC_WALL) {
                    fl[1] = wall_flux_n(p, HsR, nR, sR, tR, -1);
                } else {
                    fl[0] = tR * HsR;
                    fl[1] = tR * HsR * nR;
                    fl[2] = tR * HsR * sR;
                    fj = fmin(J0x[c], 0.0);
                }
            }
            FH[f] = fl[0];
            Fqx[f] = fl[1];  /* normal = x */
            Fqy[f] = fl[2];  /* tangential = y */
            FJ[f] = fj;
        }
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= ny; ++k) {
        for (int i = 0; i < nx; ++i) {
            size_t f = (size_t)k * nx + i;
            int jL = k - 1, jR = k;  /* cells south / north of face k */
            double fl[3] = {0.0, 0.0, 0.0}, fj = 0.0;
            if (jL >= 0 && jR < ny) {
                size_t cL = (size_t)jL * nx + i, cR = cL + nx;
                double zL = FACEV(zeta, sy[0], cL, +1), zR = FACEV(zeta, sy[0], cR, -1);
                double hL = FACEV(H, sy[1], cL, +1), hR = FACEV(H, sy[1], cR, -1);
                double tL = FACEV(uty, sy[2], cL, +1), tR = FACEV(uty, sy[2], cR, -1);
                double nL = FACEV(uLy, sy[3], cL, +1), nR = FACEV(uLy, sy[3], cR, -1);
                double sL = FACEV(uLx, sy[4], cL, +1), sR = FACEV(uLx, sy[4], cR, -1);
                double HsL, HsR;
                face_depths(zL, hL, zR, hR, &HsL, &HsR);
                orc_hll_v(p->hll_speeds, g, HsL, nL, sL, tL, HsR, nR, sR, tR, fl);
                double mag = 0.5 * (sqrt(J0x[cL] * J0x[cL] + J0y[cL] * J0y[cL]) +
                                    sqrt(J0x[cR] * J0x[cR] + J0y[cR] * J0y[cR]));
                fj = fmax(J0y[cL], 0.0) + fmin(J0y[cR], 0.0) - CJ * mag * (b[cR] - b[cL]) / dx;
            } else if (jR == ny) {  /* north boundary */
                size_t c = (size_t)(ny - 1) * nx + i;
                double zL = FACEV(zeta, sy[0], c, +1), hL = FACEV(H, sy[1], c, +1);
                double tL = FACEV(uty, sy[2], c, +1), nL = FACEV(uLy, sy[3], c, +1);
                double sL = FACEV(uLx, sy[4], c, +1);
                double HsL, HsR;
                face_depths(zL, hL, zL, hL, &HsL, &HsR);
                if (p->bc[3] == ORC_BC_WALL) {
                    fl[1] = wall_flux_n(p, HsL, nL, sL, tL, +1);
                } else {
                    fl[0] = tL * HsL;
                    fl[1] = tL * HsL * nL;
                    fl[2] = tL * HsL * sL;
                    fj = fmax(J0y[c], 0.0);
                }
            } else {  /* south boundary */
                size_t c = (size_t)i;
                double zR = FACEV(zeta, sy[0], c, -1), hR = FACEV(H, sy[1], c, -1);
                double tR = FACEV(uty, sy[2], c, -1), nR = FACEV(uLy, sy[3], c, -1);
                double sR = FACEV(uLx, sy[4], c, -1);
                double HsL, HsR;
                face_depths(zR, hR, zR, hR, &HsL, &HsR);
                if (p->bc[2] == ORC_BC_WALL) {
                    fl[1] = wall_flux_n(p, HsR, nR, sR, tR, -1);
                } else {
                    fl[0] = tR * HsR;
                    fl[1] = tR * HsR * nR;
                    fl[2] = tR * HsR * sR;
                    fj = fmin(J0y[c], 0.0);
                }
            }
            GH[f] = fl[0];
            Gqy[f] = fl[1];  /* normal = y */
            Gqx[f] = fl[2];  /* tangential = x */
            GJ[f] = fj;
        }
    }
#undef FACEV
    for (int k = 0; k < 5; ++k) {
        free(sx[k]);
        free(sy[k]);
    }

    /* Positivity: the draining limiter.  theta_i scales every flux that    */
    /* drains cell i so that its outflow over the step cannot exceed its    */
    /* water H_i dx^2.                                                      */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            double fe = FH[(size_t)j * (nx + 1) + i + 1], fw = FH[(size_t)j * (nx + 1) + i];
            double gn = GH[(size_t)(j + 1) * nx + i], gs = GH[(size_t)j * nx + i];
            double out = fmax(0.0, fe) + fmax(0.0, -fw) + fmax(0.0, gn) + fmax(0.0, -gs);
            theta[c] = out > 0.0 ? fmin(1.0, H[c] * dx / (dt * out)) : 1.0;
        }
    }
    /* Each face's water fluxes take the theta of their donor cell (the     */
    /* cell the mass leaves); a ghost donor has theta = 1.                  */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
        for (int k = 0; k <= nx; ++k) {
            size_t f = (size_t)j * (nx + 1) + k;
            double th = 1.0;
            if (FH[f] > 0.0 && k - 1 >= 0) th = theta[(size_t)j * nx + k - 1];
            if (FH[f] < 0.0 && k < nx) th = theta[(size_t)j * nx + k];
            FH[f] *= th;
            Fqx[f] *= th;
            Fqy[f] *= th;
        }
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= ny; ++k) {
        for (int i = 0; i < nx; ++i) {
            size_t f = (size_t)k * nx + i;
            double th = 1.0;
            if (GH[f] > 0.0 && k - 1 >= 0) th = theta[(size_t)(k - 1) * nx + i];
            if (GH[f] < 0.0 && k < ny) th = theta[(size_t)k * nx + i];
            GH[f] *= th;
            Gqx[f] *= th;
            Gqy[f] *= th;
        }
    }

    /* O8 (K8): conservative update from the face fluxes, the inflow source */
    /* at t_n + dt/2 and the rainfall (mass only), and the Exner update     */
    /* (Eq. 1) with the cell's porosity.  A tiny negative depth left by     */
    /* rounding is set to zero.  Absorption (the infiltration part of sigma, */
    /* reading: dH/dt = -beta H, implicit) divides depth and momentum by    */
    /* 1 + beta dt, so the water it removes leaves with its velocity.  A    */
    /* thin film's momentum is re-desingularised, q <- H w(H) q.            */
    double Qmid = orc_hydrograph(in, t + 0.5 * dt);
    double *src = calloc(n, sizeof(double));
    for (int k = 0; k < in->n_inflow; ++k)
        src[in->inflow_idx[k]] += Qmid * in->inflow_w[k] / (dx * dx);
    int nonfinite = 0;
    double absorbed = 0.0;
#pragma omp parallel for schedule(static) reduction(| : nonfinite) reduction(+ : absorbed)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            size_t c = (size_t)j * nx + i;
            size_t fw = (size_t)j * (nx + 1) + i, fe = fw + 1;
            size_t gs = (size_t)j * nx + i, gn = gs + nx;
            double r = dt / dx;
            double Hn = H[c] - r * ((FH[fe] - FH[fw]) + (GH[gn] - GH[gs])) + dt * src[c] + dt * p->rain;
            double qxn = QLx[c] - r * ((Fqx[fe] - Fqx[fw]) + (Gqx[gn] - Gqx[gs]));
            double qyn = QLy[c] - r * ((Fqy[fe] - Fqy[fw]) + (Gqy[gn] - Gqy[gs]));
            double om = 1.0 - in->psi[c];
            double bn = b[c] - dt / (om * dx) * ((FJ[fe] - FJ[fw]) + (GJ[gn] - GJ[gs]));
            if (in->qb) bn += dt * in->qb[c] / om;
            if (Hn < 0.0) Hn = 0.0;
            if (in->beta && in->beta[c] > 0.0) {
                double a = 1.0 + in->beta[c] * dt;
                double Ha = Hn / a;
                absorbed += Hn - Ha;
                Hn = Ha;
                qxn /= a;
                qyn /= a;
            }
            if (Hn < eps) {
                double s = Hn * orc_w(Hn, eps);
                qxn *= s;
                qyn *= s;
            }
            if (!isfinite(Hn) || !isfinite(qxn) || !isfinite(qyn) || !isfinite(bn)) nonfinite = 1;
            H[c] = Hn;
            qx[c] = qxn;
            qy[c] = qyn;
            b[c] = bn;
        }
    }

    /* O9: boundary outflow and source volumes of this step. */
    double ow = 0.0, os = 0.0;
    for (int j = 0; j < ny; ++j) {
        ow += -FH[(size_t)j * (nx + 1)] + FH[(size_t)j * (nx + 1) + nx];
        os += -FJ[(size_t)j * (nx + 1)] + FJ[(size_t)j * (nx + 1) + nx];
    }
    for (int i = 0; i < nx; ++i) {
        ow += -GH[i] + GH[(size_t)ny * nx + i];
        os += -GJ[i] + GJ[(size_t)ny * nx + i];
    }
    info->out_w = dt * dx * ow;
    info->out_s = dt * dx * os;
    info->in_w = in->n_inflow > 0 ? dt * Qmid : 0.0;
    double qbs = 0.0;
    if (in->qb)
        for (size_t c = 0; c < n; ++c) qbs += in->qb[c];
    info->in_s = dt * qbs * dx * dx;
    info->rain_in = dt * p->rain * (double)n * dx * dx;
    info->absorbed = absorbed * dx * dx;

    free(u); free(v); free(Sx); free(Sy); free(up); free(vpv); free(Hh); free(QPx); free(QPy);
    free(QLx); free(QLy); free(uLx); free(uLy); free(utx); free(uty); free(zeta);
    free(J0x); free(J0y); free(theta);
    free(FH); free(Fqx); free(Fqy); free(FJ); free(GH); free(Gqx); free(Gqy); free(GJ);
    free(src);
    return nonfinite ? ORC_ERR_NONFINITE : ORC_OK;
}

/* O9: water volume sum H dx^2 and sediment volume sum (1 - psi) b dx^2,    */
/* summed in cell order.                                                    */
void orc_volumes(const orc_params *p, const orc_inputs *in, const double *H, const double *b,
                 double *Vw, double *Vs)
{
    const size_t n = (size_t)p->nx * p->ny;
    double sw = 0.0, ss = 0.0;
    for (size_t c = 0; c < n; ++c) {
        sw += H[c];
        ss += (1.0 - in->psi[c]) * b[c];
    }
    *Vw = sw * p->dx * p->dx;
    *Vs = ss * p->dx * p->dx;
}
