// csph_device.h -- FP32 device arithmetic of one CSPH-TVD step on gfx950.
//
// Every kernel of the library computes a cell, a face or a force through the
// functions below, so a face flux evaluated by two different tiles (or two
// different kernel variants) uses the same operations in the same order and
// gives the same bits.  The step follows Section 3 of Khrapov & Khoperskov
// (2020): forces at t_n, predictor to t_{n+1/2}, forces at t_{n+1/2},
// corrector (K2..K6), Euler-stage fluxes by piecewise-linear reconstruction,
// TVD (minmod) limiting and HLL (K7), update (K8), with the bedload of
// Eqs. 2-5, the Exner update of Eq. 1 and the time step of Eq. 7.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csph {

constexpr int kWall = 0;
constexpr int kOpen = 1;

// Constants and per-run inputs passed by value to every kernel.
struct KPar {
    int nx, ny, pitch;      // pitch: floats per stored row (>= nx, multiple of 64)
    int bcW, bcE, bcS, bcN; // 0 wall, 1 open
    float dx, inv_dx;
    float g, eps, eps4;     // gravity, desingularisation depth and its 4th power
    float h_sed;            // no bedload at or below this depth
    float s_rel_m1;         // s - 1 of Eq. 4
    float C_J, C_Sh, A_G, m_exp;
    float half_g_inv_dx;    // g / (2 dx)
    int sed_law;            // 0 none, 1 Grass, 2 Eq. 4
    const float *nM;  float nM_s;   // Manning: per cell (pitched) or scalar
    const float *d50; float d50_s;  // grain size
    const float *psi; float psi_s;  // porosity
    const float *qb;                // q_b^+ - q_b^- per cell, or null
    const float *srcw;              // inflow weight / dx^2 per cell, or null
    float *rb;                      // bed residual per cell (null: the bed cannot change)
    // TVD limiter of the Euler stage as the bounds of its slope ratio (see
    // `limited`): minmod (1, 1, 1), MC (2, 2, 1/2), superbee (2, 2, 1)
    float lim_b, lim_t, lim_g;
    int speeds;                     // HLL wave speeds: 0 Davis, 1 two-rarefaction
    int variant;                    // 1 when the limiter or the speeds differ from minmod + Davis
    // forcing (sigma and f of Eq. 6)
    float rain;                     // rainfall rate, m/s, on every cell (mass only)
    const float *beta; float beta_s;  // absorption coefficient, 1/s: per cell or scalar
    double *ab;                     // absorbed depth per cell, FP64 (null: no absorption)
    float *rh;                      // depth residual of the compensated rainfall (null: no rain)
    float cor;                      // Coriolis parameter f_c, 1/s
    float wsx, wsy;                 // wind stress per unit density C_w |W| W, m^2/s^2
    float inv_hsed;                 // 1 / h_sed (the wind's depth ramp)
    int force;                      // 1 when the Coriolis or the wind term acts
    int force2;                     // 1: second-order Lagrangian force (strip kernels)
};

__device__ __forceinline__ float soil(const float *a, float s, int c) { return a ? a[c] : s; }

// Square root and quotient for the operands the step produces: x = 0 or
// x >= 2^-96, and divisors whose quotient needs no range scaling.  The
// hardware estimate (v_sqrt_f32 / v_rcp_f32, within 1 ulp) is corrected with
// exact fused residuals: for the square root, the neighbours s -/+ 1 ulp of
// the estimate s are taken when x - (s -/+ 1 ulp) s says the root lies past
// their midpoint with s; for the quotient, one Newton step refines the
// reciprocal and two residual steps q + r (a - b q) the quotient.  In this
// range both are the correctly rounded results (what sqrtf and a / b give),
// without the scaling and special-value handling that only operands outside
// it need.  (A numerator of -0 gives +0.)  The square root's correction is
// Tuckerman's rounding test; the quotient's, Markstein's Newton-Raphson
// refinement with a final residual correction.
__device__ __forceinline__ float nsqrt(float x)
{
    const float s = __builtin_amdgcn_sqrtf(x);
    const float lo = __int_as_float(__float_as_int(s) - 1);
    const float hi = __int_as_float(__float_as_int(s) + 1);
    const float r = fmaf(-lo, s, x) <= 0.0f ? lo : s;
    return fmaf(-hi, s, x) > 0.0f ? hi : r;
}

__device__ __forceinline__ float ndiv(float a, float b)
{
    float r = __builtin_amdgcn_rcpf(b);
    r = fmaf(fmaf(-b, r, 1.0f), r, r);
    float q = a * r;
    q = fmaf(fmaf(-b, q, a), r, q);
    return fmaf(fmaf(-b, q, a), r, q);
}

// a^2 + b^2 without fused multiply-add, so that swapping a and b (a grid and
// its transpose) gives the same bits.
__device__ __forceinline__ float sumsq(float a, float b)
{
#pragma clang fp contract(off)
    return a * a + b * b;
}

// Desingularised reciprocal depth (Kurganov & Petrova): 1/H for H >= eps,
// sqrt(2) H / sqrt(H^4 + eps^4) below, zero at H = 0.
__device__ __forceinline__ float wdes(float H, const KPar &P)
{
    if (H >= P.eps) return ndiv(1.0f, H);
    float H2 = H * H;
    return ndiv(1.41421356237f * H, nsqrt(H2 * H2 + P.eps4));
}

// minmod(a, b): 0 unless a and b share a sign, else the one nearer zero,
// i.e. min(|a|, |b|) with the sign of a.  Written without branches (one
// min with absolute-value operands, one sign insert, one select).
__device__ __forceinline__ float minmod(float a, float b)
{
    const float m = copysignf(fminf(fabsf(a), fabsf(b)), a);
    return a * b <= 0.0f ? 0.0f : m;
}

// The TVD limiter of the run, from the backward and forward differences a,
// b (V = false: minmod).  Zero unless a and b share a sign; else, with A =
// |a|, B = |b|, the sign of a and the magnitude
//   min( max(min(beta A, B), min(A, beta B)), theta min(A, B), gamma (A + B) ),
// which is min(A, B) for minmod (beta = theta = gamma = 1), min(2A, 2B,
// (A + B)/2) for MC (2, 2, 1/2) and max(min(2A, B), min(A, 2B)) for
// superbee (2, 2, 1): every min and max and the doublings are exact, so each
// is the limiter's own value, minmod bit for bit.
template <bool V>
__device__ __forceinline__ float limited(const KPar &P, float a, float b)
{
    if constexpr (!V) {
        return minmod(a, b);
    } else {
        const float A = fabsf(a), B = fabsf(b);
        float m = fmaxf(fminf(P.lim_b * A, B), fminf(A, P.lim_b * B));
        m = fminf(m, P.lim_t * fminf(A, B));
        m = fminf(m, P.lim_g * (A + B));
        return a * b <= 0.0f ? 0.0f : copysignf(m, a);
    }
}

// Powers through the hardware base-2 logarithm and exponential (v_log_f32,
// v_exp_f32, about 1 ulp): x^p = 2^(p log2 x) for x > 0.
__device__ __forceinline__ float powp(float x, float p)
{
    return __builtin_amdgcn_exp2f(p * __builtin_amdgcn_logf(x));
}

// x^(4/3) for x > 0.
__device__ __forceinline__ float pow43(float x) { return powp(x, 4.0f / 3.0f); }

// Manning friction rate g nM^2 |v| / max(H, eps)^(4/3) (semi-implicit).
__device__ __forceinline__ float friction_rate(const KPar &P, float nM, float speed, float H)
{
    float Hf = H > P.eps ? H : P.eps;
    return ndiv(P.g * nM * nM * speed, pow43(Hf));
}

// Zero-slope bedload J0 (Eqs. 3-5): zero at or below h_sed or at or below the
// Shamov critical speed C_Sh d50^(1/3) H^(1/6); else A |v|^m v.
__device__ __forceinline__ void bedload(const KPar &P, float H, float u, float v, float nM,
                                        float d50, float &jx, float &jy)
{
    jx = 0.0f;
    jy = 0.0f;
    if (P.sed_law == 0 || !(H > P.h_sed)) return;
    float speed = nsqrt(sumsq(u, v));
    float vk = P.C_Sh * powp(d50, 1.0f / 3.0f) * powp(H, 1.0f / 6.0f);
    if (!(speed > vk)) return;
    float f;
    if (P.sed_law == 1) {
        f = P.A_G * (P.m_exp == 2.0f ? speed * speed : powp(speed, P.m_exp));
    } else {
        float A = ndiv(0.05f * nM * nM * nM, P.s_rel_m1 * nsqrt(P.g * H) * d50);
        float s2 = speed * speed;
        f = A * (s2 * s2);
    }
    jx = f * u;
    jy = f * v;
}

// Exner update of Eq. 1 for one cell with the bedload divergence dJ (the sum
// of the four face-flux differences) and the bed source qb = q_b^+ - q_b^-,
// compensated: rb carries the part of the earlier updates the float32 bed
// could not hold (the stored bed is the nearest float to the accumulated bed
// b + rb), so bed changes smaller than half an ulp of the elevation add up
// instead of rounding away.  The rounding error of b + d is recovered exactly
// by Knuth's two-sum.
__device__ __forceinline__ float exner(const KPar &P, float dt, float b, float om, float dJ,
                                       float qb, float &rb)
{
    float d = -(dt / (om * P.dx)) * dJ;
    if (P.qb) d += dt * qb / om;
    d += rb;
    const float bn = b + d;
    const float bv = bn - b;
    rb = (b - (bn - bv)) + (d - bv);
    return bn;
}

// Hydrostatic-face force along one direction on cell C from its neighbours
// M (minus side) and Q (plus side), for a depth field Hd over bed b:
//   g/(2dx) [ HsL_+ (HsL_+ - HsR_+) - HsR_- (HsR_- - HsL_-) ],
// which is -(P_+ - P_-)/dx + g/(2dx) (HsL_+^2 - HsR_-^2) with face pressure
// P = g/2 HsL HsR, face bed max(b_L, b_R), side depth max(0, Hd + b - b_face).
// A missing neighbour (domain boundary) is a ghost copy of C.
__device__ __forceinline__ float face_force(const KPar &P, float HdM, float bM, float HdC,
                                            float bC, float HdQ, float bQ, bool hasM, bool hasQ)
{
    float HsLp, HsRp, HsLm, HsRm;
    if (hasQ) {
        float bf = fmaxf(bC, bQ);
        HsLp = fmaxf(0.0f, HdC + bC - bf);
        HsRp = fmaxf(0.0f, HdQ + bQ - bf);
    } else {
        HsLp = HsRp = fmaxf(0.0f, HdC + bC - bC);
    }
    if (hasM) {
        float bf = fmaxf(bM, bC);
        HsLm = fmaxf(0.0f, HdM + bM - bf);
        HsRm = fmaxf(0.0f, HdC + bC - bf);
    } else {
        HsLm = HsRm = fmaxf(0.0f, HdC + bC - bC);
    }
    return P.half_g_inv_dx * (HsLp * (HsLp - HsRp) - HsRm * (HsRm - HsLm));
}

// Second-order form of the same force (a reading; the paper names TVD
// reconstruction for the Euler stage only): the hydrostatic faces take side
// states reconstructed with the run's TVD limiter, from a cell's surface
// z = Hd + b, depth Hd and their limited slopes sz, sh along the direction
// (a boundary cell's slopes are zero): the plus side offers z + sz/2,
// Hd + sh/2, the minus side z - sz/2, Hd - sh/2, each with the bed side
// z_s - Hd_s; the face bed is the higher bed side.  Audusse et al. (2004)'s
// centred term for the bed slope inside the cell adds -g Hd sz / dx.  At rest
// (z constant where wet) every wet cell has sz = 0 and every face balances.
struct ReconQ {
    float z, h, sz, sh;
};
__device__ __forceinline__ float face_force2(const KPar &P, const ReconQ &M, const ReconQ &C,
                                             const ReconQ &Q, bool hasM, bool hasQ)
{
    float HsLp, HsRp, HsLm, HsRm;
    {
        const float zL = C.z + 0.5f * C.sz, hL = C.h + 0.5f * C.sh;
        const float zR = hasQ ? Q.z - 0.5f * Q.sz : zL, hR = hasQ ? Q.h - 0.5f * Q.sh : hL;
        const float bf = fmaxf(zL - hL, zR - hR);
        HsLp = fmaxf(0.0f, zL - bf);
        HsRp = fmaxf(0.0f, zR - bf);
    }
    {
        const float zR = C.z - 0.5f * C.sz, hR = C.h - 0.5f * C.sh;
        const float zL = hasM ? M.z + 0.5f * M.sz : zR, hL = hasM ? M.h + 0.5f * M.sh : hR;
        const float bf = fmaxf(zL - hL, zR - hR);
        HsLm = fmaxf(0.0f, zL - bf);
        HsRm = fmaxf(0.0f, zR - bf);
    }
    return P.half_g_inv_dx * ((HsLp * (HsLp - HsRp) - HsRm * (HsRm - HsLm)) - 2.0f * C.h * C.sz);
}

// Per-cell quantities the remap reconstructs along one direction:
// free surface z = H + b, depth H, normal transport velocity ut, normal and
// tangential Lagrangian velocities uLn, uLt.
struct CellQ {
    float z, h, ut, uLn, uLt;
};

// Direction-free per-cell remap inputs: surface, depth, transport velocity
// u~ = (v^n + u^L)/2 and Lagrangian velocity u^L = Q^L w(H), both components.
// A cell with zero depth has zero velocities: its Q^L is replaced by its
// (zero) momentum, so a Q^L buffer the Lagrangian stage skipped is never used.
struct CellVals {
    float z, h, utx, uty, uLx, uLy;
};

__device__ __forceinline__ CellVals cell_vals(const KPar &P, float H, float qx, float qy, float b,
                                              float QLx, float QLy)
{
    float w = wdes(H, P);
    float Lx = H > 0.0f ? QLx : qx;
    float Ly = H > 0.0f ? QLy : qy;
    float ux = qx * w, uy = qy * w;
    float uLx = Lx * w, uLy = Ly * w;
    CellVals v;
    v.z = H + b;
    v.h = H;
    v.utx = 0.5f * (ux + uLx);
    v.uty = 0.5f * (uy + uLy);
    v.uLx = uLx;
    v.uLy = uLy;
    return v;
}

// The same cell seen along x (dir 0) or y (dir 1).
__device__ __forceinline__ CellQ along(const CellVals &v, int dir)
{
    CellQ q;
    q.z = v.z;
    q.h = v.h;
    if (dir == 0) {
        q.ut = v.utx; q.uLn = v.uLx; q.uLt = v.uLy;
    } else {
        q.ut = v.uty; q.uLn = v.uLy; q.uLt = v.uLx;
    }
    return q;
}

// Ghost cell beyond a boundary normal to `dir`: a wall mirrors the normal
// velocity components, an open side copies.
__device__ __forceinline__ CellVals mirror(CellVals v, int dir, bool wall)
{
    if (wall) {
        if (dir == 0) { v.utx = -v.utx; v.uLx = -v.uLx; }
        else { v.uty = -v.uty; v.uLy = -v.uLy; }
    }
    return v;
}

__device__ __forceinline__ CellQ ghost_of(CellQ c, bool wall)
{
    if (wall) {
        c.ut = -c.ut;
        c.uLn = -c.uLn;
    }
    return c;
}

struct FaceState {
    float Hs, uLn, uLt, ut;
};

// Reconstructed face states on both sides of the face between cells L and R,
// given the outer neighbours A (beyond L) and B (beyond R): minmod slopes,
// side values L + slope/2 and R - slope/2, hydrostatic face depths.
__device__ __forceinline__ void face_states(const KPar &P, const CellQ &A, const CellQ &L,
                                            const CellQ &R, const CellQ &B, FaceState &fl,
                                            FaceState &fr)
{
    float zL = L.z + 0.5f * limited<true>(P, L.z - A.z, R.z - L.z);
    float hL = L.h + 0.5f * limited<true>(P, L.h - A.h, R.h - L.h);
    float tL = L.ut + 0.5f * limited<true>(P, L.ut - A.ut, R.ut - L.ut);
    float nL = L.uLn + 0.5f * limited<true>(P, L.uLn - A.uLn, R.uLn - L.uLn);
    float sL = L.uLt + 0.5f * limited<true>(P, L.uLt - A.uLt, R.uLt - L.uLt);
    float zR = R.z - 0.5f * limited<true>(P, R.z - L.z, B.z - R.z);
    float hR = R.h - 0.5f * limited<true>(P, R.h - L.h, B.h - R.h);
    float tR = R.ut - 0.5f * limited<true>(P, R.ut - L.ut, B.ut - R.ut);
    float nR = R.uLn - 0.5f * limited<true>(P, R.uLn - L.uLn, B.uLn - R.uLn);
    float sR = R.uLt - 0.5f * limited<true>(P, R.uLt - L.uLt, B.uLt - R.uLt);
    float bL = zL - hL, bR = zR - hR;
    float bf = fmaxf(bL, bR);
    fl.Hs = fmaxf(0.0f, zL - bf);
    fr.Hs = fmaxf(0.0f, zR - bf);
    fl.uLn = nL; fl.uLt = sL; fl.ut = tL;
    fr.uLn = nR; fr.uLt = sR; fr.ut = tR;
}

// One-sided face state of a boundary cell: its neighbour inside (A) and its
// ghost outside (G); side = +1 for the E/N face, -1 for the W/S face.
__device__ __forceinline__ FaceState boundary_state(const KPar &P, const CellQ &A,
                                                    const CellQ &C, const CellQ &G, float side)
{
    // slope of C from its two neighbours in increasing coordinate order
    const CellQ &lo = side > 0.0f ? A : G;
    const CellQ &hi = side > 0.0f ? G : A;
    float z = C.z + side * 0.5f * limited<true>(P, C.z - lo.z, hi.z - C.z);
    float h = C.h + side * 0.5f * limited<true>(P, C.h - lo.h, hi.h - C.h);
    FaceState s;
    s.ut = C.ut + side * 0.5f * limited<true>(P, C.ut - lo.ut, hi.ut - C.ut);
    s.uLn = C.uLn + side * 0.5f * limited<true>(P, C.uLn - lo.uLn, hi.uLn - C.uLn);
    s.uLt = C.uLt + side * 0.5f * limited<true>(P, C.uLt - lo.uLt, hi.uLt - C.uLt);
    float bb = z - h;
    s.Hs = fmaxf(0.0f, z - bb);
    return s;
}

// HLL flux of the remap: U = (Hs, Hs uLn, Hs uLt), F = ut U.  Wave speeds:
// Davis, SL = min(uL - cL, uR - cR), SR = max(uL + cL, uR + cR); or (V and
// P.speeds = 1) the two-rarefaction estimate SL = min(uL - cL, u* - c*),
// SR = max(uR + cR, u* + c*) with u* = (uL + uR)/2 + cL - cR and
// c* = max(0, (cL + cR)/2 + (uL - uR)/4) (Toro).
template <bool V>
__device__ __forceinline__ void hll(const KPar &P, const FaceState &l, const FaceState &r,
                                    float &fH, float &fn, float &ft)
{
    const float g = P.g;
    float UL0 = l.Hs, UL1 = l.Hs * l.uLn, UL2 = l.Hs * l.uLt;
    float UR0 = r.Hs, UR1 = r.Hs * r.uLn, UR2 = r.Hs * r.uLt;
    float FL0 = l.ut * UL0, FL1 = l.ut * UL1, FL2 = l.ut * UL2;
    float FR0 = r.ut * UR0, FR1 = r.ut * UR1, FR2 = r.ut * UR2;
    float cL = nsqrt(g * l.Hs), cR = nsqrt(g * r.Hs);
    float SL = fminf(l.ut - cL, r.ut - cR);
    float SR = fmaxf(l.ut + cL, r.ut + cR);
    if (V && P.speeds == 1) {
        const float us = 0.5f * (l.ut + r.ut) + cL - cR;
        const float cs = fmaxf(0.0f, 0.5f * (cL + cR) + 0.25f * (l.ut - r.ut));
        SL = fminf(l.ut - cL, us - cs);
        SR = fmaxf(r.ut + cR, us + cs);
    }
    // the four cases are selected, not branched: every lane evaluates the
    // HLL average and keeps the upwind flux when both speeds share a sign
    const bool left = SL >= 0.0f, right = SR <= 0.0f, fan = SR - SL > 0.0f;
    const float inv = fan ? ndiv(1.0f, SR - SL) : 0.0f;
    const float SLR = SL * SR;
    const float hH = (SR * FL0 - SL * FR0 + SLR * (UR0 - UL0)) * inv;
    const float hn = (SR * FL1 - SL * FR1 + SLR * (UR1 - UL1)) * inv;
    const float ht = (SR * FL2 - SL * FR2 + SLR * (UR2 - UL2)) * inv;
    fH = left ? FL0 : (right ? FR0 : hH);
    fn = left ? FL1 : (right ? FR1 : hn);
    ft = left ? FL2 : (right ? FR2 : ht);
}

// Wall face fluxes (HLL against the mirrored ghost): no mass, no tangential
// momentum; normal momentum Hs uLn (ut + side S), side = +1 for the interior
// cell on the minus side (E/N wall), -1 on the plus side (W/S wall).  The
// mirrored pair has symmetric speeds -S, S: Davis S = |ut| + c; the
// two-rarefaction estimate S = max(c - side ut, max(0, c + side ut / 2)).
template <bool V>
__device__ __forceinline__ float wall_flux_n(const KPar &P, const FaceState &s, float side)
{
    float c = nsqrt(P.g * s.Hs);
    float S = fabsf(s.ut) + c;
    if (V && P.speeds == 1) S = fmaxf(c - side * s.ut, fmaxf(0.0f, c + side * 0.5f * s.ut));
    return s.Hs * s.uLn * (s.ut + side * S);
}

// Bedload face flux: donor split of J0 plus the slope term of Eq. 2 with the
// mean |J0| of the two cells.
__device__ __forceinline__ float bed_face_flux(const KPar &P, float JnL, float JmagL, float bL,
                                               float JnR, float JmagR, float bR)
{
    float mag = 0.5f * (JmagL + JmagR);
    return fmaxf(JnL, 0.0f) + fminf(JnR, 0.0f) - P.C_J * mag * (bR - bL) * P.inv_dx;
}

// Raw water fluxes (mass, normal momentum, tangential momentum) of face k
// along one direction, k in [0, n] (face k lies between cells k-1 and k),
// from cells c0..c3 = k-2..k+1 (ghost cells at -1 and n).  Interior faces:
// reconstruction + HLL.  Boundary faces: the wall flux against the mirrored
// ghost, or the physical flux of the interior face state on an open side.
__device__ __forceinline__ void water_flux(const KPar &P, int k, int n, bool wallLo, bool wallHi,
                                           const CellQ &c0, const CellQ &c1, const CellQ &c2,
                                           const CellQ &c3, float &fH, float &fn, float &ft)
{
    fH = fn = ft = 0.0f;
    if (k > 0 && k < n) {
        FaceState fl, fr;
        face_states(P, c0, c1, c2, c3, fl, fr);
        hll<true>(P, fl, fr, fH, fn, ft);
    } else if (k == n) {  // high boundary: interior cell c1, its inner neighbour c0, ghost c2
        FaceState s = boundary_state(P, c0, c1, c2, 1.0f);
        if (wallHi) {
            fn = wall_flux_n<true>(P, s, 1.0f);
        } else {
            fH = s.ut * s.Hs;
            fn = s.ut * s.Hs * s.uLn;
            ft = s.ut * s.Hs * s.uLt;
        }
    } else {  // k == 0: interior cell c2, its inner neighbour c3, ghost c1
        FaceState s = boundary_state(P, c3, c2, c1, -1.0f);
        if (wallLo) {
            fn = wall_flux_n<true>(P, s, -1.0f);
        } else {
            fH = s.ut * s.Hs;
            fn = s.ut * s.Hs * s.uLn;
            ft = s.ut * s.Hs * s.uLt;
        }
    }
}

// Reconstructed values of one cell on its two faces along a direction: the
// limited slope of each quantity from the neighbours M (minus side) and Q
// (plus side), value -/+ slope/2, and the bed under each face value.  The
// face between cells k-1 and k takes the plus side of k-1 and the minus side
// of k; this gives the bits of face_states / boundary_state (same slopes,
// same contractions), with each slope computed once per cell.
struct SideQ {
    float z, h, ut, uLn, uLt, b;
};

template <bool V>
__device__ __forceinline__ void reconstruct(const KPar &P, const CellQ &M, const CellQ &C,
                                            const CellQ &Q, SideQ &minus, SideQ &plus)
{
    const float sz = limited<V>(P, C.z - M.z, Q.z - C.z);
    const float sh = limited<V>(P, C.h - M.h, Q.h - C.h);
    const float st = limited<V>(P, C.ut - M.ut, Q.ut - C.ut);
    const float sn = limited<V>(P, C.uLn - M.uLn, Q.uLn - C.uLn);
    const float ss = limited<V>(P, C.uLt - M.uLt, Q.uLt - C.uLt);
    plus.z = C.z + 0.5f * sz;
    plus.h = C.h + 0.5f * sh;
    plus.ut = C.ut + 0.5f * st;
    plus.uLn = C.uLn + 0.5f * sn;
    plus.uLt = C.uLt + 0.5f * ss;
    minus.z = C.z - 0.5f * sz;
    minus.h = C.h - 0.5f * sh;
    minus.ut = C.ut - 0.5f * st;
    minus.uLn = C.uLn - 0.5f * sn;
    minus.uLt = C.uLt - 0.5f * ss;
    plus.b = plus.z - plus.h;
    minus.b = minus.z - minus.h;
}

// Raw water fluxes of face k in [0, n] from the plus side L of cell k-1 and
// the minus side R of cell k (the result of water_flux): interior faces take
// hydrostatic face depths and HLL; a boundary face uses the interior cell's
// side only (wall flux, or the physical flux on an open side).
template <bool V>
__device__ __forceinline__ void side_flux(const KPar &P, int k, int n, bool wallLo, bool wallHi,
                                          const SideQ &L, const SideQ &R, float &fH, float &fn,
                                          float &ft)
{
    // the interior flux is evaluated in every lane (no branch around it); a
    // lane whose face is a boundary face replaces it below
    const float bf = fmaxf(L.b, R.b);
    FaceState fl, fr;
    fl.Hs = fmaxf(0.0f, L.z - bf); fl.uLn = L.uLn; fl.uLt = L.uLt; fl.ut = L.ut;
    fr.Hs = fmaxf(0.0f, R.z - bf); fr.uLn = R.uLn; fr.uLt = R.uLt; fr.ut = R.ut;
    hll<V>(P, fl, fr, fH, fn, ft);
    if (k > 0 && k < n) return;
    fH = fn = ft = 0.0f;
    const SideQ &C = k == n ? L : R;
    const float side = k == n ? 1.0f : -1.0f;
    FaceState s;
    s.Hs = fmaxf(0.0f, C.z - C.b); s.uLn = C.uLn; s.uLt = C.uLt; s.ut = C.ut;
    if (k == n ? wallHi : wallLo) {
        fn = wall_flux_n<V>(P, s, side);
    } else {
        fH = s.ut * s.Hs;
        fn = s.ut * s.Hs * s.uLn;
        ft = s.ut * s.Hs * s.uLt;
    }
}

// Bedload flux of face k (between cells k-1 and k, k in [0, n]) from the
// normal J0 components, the |J0| and the beds of the cells on its two sides;
// walls pass nothing, an open side passes only the outward part of the
// interior cell's J0.
__device__ __forceinline__ float sed_face(const KPar &P, int k, int n, bool wallLo, bool wallHi,
                                          float JnL, float magL, float bL, float JnR, float magR,
                                          float bR)
{
    // all three forms are evaluated and the face's own is selected (no branches)
    const float inner = bed_face_flux(P, JnL, magL, bL, JnR, magR, bR);
    const float hi = wallHi ? 0.0f : fmaxf(JnL, 0.0f);
    const float lo = wallLo ? 0.0f : fminf(JnR, 0.0f);
    return (k > 0 && k < n) ? inner : (k == n ? hi : lo);
}

// The same from the J0 vectors of the two side cells, along direction dir.
__device__ __forceinline__ float sed_flux(const KPar &P, int k, int n, bool wallLo, bool wallHi,
                                          int dir, float jxL, float jyL, float bL, float jxR,
                                          float jyR, float bR)
{
    return sed_face(P, k, n, wallLo, wallHi, dir == 0 ? jxL : jyL, nsqrt(sumsq(jxL, jyL)), bL,
                    dir == 0 ? jxR : jyR, nsqrt(sumsq(jxR, jyR)), bR);
}

}  // namespace csph
