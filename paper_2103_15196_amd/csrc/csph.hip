// csph.hip -- HIP (gfx950) kernels and C ABI of the CSPH-TVD shallow-water +
// Exner solver (Khrapov & Khoperskov 2020, Section 3 kernels K1..K8).
//
// Layout in HBM: structure of arrays, one float32 plane per field (h, hu, hv,
// b; Lagrangian momentum QLx, QLy; optional per-cell soil), rows padded to a
// multiple of 64 floats so that every wavefront row load is one aligned
// 256-byte line.  The state is double-buffered: step k reads buffer k&1 and
// writes buffer (k+1)&1.  Global reductions (Eq. 7 maxima, volumes, boundary
// balances) run in FP64 or as exact FP32 maxima; see the kernels below.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "csph.h"
#include "csph_device.h"

using namespace csph;

namespace {

constexpr int BX = 64;  // threads per block along x (one wavefront row)
constexpr int BY = 4;   // rows per block in the one-cell-per-thread kernels
constexpr int NSLOT = 16;  // spread of the per-step maxima over atomic slots

// Device control block: per-step maxima slots, time ring, balances, error.
struct Ctrl {
    unsigned slot[2][NSLOT][4];  // float bits of max |v|, max |v|+c, max |J0|/(1-psi); [3]: nonfinite
    double t[2];                 // model time at the start of step k (ring k&1)
    double dt[2];                // step size of step k
    double qmid[2];              // inflow discharge at t_k + dt_k/2
    double in_w, in_s;           // accumulated source volumes
    double in_rain;              // accumulated rainfall volume
    double vp, vs, D;            // Eq. 7 maxima at the start of the last step
    double last_dt;
    int err, err_k, binding, kdev;  // kdev: steps taken since the state was set
    unsigned long long work[2];     // cells processed by the Lagrangian / Euler stage
};

// One step's record in the step log (the layout of sw_step_record).
struct StepRec {
    long long step;              // steps since the state was set (the host adds its step0)
    double t, dt, vp, vs, D, q;
    int binding, reserved;
};
constexpr int kStepLog = SW_STEP_LOG;  // records in the ring (a power of two)
static_assert((kStepLog & (kStepLog - 1)) == 0, "the step log ring is a power of two");

struct StepArgs {
    int mode_fixed;              // 1: fixed dt
    double dt_fixed;
    double dx, cfl, dt_max, dt_min;
    int has_inflow;
    double q_base, q_peak, t_peak, t_sigma;
    double qb_total;             // sum over cells of (q_b^+ - q_b^-) dx^2
    double rain_area;            // rainfall rate x grid area, m^3/s
    StepRec *log;                // step log ring (kStepLog records), or null
};

// The step's record into the log ring (the thread that publishes the step).
__device__ __forceinline__ void log_step(const StepArgs &A, int kd, double tn, double dt,
                                         double vp, double vs, double D, double q, int which)
{
    if (!A.log) return;
    StepRec &r = A.log[kd & (kStepLog - 1)];
    r.step = kd; r.t = tn; r.dt = dt; r.vp = vp; r.vs = vs; r.D = D; r.q = q;
    r.binding = which; r.reserved = 0;
}

__device__ __forceinline__ unsigned fbits_nonneg(float x) { return __float_as_uint(x + 0.0f); }

// Wave64 + block max of three non-negative floats (as bits) and a flag,
// then one atomicMax per value into this block's slot.
__device__ __forceinline__ void block_maxima(unsigned a, unsigned b, unsigned c, unsigned bad,
                                             unsigned (*slot)[4], int sidx)
{
    __shared__ unsigned red[4][16];
    for (int off = 32; off > 0; off >>= 1) {
        a = max(a, (unsigned)__shfl_xor((int)a, off));
        b = max(b, (unsigned)__shfl_xor((int)b, off));
        c = max(c, (unsigned)__shfl_xor((int)c, off));
        bad = max(bad, (unsigned)__shfl_xor((int)bad, off));
    }
    int tid = threadIdx.x + threadIdx.y * blockDim.x;
    int nw = (blockDim.x * blockDim.y + 63) >> 6;
    int wv = tid >> 6;
    if ((tid & 63) == 0) {
        red[0][wv] = a; red[1][wv] = b; red[2][wv] = c; red[3][wv] = bad;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < nw; ++w) {
            a = max(a, red[0][w]); b = max(b, red[1][w]); c = max(c, red[2][w]);
            bad = max(bad, red[3][w]);
        }
        int s = sidx % NSLOT;
        if (a) atomicMax(&slot[s][0], a);
        if (b) atomicMax(&slot[s][1], b);
        if (c) atomicMax(&slot[s][2], c);
        if (bad) atomicMax(&slot[s][3], bad);
    }
}

// Eq. 7 maxima contributions of one cell of a state with Manning coefficient
// nM, grain size d50 and porosity psi; jx, jy, jm receive the cell's J0 and
// |J0| (the values the next Euler stage uses).
__device__ __forceinline__ void cell_maxima_j(const KPar &P, float H, float qx, float qy, float b,
                                              float nM, float d50, float psi, unsigned &mv,
                                              unsigned &ms, unsigned &mD, unsigned &bad, float &jx,
                                              float &jy, float &jm)
{
    float w = wdes(H, P);
    float u = qx * w, v = qy * w;
    float sp = nsqrt(sumsq(u, v));
    float cs = nsqrt(P.g * (H > 0.0f ? H : 0.0f));
    bedload(P, H, u, v, nM, d50, jx, jy);
    jm = nsqrt(sumsq(jx, jy));
    float Dc = ndiv(jm, 1.0f - psi);
    bool fin = isfinite(H) && isfinite(qx) && isfinite(qy) && isfinite(b) && isfinite(sp) &&
               isfinite(Dc);
    if (!fin) {
        bad = 1u;
        return;
    }
    mv = max(mv, fbits_nonneg(sp));
    ms = max(ms, fbits_nonneg(sp + cs));
    mD = max(mD, fbits_nonneg(Dc));
}

__device__ __forceinline__ void cell_maxima_s(const KPar &P, float H, float qx, float qy, float b,
                                              float nM, float d50, float psi, unsigned &mv,
                                              unsigned &ms, unsigned &mD, unsigned &bad)
{
    float jx, jy, jm;
    cell_maxima_j(P, H, qx, qy, b, nM, d50, psi, mv, ms, mD, bad, jx, jy, jm);
}

// The same for cell c of the grid (soil read from its per-cell planes or scalars).
__device__ __forceinline__ void cell_maxima(const KPar &P, float H, float qx, float qy, float b,
                                            int c, unsigned &mv, unsigned &ms, unsigned &mD,
                                            unsigned &bad)
{
    cell_maxima_s(P, H, qx, qy, b, soil(P.nM, P.nM_s, c), soil(P.d50, P.d50_s, c),
                  soil(P.psi, P.psi_s, c), mv, ms, mD, bad);
}

// Maxima of the initial (or externally modified) state into slot ring k&1.
__global__ void k_prepare(KPar P, Ctrl *ctrl, int k, const float *__restrict__ H,
                          const float *__restrict__ qx, const float *__restrict__ qy,
                          const float *__restrict__ b)
{
    int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    unsigned mv = 0, ms = 0, mD = 0, bad = 0;
    if (i < P.nx && j < P.ny) {
        int c = j * P.pitch + i;
        cell_maxima(P, H[c], qx[c], qy[c], b[c], c, mv, ms, mD, bad);
    }
    block_maxima(mv, ms, mD, bad, ctrl->slot[k & 1], blockIdx.x + blockIdx.y * gridDim.x);
}

// Maxima of the current fields into the given slots (sw_step_bound): the
// arithmetic of the set-up pass, without touching the step's own slots.
__global__ void k_bound(KPar P, unsigned (*slot)[4], const float *__restrict__ H,
                        const float *__restrict__ qx, const float *__restrict__ qy,
                        const float *__restrict__ b)
{
    int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    unsigned mv = 0, ms = 0, mD = 0, bad = 0;
    if (i < P.nx && j < P.ny) {
        int c = j * P.pitch + i;
        cell_maxima(P, H[c], qx[c], qy[c], b[c], c, mv, ms, mD, bad);
    }
    block_maxima(mv, ms, mD, bad, slot, blockIdx.x + blockIdx.y * gridDim.x);
}

// K3: time step of Eq. 7 from the maxima of step k's state; clears the slots
// that step k's update fills for step k+1; advances the time ring.
__global__ void k_dt(Ctrl *ctrl, int k, StepArgs A)
{
    int t = threadIdx.x;
    const int kd = ctrl->kdev;
    unsigned(*cur)[4] = ctrl->slot[k & 1];
    unsigned(*nxt)[4] = ctrl->slot[(k + 1) & 1];
    unsigned a = 0, b = 0, c = 0, bad = 0;
    if (t < NSLOT) {
        a = cur[t][0]; b = cur[t][1]; c = cur[t][2]; bad = cur[t][3];
    }
    for (int off = 32; off > 0; off >>= 1) {
        a = max(a, (unsigned)__shfl_xor((int)a, off));
        b = max(b, (unsigned)__shfl_xor((int)b, off));
        c = max(c, (unsigned)__shfl_xor((int)c, off));
        bad = max(bad, (unsigned)__shfl_xor((int)bad, off));
    }
    if (ctrl->err) return;
    if (t < NSLOT) {
        nxt[t][0] = 0u; nxt[t][1] = 0u; nxt[t][2] = 0u; nxt[t][3] = 0u;
    }
    if (t != 0) return;
    double vp = __uint_as_float(a), vs = __uint_as_float(b), D = __uint_as_float(c);
    ctrl->vp = vp; ctrl->vs = vs; ctrl->D = D;
    if (bad) {
        ctrl->err = SW_ERR_NONFINITE;
        ctrl->err_k = kd;
        return;
    }
    double h = A.dx;
    double t0 = vp > 0.0 ? h / (2.0 * vp) : INFINITY;
    double t1 = vs > 0.0 ? h / vs : INFINITY;
    double t2 = D > 0.0 ? h * h / (2.0 * D) : INFINITY;
    double m = t0;
    int which = 0;
    if (t1 < m) { m = t1; which = 1; }
    if (t2 < m) { m = t2; which = 2; }
    double dt = A.cfl * m;
    if (!(dt < A.dt_max)) { dt = A.dt_max; which = 3; }
    if (A.mode_fixed) {
        if (A.dt_fixed > dt) {
            ctrl->err = SW_ERR_CFL;
            ctrl->err_k = kd;
            return;
        }
        dt = A.dt_fixed;
        which = 4;
    }
    if (dt < A.dt_min) {
        ctrl->err = SW_ERR_DT_UNDERFLOW;
        ctrl->err_k = kd;
        return;
    }
    double tn = ctrl->t[k & 1];
    double q = 0.0;
    if (A.has_inflow) {
        double d = tn + 0.5 * dt - A.t_peak;
        double pk = A.t_sigma > 0.0 ? A.q_peak * exp(-d * d / (2.0 * A.t_sigma * A.t_sigma)) : 0.0;
        q = A.q_base + pk;
        ctrl->in_w += dt * q;
    }
    ctrl->in_s += dt * A.qb_total;
    ctrl->in_rain += dt * A.rain_area;
    ctrl->qmid[k & 1] = q;
    ctrl->dt[k & 1] = dt;
    ctrl->t[(k + 1) & 1] = tn + dt;
    ctrl->last_dt = dt;
    ctrl->binding = which;
    ctrl->kdev = kd + 1;
    log_step(A, kd, tn, dt, vp, vs, D, q, which);
}

// ---------------------------------------------------------------------------
// Lagrangian stage (K2, K4, K5, K6), one thread per cell.
// ---------------------------------------------------------------------------

struct StateView {
    const float *__restrict__ H, *__restrict__ qx, *__restrict__ qy, *__restrict__ b;
};

__device__ __forceinline__ void vel(const KPar &P, const StateView &S, int c, float &u, float &v)
{
    float w = wdes(S.H[c], P);
    u = S.qx[c] * w;
    v = S.qy[c] * w;
}

// Half-step depth of cell (i, j): H / J with J the area ratio of the column
// after dt/2 under the face-mean velocities at t_n (wall face: 0, open face:
// the cell's own velocity).
__device__ float half_depth(const KPar &P, const StateView &S, int i, int j, float hdt_dx)
{
    int c = j * P.pitch + i;
    float uc, vc;
    vel(P, S, c, uc, vc);
    float ue, uw, vn, vs, t0, t1;
    if (i + 1 < P.nx) { vel(P, S, c + 1, t0, t1); ue = 0.5f * (uc + t0); }
    else ue = (P.bcE == kWall) ? 0.0f : uc;
    if (i > 0) { vel(P, S, c - 1, t0, t1); uw = 0.5f * (t0 + uc); }
    else uw = (P.bcW == kWall) ? 0.0f : uc;
    if (j + 1 < P.ny) { vel(P, S, c + P.pitch, t0, t1); vn = 0.5f * (vc + t1); }
    else vn = (P.bcN == kWall) ? 0.0f : vc;
    if (j > 0) { vel(P, S, c - P.pitch, t0, t1); vs = 0.5f * (t1 + vc); }
    else vs = (P.bcS == kWall) ? 0.0f : vc;
    float Jx = 1.0f + hdt_dx * (ue - uw);
    float Jy = 1.0f + hdt_dx * (vn - vs);
    return ndiv(S.H[c], Jx * Jy);
}


// ---------------------------------------------------------------------------
// Euler stage, unfused: K7 raw face fluxes, then K8 limiter + update.
// ---------------------------------------------------------------------------

struct LagView {
    const float *__restrict__ QLx, *__restrict__ QLy;
};

// Cell quantities along x (dir 0) or y (dir 1) for the remap.
__device__ __forceinline__ CellQ cell_q(const KPar &P, const StateView &S, const LagView &L, int c,
                                        int dir)
{
    return along(cell_vals(P, S.H[c], S.qx[c], S.qy[c], S.b[c], L.QLx[c], L.QLy[c]), dir);
}

__device__ __forceinline__ void cell_j0(const KPar &P, const StateView &S, int c, float &jx,
                                        float &jy)
{
    float H = S.H[c];
    float w = wdes(H, P);
    bedload(P, H, S.qx[c] * w, S.qy[c] * w, soil(P.nM, P.nM_s, c), soil(P.d50, P.d50_s, c), jx, jy);
}

struct FaceView {
    float *__restrict__ xH, *__restrict__ xn, *__restrict__ xt, *__restrict__ xJ;  // [ny][nx+1]
    float *__restrict__ yH, *__restrict__ yn, *__restrict__ yt, *__restrict__ yJ;  // [ny+1][nx]
};

// Raw flux of x-face k in row j (between cells k-1 and k) or y-face k in
// column i (between cells k-1 and k along y).
__device__ void raw_face(const KPar &P, const StateView &S, const LagView &L, int dir, int k,
                         int line, float &fH, float &fn, float &ft, float &fJ)
{
    const int n = dir == 0 ? P.nx : P.ny;
    const int stride = dir == 0 ? 1 : P.pitch;
    const int base = dir == 0 ? line * P.pitch : line;
    const bool wallLo = (dir == 0 ? P.bcW : P.bcS) == kWall;
    const bool wallHi = (dir == 0 ? P.bcE : P.bcN) == kWall;
    auto q = [&](int m) -> CellQ {
        if (m < 0) return ghost_of(cell_q(P, S, L, base, dir), wallLo);
        if (m >= n) return ghost_of(cell_q(P, S, L, base + (n - 1) * stride, dir), wallHi);
        return cell_q(P, S, L, base + m * stride, dir);
    };
    water_flux(P, k, n, wallLo, wallHi, q(k - 2), q(k - 1), q(k), q(k + 1), fH, fn, ft);
    float jxL = 0.0f, jyL = 0.0f, bL = 0.0f, jxR = 0.0f, jyR = 0.0f, bR = 0.0f;
    if (k > 0) {
        int cL = base + (k - 1) * stride;
        cell_j0(P, S, cL, jxL, jyL);
        bL = S.b[cL];
    }
    if (k < n) {
        int cR = base + k * stride;
        cell_j0(P, S, cR, jxR, jyR);
        bR = S.b[cR];
    }
    fJ = sed_flux(P, k, n, wallLo, wallHi, dir, jxL, jyL, bL, jxR, jyR, bR);
}

__global__ void __launch_bounds__(BX * BY) k_faces(KPar P, const Ctrl *__restrict__ ctrl, StateView S,
                                                   LagView L, FaceView F)
{
    if (ctrl->err) return;
    int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (j < P.ny && i <= P.nx) {
        float fH, fn, ft, fJ;
        raw_face(P, S, L, 0, i, j, fH, fn, ft, fJ);
        int f = j * (P.nx + 1) + i;
        F.xH[f] = fH; F.xn[f] = fn; F.xt[f] = ft; F.xJ[f] = fJ;
    }
    if (i < P.nx && j <= P.ny) {
        float fH, fn, ft, fJ;
        raw_face(P, S, L, 1, j, i, fH, fn, ft, fJ);
        int f = j * P.nx + i;
        F.yH[f] = fH; F.yn[f] = fn; F.yt[f] = ft; F.yJ[f] = fJ;
    }
}

struct OutView {
    float *__restrict__ H, *__restrict__ qx, *__restrict__ qy, *__restrict__ b;
};

// Draining limiter of cell (i, j): theta = min(1, H dx / (dt * outflow)).
__device__ __forceinline__ float theta_of(const KPar &P, const StateView &S, const FaceView &F,
                                          int i, int j, float dt)
{
    if (i < 0 || j < 0 || i >= P.nx || j >= P.ny) return 1.0f;  // ghost donor
    float fe = F.xH[j * (P.nx + 1) + i + 1], fw = F.xH[j * (P.nx + 1) + i];
    float gn = F.yH[(j + 1) * P.nx + i], gs = F.yH[j * P.nx + i];
    float out = (fmaxf(0.0f, fe) + fmaxf(0.0f, -fw)) + (fmaxf(0.0f, gn) + fmaxf(0.0f, -gs));
    return out > 0.0f ? fminf(1.0f, S.H[j * P.pitch + i] * P.dx / (dt * out)) : 1.0f;
}



// ---------------------------------------------------------------------------
// Tiled path: one 256-thread workgroup per TX x TY tile of cells, LDS halo
// tiles, and the hierarchical grid system of Section 3 (HGS): a dry tile skips
// the Lagrangian stage; a tile whose own and four neighbour tiles are all dry
// skips the Euler stage.  A tile is dry when every cell has h = 0 and it holds
// no inflow or bed-source cell; such a tile provably stays unchanged, so the
// skip is exact.  The arithmetic per cell and per face is the one of the
// unfused kernels above (same device functions, same order), so every tile
// shape gives the same bits.  The tile functions serve a single grid (tile =
// block index) and an ensemble (tile = entry of a table over all members).
// ---------------------------------------------------------------------------

constexpr int NT = 256;

// Everything a tile of one grid needs: constants, Eq. 7 inputs, buffers, flags.
struct Inst {
    KPar P;
    StepArgs A;
    Ctrl *ctrl;
    float *H[2], *qx[2], *qy[2], *b[2];
    float *QLx, *QLy;
    float *jx[2], *jy[2], *jm[2];  // J0 and |J0| of each buffer level's state (strip kernels)
    double *bnd;
    uint8_t *act[2];
    uint8_t *synced;
    const uint8_t *force;
    uint4 *tmax[2];  // per tile: Eq. 7 maxima of the state the tile will step from (float bits) + nonfinite flag
    int ntx, nty, hgs;
    // work lists of one step (strip shapes, single grid), built by K3 in
    // nchunk segments of up to `chunk` tiles: segment b of a list sits at
    // entries [b chunk, b chunk + count) and starts at position pre[b] of the
    // whole list; totals[0] / totals[1] are the Lagrangian / Euler lengths.
    // An Euler entry -1-t asks for a buffer copy of dry tile t.
    int *totals;                 // list lengths
    int *cnt_l, *cnt_e;          // per-segment lengths
    int *pre_l, *pre_e;          // per-segment start positions (nchunk + 1)
    uint4 *part;                 // per-segment Eq. 7 maxima
    int *lag, *eul;              // the segments
    int nchunk, chunk;
};

// Block maxima of three non-negative floats (as bits) and a flag, stored with
// one plain 16-byte write for the tile (no atomics: per-tile slots).
__device__ __forceinline__ void block_maxima_store(unsigned a, unsigned b, unsigned c, unsigned bad,
                                                   uint4 *out)
{
    __shared__ unsigned red[4][NT / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a = max(a, (unsigned)__shfl_xor((int)a, off));
        b = max(b, (unsigned)__shfl_xor((int)b, off));
        c = max(c, (unsigned)__shfl_xor((int)c, off));
        bad = max(bad, (unsigned)__shfl_xor((int)bad, off));
    }
    const int tid = threadIdx.x, wv = tid >> 6;
    if ((tid & 63) == 0) {
        red[0][wv] = a; red[1][wv] = b; red[2][wv] = c; red[3][wv] = bad;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < NT / 64; ++w) {
            a = max(a, red[0][w]); b = max(b, red[1][w]); c = max(c, red[2][w]);
            bad = max(bad, red[3][w]);
        }
        *out = make_uint4(a, b, c, bad);
    }
}

// K3: the Eq. 7 step of one grid from its per-tile maxima (one 1024-thread
// block; the maximum does not depend on the order it is taken in).  Publishes
// dt, the time ring, the source balances and the step counter, or the error.
constexpr int RT = 1024;

// Block-wide maxima of the per-tile slots [t0, t1) (the result is valid in
// thread 0), with eight independent loads in flight per thread.
__device__ uint4 block_tile_maxima(const uint4 *__restrict__ tm, int t0, int t1)
{
    __shared__ unsigned red[4][RT / 64];
    const int tid = threadIdx.x;
    unsigned a = 0, b = 0, c = 0, bad = 0;
    for (int s0 = t0 + tid; s0 < t1; s0 += 8 * RT) {
        uint4 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = s0 + u * RT;
            v[u] = t < t1 ? tm[t] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a = max(a, v[u].x); b = max(b, v[u].y); c = max(c, v[u].z); bad = max(bad, v[u].w);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        a = max(a, (unsigned)__shfl_xor((int)a, off));
        b = max(b, (unsigned)__shfl_xor((int)b, off));
        c = max(c, (unsigned)__shfl_xor((int)c, off));
        bad = max(bad, (unsigned)__shfl_xor((int)bad, off));
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = a; red[1][tid >> 6] = b; red[2][tid >> 6] = c; red[3][tid >> 6] = bad;
    }
    __syncthreads();
    if (tid == 0)
        for (int w = 1; w < RT / 64; ++w) {
            a = max(a, red[0][w]); b = max(b, red[1][w]); c = max(c, red[2][w]); bad = max(bad, red[3][w]);
        }
    return make_uint4(a, b, c, bad);
}

// K3 proper (one thread): the Eq. 7 step from the maxima (float bits) of
// |v|, |v| + c and |J0|/(1-psi) and the nonfinite flag; publishes dt, the
// time ring, the source balances and the step counter, or the error.
struct Eq7 {
    double dt;
    int which, err;
};
__device__ Eq7 eq7_step(const StepArgs &A, uint4 m)
{
    double vp = __uint_as_float(m.x), vs = __uint_as_float(m.y), D = __uint_as_float(m.z);
    double h = A.dx;
    double t0 = vp > 0.0 ? h / (2.0 * vp) : INFINITY;
    double t1 = vs > 0.0 ? h / vs : INFINITY;
    double t2 = D > 0.0 ? h * h / (2.0 * D) : INFINITY;
    double mm = t0;
    int which = 0;
    if (t1 < mm) { mm = t1; which = 1; }
    if (t2 < mm) { mm = t2; which = 2; }
    double dt = A.cfl * mm;
    if (!(dt < A.dt_max)) { dt = A.dt_max; which = 3; }
    int err = 0;
    if (m.w) err = SW_ERR_NONFINITE;
    else if (A.mode_fixed && A.dt_fixed > dt) err = SW_ERR_CFL;
    if (A.mode_fixed) { dt = A.dt_fixed; which = 4; }
    if (!err && dt < A.dt_min) err = SW_ERR_DT_UNDERFLOW;
    return Eq7{dt, which, err};
}

__device__ void publish_dt(Ctrl *ctrl, int par, const StepArgs &A, uint4 m)
{
    if (ctrl->err) return;
    const int kd = ctrl->kdev;
    ctrl->vp = __uint_as_float(m.x); ctrl->vs = __uint_as_float(m.y); ctrl->D = __uint_as_float(m.z);
    const Eq7 e = eq7_step(A, m);
    const double dt = e.dt;
    const int which = e.which;
    if (e.err) {
        ctrl->err = e.err;
        ctrl->err_k = kd;
        return;
    }
    double tn = ctrl->t[par];
    double q = 0.0;
    if (A.has_inflow) {
        double d = tn + 0.5 * dt - A.t_peak;
        double pk = A.t_sigma > 0.0 ? A.q_peak * exp(-d * d / (2.0 * A.t_sigma * A.t_sigma)) : 0.0;
        q = A.q_base + pk;
        ctrl->in_w += dt * q;
    }
    ctrl->in_s += dt * A.qb_total;
    ctrl->in_rain += dt * A.rain_area;
    ctrl->qmid[par] = q;
    ctrl->dt[par] = dt;
    ctrl->t[par ^ 1] = tn + dt;
    ctrl->last_dt = dt;
    ctrl->binding = which;
    ctrl->kdev = kd + 1;
    log_step(A, kd, tn, dt, ctrl->vp, ctrl->vs, ctrl->D, q, which);
}

// K3 of one grid in one 1024-thread workgroup (the maximum does not depend
// on the order it is taken in).
__device__ void reduce_dt(Ctrl *ctrl, int par, const StepArgs &A, const uint4 *__restrict__ tm,
                          int ntiles)
{
    const uint4 m = block_tile_maxima(tm, 0, ntiles);
    if (threadIdx.x == 0) publish_dt(ctrl, par, A, m);
}

// Initial maxima (ring par) and wet-tile flags of a state set from the host.
template <int TX, int TY>
__device__ __forceinline__ void prepare_tile(const Inst &I, int par, int bx, int by)
{
    __shared__ int s_any;
    const KPar &P = I.P;
    const int tid = threadIdx.x;
    const int x0 = bx * TX, y0 = by * TY, tile = bx + by * I.ntx;
    const float *H = I.H[par], *qx = I.qx[par], *qy = I.qy[par], *b = I.b[par];
    if (tid == 0) s_any = 0;
    __syncthreads();
    unsigned mv = 0, ms = 0, mD = 0, bad = 0;
    for (int q = tid; q < TX * TY; q += NT) {
        int i = x0 + q % TX, j = y0 + q / TX;
        if (i >= P.nx || j >= P.ny) continue;
        int c = j * P.pitch + i;
        float h = H[c];
        float jx, jy, jm;
        cell_maxima_j(P, h, qx[c], qy[c], b[c], soil(P.nM, P.nM_s, c), soil(P.d50, P.d50_s, c),
                      soil(P.psi, P.psi_s, c), mv, ms, mD, bad, jx, jy, jm);
        I.jx[par][c] = jx;
        I.jy[par][c] = jy;
        I.jm[par][c] = jm;
        if (h > 0.0f) s_any = 1;
    }
    block_maxima_store(mv, ms, mD, bad, &I.tmax[par][tile]);
    if (tid == 0) I.act[par][tile] = (s_any || I.force[tile]) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Per-cell arithmetic shared by the tile and strip kernels (one copy of each
// expression, so both paths give the same bits).
// ---------------------------------------------------------------------------

// K4 half-step depth of cell (i, j) from its velocities and those of its four
// neighbours (wall face: 0, open face: the cell's own velocity).
__device__ __forceinline__ float half_depth_cell(const KPar &P, float H, float uc, float uW, float uE,
                                                 float vc, float vS, float vN, int i, int j,
                                                 float hdt_dx)
{
    float ue, uw, vn, vs;
    if (i + 1 < P.nx) ue = 0.5f * (uc + uE);
    else ue = (P.bcE == kWall) ? 0.0f : uc;
    if (i > 0) uw = 0.5f * (uW + uc);
    else uw = (P.bcW == kWall) ? 0.0f : uc;
    if (j + 1 < P.ny) vn = 0.5f * (vc + vN);
    else vn = (P.bcN == kWall) ? 0.0f : vc;
    if (j > 0) vs = 0.5f * (vS + vc);
    else vs = (P.bcS == kWall) ? 0.0f : vc;
    float Jx = 1.0f + hdt_dx * (ue - uw);
    float Jy = 1.0f + hdt_dx * (vn - vs);
    return ndiv(H, Jx * Jy);
}

// K2 + K4 + K5 + K6 of one cell: forces at t_n from the depths and beds of the
// cell (C) and its W/E/S/N neighbours, semi-implicit predictor, forces at
// t_{n+1/2} from the half-step depths, corrector to the Lagrangian momentum.
struct NbrDepths {
    float C, W, E, S, N;
};
// Predictor and corrector of one cell from its forces at t_n (Snx, Sny, on
// depth HdC) and at t_{n+1/2} (Shx, Shy, on the half-step depth HhC).
__device__ __forceinline__ void lagrange_momentum(const KPar &P, float dt, float HdC, float HhC,
                                                  float Snx, float Sny, float Shx, float Shy,
                                                  float qxc, float qyc, float nM, float &QLx,
                                                  float &QLy)
{
    float wc = wdes(HdC, P);
    float uc = qxc * wc, vc = qyc * wc;
    float gam = friction_rate(P, nM, nsqrt(sumsq(uc, vc)), HdC);
    float hdt = 0.5f * dt;
    float qpx, qpy;
    if (P.force) {  // Coriolis and wind at t_n
        const float chi = fminf(1.0f, HdC * P.inv_hsed);
        qpx = ndiv(qxc + hdt * (Snx + (P.cor * qyc + chi * P.wsx)), 1.0f + hdt * gam);
        qpy = ndiv(qyc + hdt * (Sny + (-P.cor * qxc + chi * P.wsy)), 1.0f + hdt * gam);
    } else {
        qpx = ndiv(qxc + hdt * Snx, 1.0f + hdt * gam);
        qpy = ndiv(qyc + hdt * Sny, 1.0f + hdt * gam);
    }
    float upx = qpx * wc, upy = qpy * wc;
    float gamh = friction_rate(P, nM, nsqrt(sumsq(upx, upy)), HhC);
    if (P.force) {  // at t_{n+1/2}: half-step depth, predictor momentum
        const float chi = fminf(1.0f, HhC * P.inv_hsed);
        QLx = ndiv(qxc + dt * (Shx + (P.cor * qpy + chi * P.wsx)), 1.0f + dt * gamh);
        QLy = ndiv(qyc + dt * (Shy + (-P.cor * qpx + chi * P.wsy)), 1.0f + dt * gamh);
    } else {
        QLx = ndiv(qxc + dt * Shx, 1.0f + dt * gamh);
        QLy = ndiv(qyc + dt * Shy, 1.0f + dt * gamh);
    }
}

// The same with the first-order forces from the depths and beds of the cell
// (C) and its W/E/S/N neighbours.
__device__ __forceinline__ void lagrange_cell(const KPar &P, float dt, const NbrDepths &Hd,
                                              const NbrDepths &bd, const NbrDepths &Hh, bool hasW,
                                              bool hasE, bool hasS, bool hasN, float qxc, float qyc,
                                              float nM, float &QLx, float &QLy)
{
    float Snx = face_force(P, Hd.W, bd.W, Hd.C, bd.C, Hd.E, bd.E, hasW, hasE);
    float Sny = face_force(P, Hd.S, bd.S, Hd.C, bd.C, Hd.N, bd.N, hasS, hasN);
    float HhW = hasW ? Hh.W : Hh.C, HhE = hasE ? Hh.E : Hh.C;
    float HhS = hasS ? Hh.S : Hh.C, HhN = hasN ? Hh.N : Hh.C;
    float Shx = face_force(P, HhW, bd.W, Hh.C, bd.C, HhE, bd.E, hasW, hasE);
    float Shy = face_force(P, HhS, bd.S, Hh.C, bd.C, HhN, bd.N, hasS, hasN);
    lagrange_momentum(P, dt, Hd.C, Hh.C, Snx, Sny, Shx, Shy, qxc, qyc, nM, QLx, QLy);
}

// Draining limiter of a cell of depth h from its four raw mass fluxes.
__device__ __forceinline__ float drain_theta(const KPar &P, float dt, float h, float fw, float fe,
                                             float gs, float gn)
{
    float out = (fmaxf(0.0f, fe) + fmaxf(0.0f, -fw)) + (fmaxf(0.0f, gn) + fmaxf(0.0f, -gs));
    return out > 0.0f ? fminf(1.0f, h * P.dx / (dt * out)) : 1.0f;
}

// Raw fluxes and limiters around one cell, the inputs of its K8 update.
struct CellFaces {
    float th, thW, thE, thS, thN;        // limiters of the cell and its four neighbours
    float xHw, xnw, xtw, xHe, xne, xte;  // raw x-face fluxes (mass, normal, tangential), W and E
    float yHs, yns, yts, yHn, ynn, ytn;  // raw y-face fluxes, S and N
    float Jw, Je, Js, Jn;                // bedload face fluxes
};
struct CellNew {
    float H, qx, qy, b;
    float FHw, FHe, GHs, GHn;  // limited mass fluxes (boundary balances)
    float ab;                  // depth absorbed this step
};

// K8 of one cell: each face's water fluxes take the limiter of the cell the
// mass leaves; conservative update of H and momentum from Q^L, Exner update
// of b (Eq. 1), negative depth clamped, momentum re-desingularised below eps.
// Rainfall adds depth only; absorption (dH/dt = -beta H, implicit) divides
// depth and momentum by 1 + beta dt, so the absorbed water leaves with its
// velocity.
// The rainfall is added compensated: rh carries the part of the earlier
// additions the float32 depth could not hold (as the bed's residual does for
// the Exner update), so a rain increment far below an ulp of the depth is
// not rounded away step after step.
__device__ __forceinline__ CellNew cell_update(const KPar &P, float dt, const CellFaces &F, float h,
                                               float qx, float qy, float b, float QLx, float QLy,
                                               float src, float psi, float qb, float beta, float &rb,
                                               float &rh)
{
    // the limiter of the cell the mass leaves (1 for no flux), as selects
    float sw = F.xHw < 0.0f ? F.th : 1.0f;
    sw = F.xHw > 0.0f ? F.thW : sw;
    float se = F.xHe < 0.0f ? F.thE : 1.0f;
    se = F.xHe > 0.0f ? F.th : se;
    float ss = F.yHs < 0.0f ? F.th : 1.0f;
    ss = F.yHs > 0.0f ? F.thS : ss;
    float sn = F.yHn < 0.0f ? F.thN : 1.0f;
    sn = F.yHn > 0.0f ? F.th : sn;
    CellNew o;
    o.FHw = F.xHw * sw; o.FHe = F.xHe * se; o.GHs = F.yHs * ss; o.GHn = F.yHn * sn;
    float Fxw = F.xnw * sw, Fxe = F.xne * se, Gxs = F.yts * ss, Gxn = F.ytn * sn;
    float Fyw = F.xtw * sw, Fye = F.xte * se, Gys = F.yns * ss, Gyn = F.ynn * sn;
    float QLxc = h > 0.0f ? QLx : qx;
    float QLyc = h > 0.0f ? QLy : qy;
    float r = dt * P.inv_dx;
    float Hn = h - r * ((o.FHe - o.FHw) + (o.GHn - o.GHs)) + dt * src;
    float qxn = QLxc - r * ((Fxe - Fxw) + (Gxn - Gxs));
    float qyn = QLyc - r * ((Fye - Fyw) + (Gyn - Gys));
    float om = 1.0f - psi;
    float bn = exner(P, dt, b, om, (F.Je - F.Jw) + (F.Jn - F.Js), qb, rb);
    if (P.rain > 0.0f) {
        const float d = dt * P.rain + rh;
        const float hn = Hn + d;
        const float dv = hn - Hn;
        rh = (Hn - (hn - dv)) + (d - dv);
        Hn = hn;
    }
    if (Hn < 0.0f) Hn = 0.0f;
    o.ab = 0.0f;
    if (beta > 0.0f) {
        // 1 / (1 + beta dt) = 1 - f with the absorbed fraction f formed
        // directly, so the quotient's rounding does not sit in the small
        // difference H - H / (1 + beta dt); the absorbed depth is then that
        // difference taken exactly (the two depths are within a factor 2)
        const float bd = beta * dt;
        const float f = ndiv(bd, 1.0f + bd);
        const float Ha = fmaf(-Hn, f, Hn);
        o.ab = Hn - Ha;
        Hn = Ha;
        qxn = fmaf(-qxn, f, qxn);
        qyn = fmaf(-qyn, f, qyn);
        rh = fmaf(-rh, f, rh);
    }
    if (Hn < P.eps) {
        float sc = Hn * wdes(Hn, P);
        qxn *= sc;
        qyn *= sc;
    }
    o.H = Hn; o.qx = qxn; o.qy = qyn; o.b = bn;
    return o;
}

// FP64 balances of the water and sediment leaving through the boundary faces
// of cell (i, j) (one accumulator per boundary face, owned by that cell).
__device__ __forceinline__ void boundary_balances(const KPar &P, double *bnd, double wdx, int i,
                                                  int j, const CellNew &o, const CellFaces &F)
{
    const int nx = P.nx, ny = P.ny, nb = 2 * (nx + ny);
    if (i == 0) { bnd[j] += wdx * (double)(-o.FHw); bnd[nb + j] += wdx * (double)(-F.Jw); }
    if (i == nx - 1) { bnd[ny + j] += wdx * (double)o.FHe; bnd[nb + ny + j] += wdx * (double)F.Je; }
    if (j == 0) { bnd[2 * ny + i] += wdx * (double)(-o.GHs); bnd[nb + 2 * ny + i] += wdx * (double)(-F.Js); }
    if (j == ny - 1) { bnd[2 * ny + nx + i] += wdx * (double)o.GHn; bnd[nb + 2 * ny + nx + i] += wdx * (double)F.Jn; }
}

// Unfused sequence: K2..K6 per cell, then (after the face kernel) K8 per
// cell, through the same per-cell functions as the tiled kernels.
__global__ void __launch_bounds__(BX * BY) k_lagrange(KPar P, const Ctrl *__restrict__ ctrl, int k,
                                                      StateView S, float *__restrict__ QLx,
                                                      float *__restrict__ QLy)
{
    if (ctrl->err) return;
    int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= P.nx || j >= P.ny) return;
    float dt = (float)ctrl->dt[k & 1];
    int c = j * P.pitch + i;
    bool hasW = i > 0, hasE = i + 1 < P.nx, hasS = j > 0, hasN = j + 1 < P.ny;
    int cW = hasW ? c - 1 : c, cE = hasE ? c + 1 : c;
    int cS = hasS ? c - P.pitch : c, cN = hasN ? c + P.pitch : c;
    float hdt_dx = dt / (2.0f * P.dx);
    float Hh = half_depth(P, S, i, j, hdt_dx);
    NbrDepths Hd{S.H[c], S.H[cW], S.H[cE], S.H[cS], S.H[cN]};
    NbrDepths bd{S.b[c], S.b[cW], S.b[cE], S.b[cS], S.b[cN]};
    NbrDepths Hhd{Hh, hasW ? half_depth(P, S, i - 1, j, hdt_dx) : Hh,
                  hasE ? half_depth(P, S, i + 1, j, hdt_dx) : Hh,
                  hasS ? half_depth(P, S, i, j - 1, hdt_dx) : Hh,
                  hasN ? half_depth(P, S, i, j + 1, hdt_dx) : Hh};
    float qlx, qly;
    lagrange_cell(P, dt, Hd, bd, Hhd, hasW, hasE, hasS, hasN, S.qx[c], S.qy[c],
                  soil(P.nM, P.nM_s, c), qlx, qly);
    QLx[c] = qlx;
    QLy[c] = qly;
}

__global__ void __launch_bounds__(BX * BY) k_update(KPar P, Ctrl *__restrict__ ctrl, int k,
                                                    StateView S, LagView L, FaceView F, OutView O,
                                                    double *__restrict__ bnd)
{
    unsigned mv = 0, ms = 0, mD = 0, bad = 0;
    bool live = !ctrl->err;
    int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (live && i < P.nx && j < P.ny) {
        double dtd = ctrl->dt[k & 1];
        float dt = (float)dtd;
        int c = j * P.pitch + i;
        int fw = j * (P.nx + 1) + i, fe = fw + 1;
        int gs = j * P.nx + i, gn = gs + P.nx;
        CellFaces Fc;
        Fc.th = theta_of(P, S, F, i, j, dt);
        Fc.thW = theta_of(P, S, F, i - 1, j, dt); Fc.thE = theta_of(P, S, F, i + 1, j, dt);
        Fc.thS = theta_of(P, S, F, i, j - 1, dt); Fc.thN = theta_of(P, S, F, i, j + 1, dt);
        Fc.xHw = F.xH[fw]; Fc.xnw = F.xn[fw]; Fc.xtw = F.xt[fw];
        Fc.xHe = F.xH[fe]; Fc.xne = F.xn[fe]; Fc.xte = F.xt[fe];
        Fc.yHs = F.yH[gs]; Fc.yns = F.yn[gs]; Fc.yts = F.yt[gs];
        Fc.yHn = F.yH[gn]; Fc.ynn = F.yn[gn]; Fc.ytn = F.yt[gn];
        Fc.Jw = F.xJ[fw]; Fc.Je = F.xJ[fe]; Fc.Js = F.yJ[gs]; Fc.Jn = F.yJ[gn];
        float src = P.srcw ? P.srcw[c] * (float)ctrl->qmid[k & 1] : 0.0f;
        float rb = P.rb ? P.rb[c] : 0.0f;
        float rh = P.rh ? P.rh[c] : 0.0f;
        CellNew o = cell_update(P, dt, Fc, S.H[c], S.qx[c], S.qy[c], S.b[c], L.QLx[c], L.QLy[c], src,
                                soil(P.psi, P.psi_s, c), P.qb ? P.qb[c] : 0.0f,
                                soil(P.beta, P.beta_s, c), rb, rh);
        if (P.rb) P.rb[c] = rb;
        if (P.rh) P.rh[c] = rh;
        if (P.ab) P.ab[c] += (double)o.ab;
        O.H[c] = o.H; O.qx[c] = o.qx; O.qy[c] = o.qy; O.b[c] = o.b;
        boundary_balances(P, bnd, dtd * (double)P.dx, i, j, o, Fc);
        cell_maxima(P, o.H, o.qx, o.qy, o.b, c, mv, ms, mD, bad);
    }
    block_maxima(mv, ms, mD, bad, ctrl->slot[(k + 1) & 1], blockIdx.x + blockIdx.y * gridDim.x);
}

// Lagrangian stage on a tile (K2, K4, K5, K6) with the Eq. 7 step (K3).
template <int TX, int TY>
__device__ __forceinline__ void lagrange_tile(const Inst &I, int par, int bx, int by)
{
    constexpr int LW = TX + 4, LHh = TY + 4;  // state tile with a 2-cell halo
    __shared__ float sH[LHh][LW], sb[LHh][LW], sqx[LHh][LW], sqy[LHh][LW], su[LHh][LW],
        sv[LHh][LW];
    __shared__ float sHh[TY + 2][TX + 2];
    const KPar &P = I.P;
    if (I.ctrl->err) return;
    const int tile = bx + by * I.ntx;
    if (I.hgs && !I.act[par][tile]) return;
    const float dt = (float)I.ctrl->dt[par];
    const int x0 = bx * TX, y0 = by * TY, tid = threadIdx.x;
    const float *H = I.H[par], *Qx = I.qx[par], *Qy = I.qy[par], *B = I.b[par];
    for (int q = tid; q < LW * LHh; q += NT) {
        int rx = q % LW, ry = q / LW;
        int i = x0 - 2 + rx, j = y0 - 2 + ry;
        float h = 0.0f, qx = 0.0f, qy = 0.0f, b = 0.0f, u = 0.0f, v = 0.0f;
        if ((unsigned)i < (unsigned)P.nx && (unsigned)j < (unsigned)P.ny) {
            int c = j * P.pitch + i;
            h = H[c]; qx = Qx[c]; qy = Qy[c]; b = B[c];
            float w = wdes(h, P);
            u = qx * w;
            v = qy * w;
        }
        sH[ry][rx] = h; sb[ry][rx] = b; sqx[ry][rx] = qx; sqy[ry][rx] = qy; su[ry][rx] = u;
        sv[ry][rx] = v;
    }
    __syncthreads();
    const float hdt_dx = dt / (2.0f * P.dx);
    for (int q = tid; q < (TX + 2) * (TY + 2); q += NT) {
        int cx = q % (TX + 2), cy = q / (TX + 2);
        int i = x0 - 1 + cx, j = y0 - 1 + cy;
        float Hh = 0.0f;
        if ((unsigned)i < (unsigned)P.nx && (unsigned)j < (unsigned)P.ny) {
            int rx = cx + 1, ry = cy + 1;
            Hh = half_depth_cell(P, sH[ry][rx], su[ry][rx], su[ry][rx - 1], su[ry][rx + 1],
                                 sv[ry][rx], sv[ry - 1][rx], sv[ry + 1][rx], i, j, hdt_dx);
        }
        sHh[cy][cx] = Hh;
    }
    __syncthreads();
    for (int q = tid; q < TX * TY; q += NT) {
        int lx = q % TX, ly = q / TX;
        int i = x0 + lx, j = y0 + ly;
        if (i >= P.nx || j >= P.ny) continue;
        int rx = lx + 2, ry = ly + 2, cx = lx + 1, cy = ly + 1;
        bool hasW = i > 0, hasE = i + 1 < P.nx, hasS = j > 0, hasN = j + 1 < P.ny;
        NbrDepths Hd{sH[ry][rx], sH[ry][rx - 1], sH[ry][rx + 1], sH[ry - 1][rx], sH[ry + 1][rx]};
        NbrDepths bd{sb[ry][rx], sb[ry][rx - 1], sb[ry][rx + 1], sb[ry - 1][rx], sb[ry + 1][rx]};
        NbrDepths Hh{sHh[cy][cx], sHh[cy][cx - 1], sHh[cy][cx + 1], sHh[cy - 1][cx], sHh[cy + 1][cx]};
        int c = j * P.pitch + i;
        float QLx, QLy;
        lagrange_cell(P, dt, Hd, bd, Hh, hasW, hasE, hasS, hasN, sqx[ry][rx], sqy[ry][rx],
                      soil(P.nM, P.nM_s, c), QLx, QLy);
        I.QLx[c] = QLx;
        I.QLy[c] = QLy;
    }
}

// Euler stage on a tile (K7 + limiter + K8) with the epilogue reductions
// (Eq. 7 maxima and wet flags of the new state, FP64 boundary balances).
template <int TX, int TY>
__device__ __forceinline__ void euler_tile(const Inst &I, int par, int bx, int by)
{
    constexpr int EW = TX + 6, EHt = TY + 6;  // remap inputs with a 3-cell halo
    constexpr int RW = TX + 2, RH = TY + 2;   // the tile plus a 1-cell ring
    __shared__ float cz[EHt][EW], ch[EHt][EW], cux[EHt][EW], cuy[EHt][EW], cLx[EHt][EW],
        cLy[EHt][EW];
    __shared__ float rjx[RH][RW], rjy[RH][RW], rb[RH][RW], rth[RH][RW];
    __shared__ float fxH[RH][TX + 3], fxn[RH][TX + 3], fxt[RH][TX + 3];
    __shared__ float fyH[TY + 3][RW], fyn[TY + 3][RW], fyt[TY + 3][RW];
    __shared__ int s_flag;
    const KPar &P = I.P;
    Ctrl *ctrl = I.ctrl;
    if (ctrl->err) return;
    const int ntx = I.ntx, nty = I.nty;
    const int tile = bx + by * ntx, tid = threadIdx.x;
    const int x0 = bx * TX, y0 = by * TY;
    const int nx = P.nx, ny = P.ny;
    const float *SH = I.H[par], *Sqx = I.qx[par], *Sqy = I.qy[par], *Sb = I.b[par];
    float *OH = I.H[par ^ 1], *Oqx = I.qx[par ^ 1], *Oqy = I.qy[par ^ 1], *Ob = I.b[par ^ 1];
    const float *QLx = I.QLx, *QLy = I.QLy;
    const uint8_t *act_in = I.act[par];
    if (I.hgs) {
        bool run = act_in[tile] || (bx > 0 && act_in[tile - 1]) ||
                   (bx + 1 < ntx && act_in[tile + 1]) || (by > 0 && act_in[tile - ntx]) ||
                   (by + 1 < nty && act_in[tile + ntx]);
        if (!run) {
            if (tid == 0) s_flag = I.synced[tile];
            __syncthreads();
            if (!s_flag) {  // first skip since the tile last changed: bring the other buffer level
                for (int q = tid; q < TX * TY; q += NT) {
                    int i = x0 + q % TX, j = y0 + q / TX;
                    if (i >= nx || j >= ny) continue;
                    int c = j * P.pitch + i;
                    OH[c] = SH[c]; Oqx[c] = Sqx[c]; Oqy[c] = Sqy[c]; Ob[c] = Sb[c];
                }
            }
            if (tid == 0) {
                I.synced[tile] = 1;
                I.act[par ^ 1][tile] = 0;
                I.tmax[par ^ 1][tile] = make_uint4(0u, 0u, 0u, 0u);
            }
            return;
        }
        if (tid == 0) I.synced[tile] = 0;
    }
    const float dt = (float)ctrl->dt[par];
    const double dtd = ctrl->dt[par];
    const bool wW = P.bcW == kWall, wE = P.bcE == kWall, wS = P.bcS == kWall, wN = P.bcN == kWall;

    // remap inputs of every cell within 3 of the tile (ghost cells beyond the domain edge)
    for (int q = tid; q < EW * EHt; q += NT) {
        int rx = q % EW, ry = q / EW;
        int i = x0 - 3 + rx, j = y0 - 3 + ry;
        bool inx = (unsigned)i < (unsigned)nx, iny = (unsigned)j < (unsigned)ny;
        CellVals v{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (inx && iny) {
            int c = j * P.pitch + i;
            float h = SH[c], qx = Sqx[c], qy = Sqy[c], b = Sb[c];
            v = cell_vals(P, h, qx, qy, b, QLx[c], QLy[c]);
            int cx = rx - 2, cy = ry - 2;
            if ((unsigned)cx < (unsigned)RW && (unsigned)cy < (unsigned)RH) {
                float w = wdes(h, P);
                float jx, jy;
                bedload(P, h, qx * w, qy * w, soil(P.nM, P.nM_s, c), soil(P.d50, P.d50_s, c), jx,
                        jy);
                rjx[cy][cx] = jx;
                rjy[cy][cx] = jy;
                rb[cy][cx] = b;
            }
        } else if (iny && (i == -1 || i == nx)) {
            int c = j * P.pitch + (i < 0 ? 0 : nx - 1);
            v = mirror(cell_vals(P, SH[c], Sqx[c], Sqy[c], Sb[c], QLx[c], QLy[c]), 0,
                       i < 0 ? wW : wE);
        } else if (inx && (j == -1 || j == ny)) {
            int c = (j < 0 ? 0 : ny - 1) * P.pitch + i;
            v = mirror(cell_vals(P, SH[c], Sqx[c], Sqy[c], Sb[c], QLx[c], QLy[c]), 1,
                       j < 0 ? wS : wN);
        }
        cz[ry][rx] = v.z; ch[ry][rx] = v.h; cux[ry][rx] = v.utx; cuy[ry][rx] = v.uty;
        cLx[ry][rx] = v.uLx; cLy[ry][rx] = v.uLy;
    }
    __syncthreads();

    // raw water fluxes of every face of the tile and its ring
    auto cq = [&](int ry, int rx, int dir) -> CellQ {
        CellVals v{cz[ry][rx], ch[ry][rx], cux[ry][rx], cuy[ry][rx], cLx[ry][rx], cLy[ry][rx]};
        return along(v, dir);
    };
    for (int q = tid; q < RH * (TX + 3); q += NT) {
        int kk = q % (TX + 3), fr = q / (TX + 3);
        int k = x0 - 1 + kk, j = y0 - 1 + fr;
        float fH = 0.0f, fn = 0.0f, ft = 0.0f;
        if ((unsigned)j < (unsigned)ny && k >= 0 && k <= nx) {
            int ry = fr + 2;
            water_flux(P, k, nx, wW, wE, cq(ry, kk, 0), cq(ry, kk + 1, 0), cq(ry, kk + 2, 0),
                       cq(ry, kk + 3, 0), fH, fn, ft);
        }
        fxH[fr][kk] = fH; fxn[fr][kk] = fn; fxt[fr][kk] = ft;
    }
    for (int q = tid; q < (TY + 3) * RW; q += NT) {
        int cxk = q % RW, kk = q / RW;
        int i = x0 - 1 + cxk, k = y0 - 1 + kk;
        float fH = 0.0f, fn = 0.0f, ft = 0.0f;
        if ((unsigned)i < (unsigned)nx && k >= 0 && k <= ny) {
            int rx = cxk + 2;
            water_flux(P, k, ny, wS, wN, cq(kk, rx, 1), cq(kk + 1, rx, 1), cq(kk + 2, rx, 1),
                       cq(kk + 3, rx, 1), fH, fn, ft);
        }
        fyH[kk][cxk] = fH; fyn[kk][cxk] = fn; fyt[kk][cxk] = ft;
    }
    __syncthreads();

    // draining limiter of the tile and its ring (ghost donors: 1)
    for (int q = tid; q < RW * RH; q += NT) {
        int cx = q % RW, cy = q / RW;
        int i = x0 - 1 + cx, j = y0 - 1 + cy;
        float th = 1.0f;
        if ((unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny) {
            th = drain_theta(P, dt, ch[cy + 2][cx + 2], fxH[cy][cx], fxH[cy][cx + 1], fyH[cy][cx],
                             fyH[cy + 1][cx]);
        }
        rth[cy][cx] = th;
    }
    if (tid == 0) s_flag = 0;
    __syncthreads();

    // update of the tile's own cells
    unsigned mv = 0, ms = 0, mD = 0, bad = 0;
    double *bnd = I.bnd;
    for (int q = tid; q < TX * TY; q += NT) {
        int lx = q % TX, ly = q / TX;
        int i = x0 + lx, j = y0 + ly;
        if (i >= nx || j >= ny) continue;
        int cx = lx + 1, cy = ly + 1, c = j * P.pitch + i;
        CellFaces F;
        F.th = rth[cy][cx];
        F.thW = rth[cy][cx - 1]; F.thE = rth[cy][cx + 1]; F.thS = rth[cy - 1][cx]; F.thN = rth[cy + 1][cx];
        F.xHw = fxH[cy][cx]; F.xnw = fxn[cy][cx]; F.xtw = fxt[cy][cx];
        F.xHe = fxH[cy][cx + 1]; F.xne = fxn[cy][cx + 1]; F.xte = fxt[cy][cx + 1];
        F.yHs = fyH[cy][cx]; F.yns = fyn[cy][cx]; F.yts = fyt[cy][cx];
        F.yHn = fyH[cy + 1][cx]; F.ynn = fyn[cy + 1][cx]; F.ytn = fyt[cy + 1][cx];
        F.Jw = sed_flux(P, i, nx, wW, wE, 0, rjx[cy][cx - 1], rjy[cy][cx - 1], rb[cy][cx - 1],
                        rjx[cy][cx], rjy[cy][cx], rb[cy][cx]);
        F.Je = sed_flux(P, i + 1, nx, wW, wE, 0, rjx[cy][cx], rjy[cy][cx], rb[cy][cx],
                        rjx[cy][cx + 1], rjy[cy][cx + 1], rb[cy][cx + 1]);
        F.Js = sed_flux(P, j, ny, wS, wN, 1, rjx[cy - 1][cx], rjy[cy - 1][cx], rb[cy - 1][cx],
                        rjx[cy][cx], rjy[cy][cx], rb[cy][cx]);
        F.Jn = sed_flux(P, j + 1, ny, wS, wN, 1, rjx[cy][cx], rjy[cy][cx], rb[cy][cx],
                        rjx[cy + 1][cx], rjy[cy + 1][cx], rb[cy + 1][cx]);
        float src = P.srcw ? P.srcw[c] * (float)ctrl->qmid[par] : 0.0f;
        float rbc = P.rb ? P.rb[c] : 0.0f;
        float rhc = P.rh ? P.rh[c] : 0.0f;
        CellNew o = cell_update(P, dt, F, SH[c], Sqx[c], Sqy[c], Sb[c], QLx[c], QLy[c], src,
                                soil(P.psi, P.psi_s, c), P.qb ? P.qb[c] : 0.0f,
                                soil(P.beta, P.beta_s, c), rbc, rhc);
        OH[c] = o.H; Oqx[c] = o.qx; Oqy[c] = o.qy; Ob[c] = o.b;
        if (P.rb) P.rb[c] = rbc;
        if (P.rh) P.rh[c] = rhc;
        if (P.ab) P.ab[c] += (double)o.ab;
        boundary_balances(P, bnd, dtd * (double)P.dx, i, j, o, F);
        cell_maxima(P, o.H, o.qx, o.qy, o.b, c, mv, ms, mD, bad);
        if (o.H > 0.0f) s_flag = 1;
    }
    block_maxima_store(mv, ms, mD, bad, &I.tmax[par ^ 1][tile]);
    if (tid == 0) I.act[par ^ 1][tile] = (s_flag || I.force[tile]) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Strip path: one wavefront per tile of SX = 58 columns x S rows.  Lane l
// holds column x0 - 3 + l, so the 3-column halo on each side sits in lanes
// 0-2 and 61-63 and a cell's x neighbours are one DPP lane shift away; the
// wave marches up its rows, keeping the rows its stencil still needs in
// registers (the y neighbours), with the loads of the row two ahead in
// flight.  No LDS and no barriers: the four waves of a workgroup are four
// independent tiles stacked along y.  Every cell and face goes through the
// same device functions as in the tile kernels, so the bits are the same.
// ---------------------------------------------------------------------------

constexpr int SX = 58;           // interior columns of a strip tile
constexpr int SHALO = 3;         // halo columns on each side
constexpr int SWAVES = NT / 64;  // strip tiles per workgroup (stacked along y)
// Largest stage grid of a single grid's strip kernels (workgroups): dispatching
// a workgroup that finds no entry still costs time, so a mostly dry grid does
// not launch one per tile.
constexpr int kMaxStageGroups = 8192;
// Wavefronts per listed tile in a single grid's Lagrangian stage when tiles
// are skipped or the grid is small (each marches S / kLagHalves rows): more,
// shorter wavefronts hide the latency of the few tiles a step lists better
// than they cost in extra halo rows.
constexpr int kLagHalves = 2;
// Tiles per wavefront in a single grid's Lagrangian stage when every tile of a
// large grid is listed: one wavefront marches kLagGroup vertically stacked
// tiles as one strip, so their shared halo rows are loaded and computed once
// (the wavefronts are plentiful there).
constexpr int kLagGroup = 4;

// The value lane l-1 (lane_prev) or l+1 (lane_next) holds; 0 in the lane that
// has no such neighbour.  Called only where all 64 lanes are active.
// bound_ctrl set: the lane without a source reads 0, so no register has to
// be cleared before the move (lane layout checked on the GPU).
__device__ __forceinline__ float lane_prev(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_next(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ CellQ q_prev(const CellQ &q)
{
    return CellQ{lane_prev(q.z), lane_prev(q.h), lane_prev(q.ut), lane_prev(q.uLn), lane_prev(q.uLt)};
}
__device__ __forceinline__ CellQ q_next(const CellQ &q)
{
    return CellQ{lane_next(q.z), lane_next(q.h), lane_next(q.ut), lane_next(q.uLn), lane_next(q.uLt)};
}

// Maximum over the 64 lanes (all active), uniform: DPP swaps within quads
// (quad_perm [1,0,3,2] and [2,3,0,1]), half rows (row_half_mirror) and rows
// of 16 (row_mirror) leave each row's maximum in all its lanes; the four row
// maxima are then read as scalars.
template <int CTRL>
__device__ __forceinline__ unsigned dpp_max(unsigned x)
{
    return max(x, (unsigned)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ unsigned wave_max_u32(unsigned x)
{
    x = dpp_max<0xb1>(x);
    x = dpp_max<0x4e>(x);
    x = dpp_max<0x141>(x);
    x = dpp_max<0x140>(x);
    const unsigned r0 = __builtin_amdgcn_readlane((int)x, 0), r1 = __builtin_amdgcn_readlane((int)x, 16);
    const unsigned r2 = __builtin_amdgcn_readlane((int)x, 32), r3 = __builtin_amdgcn_readlane((int)x, 48);
    return max(max(r0, r1), max(r2, r3));
}

// Wave-wide maxima of the Eq. 7 contributions and the wet flag of a strip
// tile, stored with plain writes into the tile's slots.
__device__ __forceinline__ void strip_maxima_store(const Inst &I, int par_out, int tile, unsigned a,
                                                   unsigned b, unsigned c, unsigned bad, bool wet)
{
    a = wave_max_u32(a);
    b = wave_max_u32(b);
    c = wave_max_u32(c);
    bad = wave_max_u32(bad);
    const bool any_wet = __ballot(wet) != 0;
    if ((threadIdx.x & 63) == 0) {
        I.tmax[par_out][tile] = make_uint4(a, b, c, bad);
        I.act[par_out][tile] = (any_wet || I.force[tile]) ? 1 : 0;
    }
}

// One row of a strip as loaded (clamped into the grid; the consumer zeroes
// what lies outside): state, Lagrangian momentum, soil and sources.
struct StripRow {
    float h, qx, qy, b, Lx, Ly;
    float nM, d50, psi, src, qb;
};

struct Flux3 {
    float H, n, t;
};
struct BedCell {
    float jx, jy, b;
};

// Lagrangian stage on a strip tile (CS: per-cell Manning coefficient).  Its
// callers pass listed tiles only: under skipping, the list holds exactly the
// tiles whose wet flag is set, so the flag is not read again here.
template <int S, bool CS>
__device__ __forceinline__ void lagrange_strip(const Inst &I, int par, int bx, int by, float dt)
{
    const KPar &P = I.P;
    const int lane = threadIdx.x & 63;
    const int nx = P.nx, ny = P.ny, pitch = P.pitch;
    const int x0 = bx * SX, y0 = by * S;
    const int i = x0 - SHALO + lane;
    const bool inx = (unsigned)i < (unsigned)nx;
    const bool mine = lane >= SHALO && lane < SHALO + SX && inx;
    const int ci = min(max(i, 0), nx - 1);
    const int jend = min(y0 + S, ny);
    const float *H = I.H[par], *Qx = I.qx[par], *Qy = I.qy[par], *B = I.b[par];
    const float hdt_dx = dt / (2.0f * P.dx);
    struct LRow {
        float h, qx, qy, b, nM;
    };
    auto load_row = [&](int r, LRow &w) {
        const int c = min(max(r, 0), ny - 1) * pitch + ci;
        w.h = H[c]; w.qx = Qx[c]; w.qy = Qy[c]; w.b = B[c];
        w.nM = CS && P.nM ? P.nM[c] : P.nM_s;
    };
    // rows r-3 .. r of depth and bed, r-2 .. r of momentum and Manning n,
    // r-1 .. r of u, r-2 .. r of v, half-step depths of rows r-3 .. r-1
    float H0 = 0, H1 = 0, H2 = 0, H3 = 0, b0 = 0, b1 = 0, b2 = 0, b3 = 0;
    float qx1 = 0, qx2 = 0, qx3 = 0, qy1 = 0, qy2 = 0, qy3 = 0, n1 = 0, n2 = 0, n3 = 0;
    float u2 = 0, u3 = 0, v1 = 0, v2 = 0, v3 = 0;
    float Hh0 = 0, Hh1 = 0, Hh2 = 0;
    auto step = [&](int r, const LRow &in) {
        H0 = H1; H1 = H2; H2 = H3; b0 = b1; b1 = b2; b2 = b3;
        qx1 = qx2; qx2 = qx3; qy1 = qy2; qy2 = qy3; n1 = n2; n2 = n3;
        u2 = u3; v1 = v2; v2 = v3;
        const bool ok = inx && (unsigned)r < (unsigned)ny;
        H3 = ok ? in.h : 0.0f;
        b3 = ok ? in.b : 0.0f;
        qx3 = ok ? in.qx : 0.0f;
        qy3 = ok ? in.qy : 0.0f;
        n3 = in.nM;
        const float w = wdes(H3, P);
        u3 = ok ? qx3 * w : 0.0f;
        v3 = ok ? qy3 * w : 0.0f;
        {  // K4 half-step depth of row r-1 (the tile's rows and a one-row ring)
            const int j = r - 1;
            const float uW = lane_prev(u2), uE = lane_next(u2);
            float hh = 0.0f;
            if (j >= y0 - 1 && j <= y0 + S && inx && (unsigned)j < (unsigned)ny)
                hh = half_depth_cell(P, H2, u2, uW, uE, v2, v1, v3, i, j, hdt_dx);
            Hh0 = Hh1; Hh1 = Hh2; Hh2 = hh;
        }
        const int j = r - 2;  // K2, K4, K5, K6 of row r-2
        if (j >= y0 && j < jend) {
            const float HW = lane_prev(H1), HE = lane_next(H1);
            const float bW = lane_prev(b1), bE = lane_next(b1);
            const float hW = lane_prev(Hh1), hE = lane_next(Hh1);
            if (mine) {
                NbrDepths Hd{H1, HW, HE, H0, H2};
                NbrDepths bd{b1, bW, bE, b0, b2};
                NbrDepths Hh{Hh1, hW, hE, Hh0, Hh2};
                float QLx, QLy;
                lagrange_cell(P, dt, Hd, bd, Hh, i > 0, i + 1 < nx, j > 0, j + 1 < ny, qx1, qy1, n1,
                              QLx, QLy);
                const int c = j * pitch + i;
                I.QLx[c] = QLx;
                I.QLy[c] = QLy;
            }
        }
    };
    const int rlo = y0 - 2, rhi = y0 + S + 1;  // S + 4 rows, an even count
    LRow A, Bq;
    load_row(rlo, A);
    load_row(rlo + 1, Bq);
    for (int r = rlo; r <= rhi; r += 2) {
        step(r, A);
        if (r + 2 <= rhi) load_row(r + 2, A);
        step(r + 1, Bq);
        if (r + 3 <= rhi) load_row(r + 3, Bq);
    }
}

// Lagrangian stage on a strip tile with the second-order force (hydrostatic
// faces on limited reconstructions of surface and depth, face_force2).  Its
// stencil reaches two cells past the cell, and the half-step depths it uses
// need the velocities one more row out, so the march covers rows y0-3 ..
// y0+S+2 and computes K2..K6 of row r-3 at row r (the first-order march:
// y0-2 .. y0+S+1, row r-2).  x neighbours: three halo lanes suffice.
template <int S, bool CS>
__device__ __forceinline__ void lagrange_strip2(const Inst &I, int par, int bx, int by, float dt)
{
    const KPar &P = I.P;
    const int lane = threadIdx.x & 63;
    const int nx = P.nx, ny = P.ny, pitch = P.pitch;
    const int x0 = bx * SX, y0 = by * S;
    const int i = x0 - SHALO + lane;
    const bool inx = (unsigned)i < (unsigned)nx;
    const bool mine = lane >= SHALO && lane < SHALO + SX && inx;
    const bool hasW = i > 0, hasE = i + 1 < nx;
    const int ci = min(max(i, 0), nx - 1);
    const int jend = min(y0 + S, ny);
    const float *H = I.H[par], *Qx = I.qx[par], *Qy = I.qy[par], *B = I.b[par];
    const float hdt_dx = dt / (2.0f * P.dx);
    struct LRow {
        float h, qx, qy, b, nM;
    };
    auto load_row = [&](int r, LRow &w) {
        const int c = min(max(r, 0), ny - 1) * pitch + ci;
        w.h = H[c]; w.qx = Qx[c]; w.qy = Qy[c]; w.b = B[c];
        w.nM = CS && P.nM ? P.nM[c] : P.nM_s;
    };
    // for the current row r: depth and bed of rows r-5 .. r (H5 .. H0),
    // momentum and Manning n of rows r-3 .. r, u of rows r-1 .. r, v of rows
    // r-2 .. r, half-step depths of rows r-5 .. r-1 (Hh5 .. Hh1)
    float H5 = 0, H4 = 0, H3 = 0, H2 = 0, H1 = 0, H0 = 0;
    float b5 = 0, b4 = 0, b3 = 0, b2 = 0, b1 = 0, b0 = 0;
    float qx3 = 0, qx2 = 0, qx1 = 0, qx0 = 0, qy3 = 0, qy2 = 0, qy1 = 0, qy0 = 0;
    float n3 = 0, n2 = 0, n1 = 0, n0 = 0;
    float u1 = 0, u0 = 0, v2 = 0, v1 = 0, v0 = 0;
    float Hh5 = 0, Hh4 = 0, Hh3 = 0, Hh2 = 0, Hh1 = 0;
    // limited slopes (a boundary cell's ghost is the cell itself)
    auto xslope = [&](float a, float aW, float aE) {
        return limited<true>(P, hasW ? a - aW : 0.0f, hasE ? aE - a : 0.0f);
    };
    auto yslope = [&](int j, float am, float a, float ap) {
        return limited<true>(P, j > 0 ? a - am : 0.0f, j + 1 < ny ? ap - a : 0.0f);
    };
    // both force components on row j of depth rows d[j-2 .. j+2] over bed
    // rows e[j-2 .. j+2]; the lane shifts run with every lane active
    auto forces2 = [&](int j, float dm2, float dm1, float d, float dp1, float dp2, float em2,
                       float em1, float e, float ep1, float ep2, float &Sx, float &Sy) {
        const float z = d + e;
        const float zW = lane_prev(z), zE = lane_next(z);
        const float dW = lane_prev(d), dE = lane_next(d);
        const float sz = xslope(z, zW, zE), sh = xslope(d, dW, dE);
        const ReconQ Wx{zW, dW, lane_prev(sz), lane_prev(sh)};
        const ReconQ Cx{z, d, sz, sh};
        const ReconQ Ex{zE, dE, lane_next(sz), lane_next(sh)};
        Sx = face_force2(P, Wx, Cx, Ex, hasW, hasE);
        const float zm2 = dm2 + em2, zm1 = dm1 + em1, zp1 = dp1 + ep1, zp2 = dp2 + ep2;
        const ReconQ Sq{zm1, dm1, yslope(j - 1, zm2, zm1, z), yslope(j - 1, dm2, dm1, d)};
        const ReconQ Cy{z, d, yslope(j, zm1, z, zp1), yslope(j, dm1, d, dp1)};
        const ReconQ Nq{zp1, dp1, yslope(j + 1, z, zp1, zp2), yslope(j + 1, d, dp1, dp2)};
        Sy = face_force2(P, Sq, Cy, Nq, j > 0, j + 1 < ny);
    };
    auto step = [&](int r, const LRow &in) {
        H5 = H4; H4 = H3; H3 = H2; H2 = H1; H1 = H0;
        b5 = b4; b4 = b3; b3 = b2; b2 = b1; b1 = b0;
        qx3 = qx2; qx2 = qx1; qx1 = qx0; qy3 = qy2; qy2 = qy1; qy1 = qy0;
        n3 = n2; n2 = n1; n1 = n0;
        u1 = u0; v2 = v1; v1 = v0;
        Hh5 = Hh4; Hh4 = Hh3; Hh3 = Hh2; Hh2 = Hh1;
        const bool ok = inx && (unsigned)r < (unsigned)ny;
        H0 = ok ? in.h : 0.0f;
        b0 = ok ? in.b : 0.0f;
        qx0 = ok ? in.qx : 0.0f;
        qy0 = ok ? in.qy : 0.0f;
        n0 = in.nM;
        const float w = wdes(H0, P);
        u0 = ok ? qx0 * w : 0.0f;
        v0 = ok ? qy0 * w : 0.0f;
        {  // K4 half-step depth of row r-1 (the tile's rows and two-row rings)
            const int j = r - 1;
            const float uW = lane_prev(u1), uE = lane_next(u1);
            float hh = 0.0f;
            if (j >= y0 - 2 && j <= y0 + S + 1 && inx && (unsigned)j < (unsigned)ny)
                hh = half_depth_cell(P, H1, u1, uW, uE, v1, v2, v0, i, j, hdt_dx);
            Hh1 = hh;
        }
        const int j = r - 3;  // K2, K4, K5, K6 of row r-3
        if (j >= y0 && j < jend) {
            float Snx, Sny, Shx, Shy;
            forces2(j, H5, H4, H3, H2, H1, b5, b4, b3, b2, b1, Snx, Sny);
            forces2(j, Hh5, Hh4, Hh3, Hh2, Hh1, b5, b4, b3, b2, b1, Shx, Shy);
            if (mine) {
                float QLx, QLy;
                lagrange_momentum(P, dt, H3, Hh3, Snx, Sny, Shx, Shy, qx3, qy3, n3, QLx, QLy);
                const int c = j * pitch + i;
                I.QLx[c] = QLx;
                I.QLy[c] = QLy;
            }
        }
    };
    const int rlo = y0 - 3, rhi = y0 + S + 2;  // S + 6 rows, an even count
    LRow A, Bq;
    load_row(rlo, A);
    load_row(rlo + 1, Bq);
    for (int r = rlo; r <= rhi; r += 2) {
        step(r, A);
        if (r + 2 <= rhi) load_row(r + 2, A);
        step(r + 1, Bq);
        if (r + 3 <= rhi) load_row(r + 3, Bq);
    }
}

// Euler stage on a strip tile (K7 + limiter + K8) with the epilogue
// reductions (Eq. 7 maxima and wet flag of the new state, boundary balances).
// CS: some soil or source field is a per-cell plane (else all are scalars).
// The caller has checked the error flag (one memory round trip per
// wavefront saved: the step and the first rows load together).
template <int S, bool CS, bool V>
__device__ __forceinline__ void euler_strip(const Inst &I, int par, int bx, int by)
{
    const KPar &P = I.P;
    Ctrl *ctrl = I.ctrl;
    const int ntx = I.ntx, tile = bx + by * ntx;
    const int lane = threadIdx.x & 63;
    const int nx = P.nx, ny = P.ny, pitch = P.pitch;
    const int x0 = bx * SX, y0 = by * S;
    const int i0 = x0 - SHALO + lane;  // this lane's column
    const int jend = min(y0 + S, ny);
    const float *SH = I.H[par], *Sqx = I.qx[par], *Sqy = I.qy[par], *Sb = I.b[par];
    float *OH = I.H[par ^ 1], *Oqx = I.qx[par ^ 1], *Oqy = I.qy[par ^ 1], *Ob = I.b[par ^ 1];
    const float *QLx = I.QLx, *QLy = I.QLy;
    const double dtd = ctrl->dt[par];
    const float dt = (float)dtd;
    const float qmid = (float)ctrl->qmid[par];
    const double wdx = dtd * (double)P.dx;
    const bool wW = P.bcW == kWall, wE = P.bcE == kWall, wS = P.bcS == kWall, wN = P.bcN == kWall;
    const int ci = min(max(i0, 0), nx - 1);
    const float *Jx = I.jx[par], *Jy = I.jy[par], *Jm = I.jm[par];
    // every plane is addressed as a uniform base plus one 32-bit byte offset
    auto at = [](const float *base, unsigned o) -> float {
        return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) + o);
    };
    auto put = [](float *base, unsigned o, float v) {
        *reinterpret_cast<float *>(reinterpret_cast<char *>(base) + o) = v;
    };
    auto soil_at = [&](const float *a, float sc, unsigned o) -> float {
        return CS && a ? at(a, o) : sc;
    };
    // a row as loaded (clamped into the grid; the consumer zeroes what lies
    // outside): state, Lagrangian momentum, J0 and |J0| of the state
    struct Row {
        float h, qx, qy, b, Lx, Ly, jx, jy, jm;
    };
    auto load_row = [&](int r, Row &w) {
        const unsigned o = (unsigned)(min(max(r, 0), ny - 1) * pitch + ci) * 4u;
        w.h = at(SH, o); w.qx = at(Sqx, o); w.qy = at(Sqy, o); w.b = at(Sb, o);
        w.Lx = at(QLx, o); w.Ly = at(QLy, o);
        w.jx = at(Jx, o); w.jy = at(Jy, o); w.jm = at(Jm, o);
    };
    // registers carried along the march, for the current row r:
    CellVals v1{}, v2{}, v3{};                 // remap inputs of rows r-2 .. r
    SideQ yp{};                                // plus (north) side of row r-2 along y
    Flux3 X3{}, X2{};                          // raw x fluxes of this lane's W face, rows r-3, r-2
    Flux3 Y3{}, Y2{}, Y1{};                    // raw y fluxes of faces r-3, r-2, r-1
    float th4 = 1.0f, th3 = 1.0f, th2 = 1.0f;  // limiters of rows r-4 .. r-2
    float xs3 = 0, xs2 = 0, xs1 = 0, xs0 = 0;  // bedload flux of this lane's W face, rows r-3 .. r
    float ys3 = 0, ys2 = 0, ys1 = 0, ys0 = 0;  // bedload flux of y faces r-3 .. r
    float pjy = 0, pmag = 0, pb = 0;           // J0_y, |J0| and bed of row r-1
    unsigned mv = 0, ms = 0, mD = 0, bad = 0;
    bool wet = false;
    // The parts of the march a row takes, by its offset k = r - (y0 - 3) from
    // the first row: bedload of row r (2 <= k <= S + 3; W faces 3 <= k <= S + 2,
    // y faces from k = 3), y reconstruction of row r - 1 (k >= 2; its face
    // from k = 3), x faces and limiter of row r - 2 (4 <= k <= S + 5), K8 of
    // row r - 3 (k >= 6).  K >= 0: k is known at compile time (the first six
    // and last four rows); K = -1: a row of the middle of the march
    // (6 <= k <= S + 1), which takes every part.  Only the grid's own edges
    // are left to run-time (uniform) tests.
    auto step = [&](auto KC, int r, const Row &in) {
        constexpr int K = decltype(KC)::value;
        constexpr bool mid = K < 0;
        constexpr bool part_j = mid || (K >= 2 && K <= S + 3);
        constexpr bool part_jx = mid || (K >= 3 && K <= S + 2);
        constexpr bool part_jy = mid || (K >= 3 && K <= S + 3);
        constexpr bool part_y = mid || K >= 2;
        constexpr bool part_yface = mid || K >= 3;
        constexpr bool part_x = mid || (K >= 4 && K <= S + 5);
        constexpr bool part_upd = mid || K >= 6;
        // the column and its lane predicates are derived again in every row
        // from a copy the compiler cannot see through: kept across the march
        // they were 64-bit lane masks in scalar registers, more than fit, and
        // spilled to vector lanes to be read back row after row
        int ic = i0;
        asm volatile("" : "+v"(ic));
        const int i = ic;
        const bool inx = (unsigned)i < (unsigned)nx;
        const bool mine = (unsigned)(i - x0) < (unsigned)SX && inx;
        const bool xghost = i == -1 || i == nx;
        const bool face_x = i >= 0 && i <= nx;  // this lane's west face is a grid face
        // the cells K8 updates in this step (row r-3), loaded again (cache
        // hits); loaded in every step, from the nearest row of the tile when
        // r-3 lies outside it (then unused), so no row outside the march is read
        const int ju = r - 3;
        const bool upd = part_upd && ju < jend;
        unsigned uo = 0;
        float uh = 0, uqx = 0, uqy = 0, ub = 0, uLx = 0, uLy = 0, upsi = 0, usrc = 0, uqb = 0,
              unM = 0, ud50 = 0;
        if constexpr (part_upd) {
            uo = (unsigned)(min(ju, jend - 1) * pitch + ci) * 4u;
            uh = at(SH, uo); uqx = at(Sqx, uo); uqy = at(Sqy, uo); ub = at(Sb, uo);
            uLx = at(QLx, uo); uLy = at(QLy, uo);
            upsi = soil_at(P.psi, P.psi_s, uo);
            usrc = soil_at(P.srcw, 0.0f, uo);
            uqb = soil_at(P.qb, 0.0f, uo);
            unM = soil_at(P.nM, P.nM_s, uo);
            ud50 = soil_at(P.d50, P.d50_s, uo);
        }
        const bool iny = (unsigned)r < (unsigned)ny;
        {  // remap inputs of row r (ghost cells beyond the domain edge)
            const bool yghost = r == -1 || r == ny;
            const CellVals v = cell_vals(P, in.h, in.qx, in.qy, in.b, in.Lx, in.Ly);
            v1 = v2; v2 = v3;
            // a cell inside, a ghost beyond one edge (a wall mirrors the normal
            // components: the sign flips of `mirror`), or zero; selected per lane
            const bool gx = iny && !inx && xghost, gy = inx && !iny && yghost;
            const bool keep = (inx && iny) || gx || gy;
            const bool fx = gx && (i < 0 ? wW : wE), fy = gy && (r < 0 ? wS : wN);
            v3.z = keep ? v.z : 0.0f;
            v3.h = keep ? v.h : 0.0f;
            v3.utx = keep ? (fx ? -v.utx : v.utx) : 0.0f;
            v3.uLx = keep ? (fx ? -v.uLx : v.uLx) : 0.0f;
            v3.uty = keep ? (fy ? -v.uty : v.uty) : 0.0f;
            v3.uLy = keep ? (fy ? -v.uLy : v.uLy) : 0.0f;
        }
        xs3 = xs2; xs2 = xs1; xs1 = xs0;
        ys3 = ys2; ys2 = ys1; ys1 = ys0;
        if constexpr (part_j) {  // J0 (Eqs. 3-5) of row r and its bedload faces
            // J0 and |J0| of the state were stored by the step that produced it
            const bool in_dom = inx && iny;
            const float jx = in_dom ? in.jx : 0.0f, jy = in_dom ? in.jy : 0.0f;
            const float mag = in_dom ? in.jm : 0.0f, b = in_dom ? in.b : 0.0f;
            const float jxW = lane_prev(jx), magW = lane_prev(mag), bW = lane_prev(b);
            float xs = 0.0f, ys = 0.0f;
            if (part_jx && r < jend && face_x)  // W face of this lane in row r
                xs = sed_face(P, i, nx, wW, wE, jxW, magW, bW, jx, mag, b);
            if (part_jy && inx && r <= ny)  // y face r, between rows r-1 and r
                ys = sed_face(P, r, ny, wS, wN, pjy, pmag, pb, jy, mag, b);
            xs0 = xs; ys0 = ys;
            pjy = jy; pmag = mag; pb = b;
        }
        Y3 = Y2; Y2 = Y1;
        {  // y reconstruction of row r-1 and y face r-1 (between rows r-2 and r-1)
            const int k = r - 1;
            Flux3 f{0.0f, 0.0f, 0.0f};
            if constexpr (part_y) {
                SideQ ym, ypn;
                reconstruct<V>(P, along(v1, 1), along(v2, 1), along(v3, 1), ym, ypn);
                if (part_yface && k >= 0 && k <= ny) {  // the face row (uniform); lanes inside the grid keep it
                    side_flux<V>(P, k, ny, wS, wN, yp, ym, f.H, f.n, f.t);
                    if (!inx) f = Flux3{0.0f, 0.0f, 0.0f};
                }
                yp = ypn;
            }
            Y1 = f;
        }
        const int jr = r - 2;  // ring/tile row whose x faces and limiter are due
        X3 = X2;
        th4 = th3; th3 = th2;
        if constexpr (part_x) {
            const bool row_in = (unsigned)jr < (unsigned)ny;
            {  // x reconstruction of row r-2 and this lane's W face (west lane's plus side)
                const CellQ c = along(v1, 0);
                SideQ xm, xp;
                reconstruct<V>(P, q_prev(c), c, q_next(c), xm, xp);
                const SideQ xl{lane_prev(xp.z), lane_prev(xp.h), lane_prev(xp.ut),
                               lane_prev(xp.uLn), lane_prev(xp.uLt), lane_prev(xp.b)};
                Flux3 f;
                side_flux<V>(P, i, nx, wW, wE, xl, xm, f.H, f.n, f.t);
                const bool on = row_in && face_x;
                X2 = Flux3{on ? f.H : 0.0f, on ? f.n : 0.0f, on ? f.t : 0.0f};
            }
            {  // draining limiter of row r-2
                const float fe = lane_next(X2.H);
                th2 = (inx && row_in) ? drain_theta(P, dt, v1.h, X2.H, fe, Y2.H, Y1.H) : 1.0f;
            }
        } else {
            X2 = Flux3{0.0f, 0.0f, 0.0f};
            th2 = 1.0f;
        }
        if (upd) {  // K8 of row r-3
            CellFaces F;
            F.thW = lane_prev(th3); F.thE = lane_next(th3);
            F.xHe = lane_next(X3.H); F.xne = lane_next(X3.n); F.xte = lane_next(X3.t);
            F.Je = lane_next(xs3);
            if (mine) {
                F.th = th3; F.thS = th4; F.thN = th2;
                F.xHw = X3.H; F.xnw = X3.n; F.xtw = X3.t;
                F.yHs = Y3.H; F.yns = Y3.n; F.yts = Y3.t;
                F.yHn = Y2.H; F.ynn = Y2.n; F.ytn = Y2.t;
                F.Jw = xs3; F.Js = ys3; F.Jn = ys2;
                const float src = P.srcw ? usrc * qmid : 0.0f;
                float rbc = P.rb ? at(P.rb, uo) : 0.0f;
                float rhc = P.rh ? at(P.rh, uo) : 0.0f;
                const float ubeta = soil_at(P.beta, P.beta_s, uo);
                const CellNew o = cell_update(P, dt, F, uh, uqx, uqy, ub, uLx, uLy, src, upsi, uqb,
                                              ubeta, rbc, rhc);
                put(OH, uo, o.H); put(Oqx, uo, o.qx); put(Oqy, uo, o.qy); put(Ob, uo, o.b);
                if (P.rb) put(P.rb, uo, rbc);
                if (P.rh) put(P.rh, uo, rhc);
                if (P.ab)  // FP64 plane: twice the float plane's byte offset
                    *reinterpret_cast<double *>(reinterpret_cast<char *>(P.ab) + 2 * (size_t)uo) +=
                        (double)o.ab;
                boundary_balances(P, I.bnd, wdx, i, ju, o, F);
                float njx, njy, njm;
                cell_maxima_j(P, o.H, o.qx, o.qy, o.b, unM, ud50, upsi, mv, ms, mD, bad, njx, njy,
                              njm);
                put(I.jx[par ^ 1], uo, njx); put(I.jy[par ^ 1], uo, njy); put(I.jm[par ^ 1], uo, njm);
                if (o.H > 0.0f) wet = true;
            }
        }
    };
    // S + 6 rows: the first six and the last four unrolled with their parts
    // known at compile time, the middle S - 4 in pairs (unrolled for S = 8);
    // the loads of the row two ahead are in flight while a row is computed
    using std::integral_constant;
    constexpr int kMidUnroll = S == 8 ? 2 : 1;
    const int rlo = y0 - 3;
    Row A, B;
    load_row(rlo, A);
    load_row(rlo + 1, B);
    step(integral_constant<int, 0>{}, rlo + 0, A); load_row(rlo + 2, A);
    step(integral_constant<int, 1>{}, rlo + 1, B); load_row(rlo + 3, B);
    step(integral_constant<int, 2>{}, rlo + 2, A); load_row(rlo + 4, A);
    step(integral_constant<int, 3>{}, rlo + 3, B); load_row(rlo + 5, B);
    step(integral_constant<int, 4>{}, rlo + 4, A); load_row(rlo + 6, A);
    step(integral_constant<int, 5>{}, rlo + 5, B); load_row(rlo + 7, B);
#pragma unroll kMidUnroll
    for (int k = 6; k < S + 2; k += 2) {
        step(integral_constant<int, -1>{}, rlo + k, A);
        load_row(rlo + k + 2, A);
        step(integral_constant<int, -1>{}, rlo + k + 1, B);
        load_row(rlo + k + 3, B);
    }
    step(integral_constant<int, S + 2>{}, rlo + S + 2, A); load_row(rlo + S + 4, A);
    step(integral_constant<int, S + 3>{}, rlo + S + 3, B); load_row(rlo + S + 5, B);
    step(integral_constant<int, S + 4>{}, rlo + S + 4, A);
    step(integral_constant<int, S + 5>{}, rlo + S + 5, B);
    strip_maxima_store(I, par ^ 1, tile, mv, ms, mD, bad, wet);
}

__global__ void __launch_bounds__(RT) k_dt_t(Inst I, int par)
{
    reduce_dt(I.ctrl, par, I.A, I.tmax[par], I.ntx * I.nty);
}

// Ensemble: block m reduces member m.
__global__ void __launch_bounds__(RT) k_dt_b(const Inst *__restrict__ insts, int par)
{
    const Inst &I = insts[blockIdx.x];
    reduce_dt(I.ctrl, par, I.A, I.tmax[par], I.ntx * I.nty);
}

// Measurement only: cells the two stages of the step that read flag ring `par`
// processed (a tile runs the Lagrangian stage if wet, the Euler stage if it or
// a side neighbour is wet), added to ctrl->work.
__global__ void __launch_bounds__(RT) k_count_t(Inst I, int par, int tx, int ty)
{
    __shared__ unsigned long long red[2][RT / 64];
    unsigned long long nl = 0, ne = 0;
    const uint8_t *act = I.act[par];
    for (int t = threadIdx.x; t < I.ntx * I.nty; t += RT) {
        int bx = t % I.ntx, by = t / I.ntx;
        unsigned long long cells = (unsigned long long)(min(tx, I.P.nx - bx * tx) * min(ty, I.P.ny - by * ty));
        bool run = act[t] || (bx > 0 && act[t - 1]) || (bx + 1 < I.ntx && act[t + 1]) ||
                   (by > 0 && act[t - I.ntx]) || (by + 1 < I.nty && act[t + I.ntx]);
        if (!I.hgs) run = true;
        if (act[t] || !I.hgs) nl += cells;
        if (run) ne += cells;
    }
    for (int off = 32; off > 0; off >>= 1) {
        nl += __shfl_xor(nl, off);
        ne += __shfl_xor(ne, off);
    }
    if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = nl; red[1][threadIdx.x >> 6] = ne; }
    __syncthreads();
    if (threadIdx.x == 0 && !I.ctrl->err) {
        for (int w = 1; w < RT / 64; ++w) { nl += red[0][w]; ne += red[1][w]; }
        I.ctrl->work[0] += nl;
        I.ctrl->work[1] += ne;
    }
}

// Single grid: tile = block index.
template <int TX, int TY>
__global__ void __launch_bounds__(NT) k_prepare_t(Inst I, int par)
{
    prepare_tile<TX, TY>(I, par, blockIdx.x, blockIdx.y);
}
template <int TX, int TY>
__global__ void __launch_bounds__(NT) k_lagrange_t(Inst I, int par)
{
    lagrange_tile<TX, TY>(I, par, blockIdx.x, blockIdx.y);
}
template <int TX, int TY>
__global__ void __launch_bounds__(NT) k_euler_t(Inst I, int par)
{
    euler_tile<TX, TY>(I, par, blockIdx.x, blockIdx.y);
}

// Ensemble: block b handles tile (table[3b+1], table[3b+2]) of member table[3b].
template <int TX, int TY>
__global__ void __launch_bounds__(NT) k_lagrange_b(const Inst *__restrict__ insts,
                                                   const int *__restrict__ table, int par)
{
    const int *t = table + 3 * blockIdx.x;
    lagrange_tile<TX, TY>(insts[t[0]], par, t[1], t[2]);
}
template <int TX, int TY>
__global__ void __launch_bounds__(NT) k_euler_b(const Inst *__restrict__ insts,
                                                const int *__restrict__ table, int par)
{
    const int *t = table + 3 * blockIdx.x;
    euler_tile<TX, TY>(insts[t[0]], par, t[1], t[2]);
}

// ---------------------------------------------------------------------------
// Work lists (strips on a single grid).  Launching one workgroup per tile
// leaves the wet tiles scattered among dry ones, so some CUs get twice the
// average work.  Instead K3 compacts, in tile order, the tiles whose
// Lagrangian stage runs (wet or forced) and those whose Euler stage runs (wet
// or a side neighbour wet), plus one copy entry for each newly dry tile whose
// two buffer levels still differ; it also gives every tile left out zero
// maxima and a dry flag for the next state.  The stage kernels then run one
// wavefront per list entry: the listed tiles are dispatched first and
// back-to-back, so the hardware spreads them evenly over the CUs.
// ---------------------------------------------------------------------------

// Wave64 inclusive prefix sum (all lanes active): DPP row shifts by 1, 2, 4
// and 8 (a lane without a source in its row of 16 adds 0) give the sum
// within each row; the totals of the rows below are added from lanes 15, 31
// and 47 as scalars.
template <int CTRL>
__device__ __forceinline__ int dpp_add_shifted(int x)
{
    return x + __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, true);
}
__device__ __forceinline__ int wave_scan(int v)
{
    v = dpp_add_shifted<0x111>(v);
    v = dpp_add_shifted<0x112>(v);
    v = dpp_add_shifted<0x114>(v);
    v = dpp_add_shifted<0x118>(v);
    const int row = (threadIdx.x & 63) >> 4;
    const int t0 = __builtin_amdgcn_readlane(v, 15), t1 = __builtin_amdgcn_readlane(v, 31);
    const int t2 = __builtin_amdgcn_readlane(v, 47);
    return v + (row >= 1 ? t0 : 0) + (row >= 2 ? t1 : 0) + (row >= 3 ? t2 : 0);
}

// K3 for strips (nchunk workgroups): workgroup b reduces the Eq. 7 maxima of
// its tiles and, under dry-tile skipping, writes its segment of each list,
// each thread classifying a contiguous run of tiles so that entries come out
// in tile order.  The segments are combined by the Lagrangian kernel that
// follows (the kernel boundary makes these writes visible): every wavefront
// derives its entry and the Eq. 7 step from the segment lengths and maxima,
// and wavefront 0 publishes the step and the Euler list's start positions.
// A list workgroup has list_threads(chunk) threads, at most LT.
constexpr int LT = 1024;
__device__ void dt_lists(const Inst &I, int par, int b)
{
    __shared__ unsigned red[4][LT / 64];
    __shared__ int wl[LT / 64], we[LT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nthr = blockDim.x, nw = nthr >> 6;
    const int nt = I.ntx * I.nty;
    const int c0 = b * I.chunk, c1 = min(nt, c0 + I.chunk);
    const int ntx = I.ntx, nty = I.nty;
    const uint8_t *act = I.act[par];
    const uint8_t *synced = I.synced;
    const uint4 *tm = I.tmax[par];
    const int per = (c1 - c0 + nthr - 1) / nthr;  // at most 32 (chunk <= 32 threads)
    const int t0 = min(c1, c0 + tid * per), t1 = min(c1, t0 + per);
    // every load first: the tiles' maxima and (under skipping) the five wet
    // flags and the synced flag of each tile of this thread's run
    unsigned a = 0, bb = 0, c = 0, bad = 0;
    unsigned m_act = 0u, m_run = 0u, m_copy = 0u;
    int bx = t0 % ntx, by = t0 / ntx;
    for (int t = t0; t < t1; ++t) {
        const uint4 v = tm[t];
        a = max(a, v.x); bb = max(bb, v.y); c = max(c, v.z); bad = max(bad, v.w);
        if (I.hgs) {
            const unsigned fa = act[t], fw = act[bx > 0 ? t - 1 : t], fe = act[bx + 1 < ntx ? t + 1 : t];
            const unsigned fs = act[by > 0 ? t - ntx : t], fn = act[by + 1 < nty ? t + ntx : t];
            const unsigned sy = synced[t];
            const int q = t - t0;
            const bool r = (fa | fw | fe | fs | fn) != 0;
            m_act |= (unsigned)(fa != 0) << q;
            m_run |= (unsigned)r << q;
            m_copy |= (unsigned)(!r && !sy) << q;
        }
        if (++bx == ntx) { bx = 0; ++by; }
    }
    // wave maxima and wave prefix sums of the list counts, one barrier
    const int nl = __popc(m_act), ne = __popc(m_run | m_copy);
    const int il = wave_scan(nl), ie = wave_scan(ne);
    a = wave_max_u32(a); bb = wave_max_u32(bb); c = wave_max_u32(c); bad = wave_max_u32(bad);
    if (lane == 63) { wl[wv] = il; we[wv] = ie; }
    if (lane == 0) { red[0][wv] = a; red[1][wv] = bb; red[2][wv] = c; red[3][wv] = bad; }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < nw; ++w) {
            a = max(a, red[0][w]); bb = max(bb, red[1][w]); c = max(c, red[2][w]); bad = max(bad, red[3][w]);
        }
        I.part[b] = make_uint4(a, bb, c, bad);
    }
    if (!I.hgs) return;
    int ol = il - nl, oe = ie - ne, tl = 0, te = 0;
    for (int k = 0; k < nw; ++k) {
        if (k < wv) { ol += wl[k]; oe += we[k]; }
        tl += wl[k]; te += we[k];
    }
    uint8_t *act_next = I.act[par ^ 1];
    uint4 *tm_next = I.tmax[par ^ 1];
    uint8_t *synced_w = I.synced;
    int *lag = I.lag + c0, *eul = I.eul + c0;
    for (int t = t0; t < t1; ++t) {
        const unsigned bit = 1u << (t - t0);
        if (m_act & bit) lag[ol++] = t;
        if (m_run & bit) {
            eul[oe++] = t;
            synced_w[t] = 0;
        } else {
            if (m_copy & bit) {
                eul[oe++] = -1 - t;
                synced_w[t] = 1;
            }
            act_next[t] = 0;
            tm_next[t] = make_uint4(0u, 0u, 0u, 0u);
        }
    }
    if (tid == 0) {
        I.cnt_l[b] = tl;
        I.cnt_e[b] = te;
    }
}

__global__ void __launch_bounds__(LT) k_dt_lists(Inst I, int par) { dt_lists(I, par, blockIdx.x); }

// Ensemble: workgroup b runs segment table[2b+1] of member table[2b].
__global__ void __launch_bounds__(LT) k_dt_lists_b(const Inst *__restrict__ insts,
                                                   const int *__restrict__ table, int par)
{
    dt_lists(insts[table[2 * blockIdx.x]], par, table[2 * blockIdx.x + 1]);
}

// Entry w of a list kept in segments: the segment is the last one whose
// start position is <= w (one ballot per 64 segments).
// p0: this lane's start position in the first group of 64, loaded by the caller.
__device__ __forceinline__ int list_entry(const int *seg, const int *pre, int p0, int nb, int chunk,
                                          int w)
{
    const int lane = threadIdx.x & 63;
    int b = -1;
    for (int g = 0; g < nb; g += 64) {
        const int k = g + lane;
        const unsigned long long le = __ballot(k < nb && (g == 0 ? p0 : pre[k]) <= w);
        b += __popcll(le);
        if (le != ~0ull) break;
    }
    return seg[b * chunk + (w - pre[b])];
}

// Bring the other buffer level of a dry strip tile to the current state.
template <int S>
__device__ void strip_copy(const Inst &I, int par, int bx, int by)
{
    const int lane = threadIdx.x & 63;
    const int i = bx * SX + lane;
    if (lane >= SX || i >= I.P.nx) return;
    const int y0 = by * S, jend = min(y0 + S, I.P.ny);
    for (int j = y0; j < jend; ++j) {
        const int c = j * I.P.pitch + i;
        I.H[par ^ 1][c] = I.H[par][c];
        I.qx[par ^ 1][c] = I.qx[par][c];
        I.qy[par ^ 1][c] = I.qy[par][c];
        I.b[par ^ 1][c] = I.b[par][c];
        I.jx[par ^ 1][c] = I.jx[par][c];
        I.jy[par ^ 1][c] = I.jy[par][c];
        I.jm[par ^ 1][c] = I.jm[par][c];
    }
}

// Strip stages over the step's lists: wavefront w takes entry w (tile w when
// nothing is skipped).  The grid covers the longest possible list; the
// listed tiles come first in dispatch order and the waves past the end of
// the list leave at once.
// Start position of every segment of a list from the segment lengths (one
// wave scan per 64 segments): returns the list length; *seg / *start receive
// the segment holding entry w and its start (when w is below the length).
// c0: this lane's length in the first group of 64 segments, loaded by the caller.
__device__ __forceinline__ int list_locate(const int *cnt, int c0, int nb, int w, int &seg,
                                           int &start, int *pre_out)
{
    const int lane = threadIdx.x & 63;
    int base = 0;
    seg = 0;
    start = 0;
    for (int g = 0; g < nb; g += 64) {
        const int k = g + lane;
        const int c = g == 0 ? c0 : (k < nb ? cnt[k] : 0);
        const int inc = wave_scan(c);
        const int st = base + inc - c;
        if (pre_out && k < nb) pre_out[k] = st;
        const unsigned long long le = __ballot(k < nb && st <= w);
        if (le) {
            const int j = 63 - __clzll(le);  // the set lanes are a prefix (starts never decrease)
            seg = g + j;
            start = __builtin_amdgcn_readlane(st, j);
        }
        base += __builtin_amdgcn_readlane(inc, 63);
    }
    return base;
}

// Workgroups are dispatched to the 8 XCDs in turn (workgroup b to XCD b % 8).
// Of the nwg workgroups a list needs, XCD x instead takes one contiguous run
// of the list, so tiles that are neighbours along y (and the halo rows they
// both read) mostly meet in the same L2.  A bijection of [0, nwg): XCD x
// holds q + (x < r) of them (nwg = 8 q + r), starting at x q + min(x, r).
__device__ __forceinline__ int xcd_block(int b, int nwg)
{
    const int q = nwg >> 3, r = nwg & 7, x = b & 7, k = b >> 3;
    return x * q + min(x, r) + k;
}
// Entry of wavefront wave of workgroup b for a list of n entries.
__device__ __forceinline__ int xcd_entry(int b, int wave, int n)
{
    const int nwg = (n + SWAVES - 1) / SWAVES;
    return b < nwg ? xcd_block(b, nwg) * SWAVES + wave : b * SWAVES + wave;
}

// The entry index and the tile it names are the same in every lane of the
// wavefront; readfirstlane states that, so tile coordinates and the row
// ranges derived from them live in scalar registers and branch as scalars.
// How a wavefront finds its list entry from w:
//   XP = 0: w is the entry itself (ensembles: one wavefront per entry);
//   XP = 1: w = blockIdx.x * SWAVES + wave of a single grid whose stage grid
//           has a wavefront per possible entry; spread over the XCDs once the
//           list length is known;
//   XP = 2: as 1, for grids with dry tiles skipped and more tiles than
//           kMaxStageGroups workgroups hold: the grid's G4 = gridDim.x * SWAVES
//           wavefronts take the list in passes of at most G4 entries, each
//           pass spread over the XCDs;
//   XP = 3: (Lagrangian stage) as 1 with one wavefront per kLagGroup
//           vertically stacked tiles, for grids of more tiles than that with
//           every tile listed: they fill the chip, and the taller strips
//           spare the halo rows the halves and single tiles add.
// (XP = 2 is a kernel of its own: the pass loop costs the Euler kernel
// registers, and with them a wavefront per SIMD, that XP = 1 keeps.)
template <int S, bool CS, int XP, bool F2>
__device__ __forceinline__ void lagrange_listed(const Inst &I, int par, int w)
{
    w = __builtin_amdgcn_readfirstlane(w);
    Ctrl *ctrl = I.ctrl;
    const int lane = threadIdx.x & 63;
    const bool publisher = w == 0;
    const int nb = I.nchunk;
    // the error flag and the first 64 segment lengths and maxima are loaded
    // together, before any of them is used (one round trip, not three)
    const int err = ctrl->err;
    const int cl0 = I.hgs && lane < nb ? I.cnt_l[lane] : 0;
    const int ce0 = I.hgs && publisher && lane < nb ? I.cnt_e[lane] : 0;
    uint4 v = lane < nb ? I.part[lane] : make_uint4(0u, 0u, 0u, 0u);
    // XP = 3: entries are groups of kLagGroup stacked tiles (every tile listed)
    int n = XP == 3 ? I.ntx * ((I.nty + kLagGroup - 1) / kLagGroup) : I.ntx * I.nty;
    int seg = 0, start = 0;
    const int G4 = XP == 2 ? (int)gridDim.x * SWAVES : 0;
    // XP = 1, 2: LH wavefronts per listed tile, each on S / LH of its rows
    constexpr int LH = XP == 1 || XP == 2 ? kLagHalves : 1;
    if (XP && I.hgs) n = list_locate(I.cnt_l, cl0, nb, 0, seg, start, nullptr);
    if (XP == 1 || XP == 3)
        w = __builtin_amdgcn_readfirstlane(xcd_entry(w / SWAVES, w % SWAVES, LH * n));
    const int part = w % LH;
    if (XP != 2) w /= LH;
    if (XP != 2 && I.hgs) n = list_locate(I.cnt_l, cl0, nb, w, seg, start, nullptr);
    // XP = 2: LH wavefronts per entry when the list is short enough for one
    // pass of them (the launch's idle wavefronts take the halves), else one;
    // workgroups past those the first (fullest) pass needs have no entry
    const int lh = XP == 2 && LH * n <= G4 ? LH : 1;
    const bool idle = XP == 2 ? w / SWAVES >= (min(G4, lh * n) + SWAVES - 1) / SWAVES : w >= n;
    if (idle && !publisher) return;
    // the Eq. 7 step from the segment maxima (K3 proper)
    unsigned a = v.x, b = v.y, c = v.z, bad = v.w;
    for (int g = 64; g < nb; g += 64) {
        v = g + lane < nb ? I.part[g + lane] : make_uint4(0u, 0u, 0u, 0u);
        a = max(a, v.x); b = max(b, v.y); c = max(c, v.z); bad = max(bad, v.w);
    }
    const uint4 m = make_uint4(wave_max_u32(a), wave_max_u32(b), wave_max_u32(c), wave_max_u32(bad));
    if (publisher) {
        if (I.hgs) {  // start positions of the Euler list for the Euler kernel
            int s0, s1;
            const int ne = list_locate(I.cnt_e, ce0, nb, 0, s0, s1, I.pre_e);
            if (lane == 0) I.totals[1] = ne;
        }
        if (lane == 0) publish_dt(ctrl, par, I.A, m);
    }
    const Eq7 e = eq7_step(I.A, m);
    if (err || e.err) return;
    const float dt = (float)e.dt;
    if (XP != 2) {
        if (w >= n) return;
        const int t = __builtin_amdgcn_readfirstlane(I.hgs ? I.lag[seg * I.chunk + (w - start)] : w);
        if constexpr (XP == 3) {  // a group of stacked tiles as one strip
            if constexpr (F2) lagrange_strip2<S * kLagGroup, CS>(I, par, t % I.ntx, t / I.ntx, dt);
            else lagrange_strip<S * kLagGroup, CS>(I, par, t % I.ntx, t / I.ntx, dt);
        } else {
            if constexpr (F2) lagrange_strip2<S / LH, CS>(I, par, t % I.ntx, (t / I.ntx) * LH + part, dt);
            else lagrange_strip<S / LH, CS>(I, par, t % I.ntx, (t / I.ntx) * LH + part, dt);
        }
        return;
    }
    if (lh > 1) {  // one pass: wavefront w takes part w % LH of entry w / LH
        const int wi = __builtin_amdgcn_readfirstlane(xcd_entry(w / SWAVES, w % SWAVES, LH * n));
        if (wi >= LH * n) return;
        const int we = wi / LH, pt = wi % LH;
        if (I.hgs) list_locate(I.cnt_l, cl0, nb, we, seg, start, nullptr);
        const int t = __builtin_amdgcn_readfirstlane(I.hgs ? I.lag[seg * I.chunk + (we - start)] : we);
        if constexpr (F2) lagrange_strip2<S / LH, CS>(I, par, t % I.ntx, (t / I.ntx) * LH + pt, dt);
        else lagrange_strip<S / LH, CS>(I, par, t % I.ntx, (t / I.ntx) * LH + pt, dt);
        return;
    }
    for (int base = 0; base < n; base += G4) {
        const int cnt = min(G4, n - base);
        const int we = __builtin_amdgcn_readfirstlane(base + xcd_entry(w / SWAVES, w % SWAVES, cnt));
        if (we >= base + cnt) continue;
        if (I.hgs) list_locate(I.cnt_l, cl0, nb, we, seg, start, nullptr);
        const int t = __builtin_amdgcn_readfirstlane(I.hgs ? I.lag[seg * I.chunk + (we - start)] : we);
        if constexpr (F2) lagrange_strip2<S, CS>(I, par, t % I.ntx, t / I.ntx, dt);
        else lagrange_strip<S, CS>(I, par, t % I.ntx, t / I.ntx, dt);
    }
}
template <int S, bool CS, bool V>
__device__ __forceinline__ void euler_entry(const Inst &I, int par, int p0, int w)
{
    const int e = __builtin_amdgcn_readfirstlane(
        I.hgs ? list_entry(I.eul, I.pre_e, p0, I.nchunk, I.chunk, w) : w);
    const int t = e < 0 ? -1 - e : e;
    if (e < 0) strip_copy<S>(I, par, t % I.ntx, t / I.ntx);
    else euler_strip<S, CS, V>(I, par, t % I.ntx, t / I.ntx);
}
template <int S, bool CS, int XP, bool V>
__device__ __forceinline__ void euler_listed(const Inst &I, int par, int w)
{
    // error flag, list length and the first 64 start positions in one round trip
    w = __builtin_amdgcn_readfirstlane(w);
    const int lane = threadIdx.x & 63;
    const int err = I.ctrl->err;
    const int n = I.hgs ? I.totals[1] : I.ntx * I.nty;
    const int p0 = I.hgs && lane < I.nchunk ? I.pre_e[lane] : 0;
    if (XP != 2) {
        if (XP == 1) w = __builtin_amdgcn_readfirstlane(xcd_entry(w / SWAVES, w % SWAVES, n));
        if (err || w >= n) return;
        euler_entry<S, CS, V>(I, par, p0, w);
        return;
    }
    if (err) return;
    const int G4 = (int)gridDim.x * SWAVES;
    for (int base = 0; base < n; base += G4) {
        const int cnt = min(G4, n - base);
        const int we = __builtin_amdgcn_readfirstlane(base + xcd_entry(w / SWAVES, w % SWAVES, cnt));
        if (we >= base + cnt) {
            if (base == 0) return;  // no entry in the first (fullest) pass: none later
            continue;
        }
        euler_entry<S, CS, V>(I, par, p0, we);
    }
}

// F2: the second-order force (lagrange_strip2).
template <int S, bool CS, int XP, bool F2>
__global__ void __launch_bounds__(NT) k_lagrange_sl(Inst I, int par)
{
    lagrange_listed<S, CS, XP, F2>(I, par, blockIdx.x * SWAVES + (threadIdx.x >> 6));
}
// V: the limiter or the wave-speed estimate is not minmod + Davis (read from
// the run's constants); V = false keeps the default arithmetic branch-free.
template <int S, bool CS, int XP, bool V>
__global__ void __launch_bounds__(NT) k_euler_sl(Inst I, int par)
{
    euler_listed<S, CS, XP, V>(I, par, blockIdx.x * SWAVES + (threadIdx.x >> 6));
}

// Ensemble: workgroup b runs waves SWAVES table[2b+1] + w of member table[2b].
template <int S, bool CS, bool F2>
__global__ void __launch_bounds__(NT) k_lagrange_slb(const Inst *__restrict__ insts,
                                                     const int *__restrict__ table, int par)
{
    const int *t = table + 2 * blockIdx.x;
    lagrange_listed<S, CS, 0, F2>(insts[t[0]], par, t[1] * SWAVES + (threadIdx.x >> 6));
}
template <int S, bool CS, bool V>
__global__ void __launch_bounds__(NT) k_euler_slb(const Inst *__restrict__ insts,
                                                  const int *__restrict__ table, int par)
{
    const int *t = table + 2 * blockIdx.x;
    euler_listed<S, CS, 0, V>(insts[t[0]], par, t[1] * SWAVES + (threadIdx.x >> 6));
}

// Tile shapes the autotuner chooses from: TX x TY cells per 256-thread
// workgroup (LDS tiles), or SX x S cells per wavefront (strips, TX = SX).
struct Shape {
    int tx, ty;
};
constexpr Shape kShapes[] = {{64, 8}, {64, 4}, {64, 16}, {128, 4}, {SX, 8}, {SX, 16}, {SX, 32}};
constexpr int kNumShapes = 7;
constexpr bool is_strip(int shape) { return kShapes[shape].tx == SX; }
constexpr int kDefaultShape = 4;  // 58 x 8 strips

// ---------------------------------------------------------------------------
// FP64 sums: water volume, sediment volume, wet cells (two fixed-order passes).
// ---------------------------------------------------------------------------

constexpr int SUM_THREADS = 256;

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    return v;
}

__global__ void __launch_bounds__(SUM_THREADS) k_sums1(KPar P, const float *__restrict__ H,
                                                       const float *__restrict__ b,
                                                       double *__restrict__ part, int rows_per_block)
{
    __shared__ double sh[4][SUM_THREADS / 64];
    double sw = 0.0, ss = 0.0, wet = 0.0, ab = 0.0;
    int j0 = blockIdx.x * rows_per_block, j1 = min(P.ny, j0 + rows_per_block);
    for (int j = j0; j < j1; ++j)
        for (int i = threadIdx.x; i < P.nx; i += SUM_THREADS) {
            int c = j * P.pitch + i;
            float h = H[c];
            // the accumulated depth: the stored float plus its rainfall residual
            sw += (double)h + (P.rh ? (double)P.rh[c] : 0.0);
            // the accumulated bed: the stored float plus its residual
            const double bc = (double)b[c] + (P.rb ? (double)P.rb[c] : 0.0);
            ss += (1.0 - (double)soil(P.psi, P.psi_s, c)) * bc;
            wet += h > 0.0f ? 1.0 : 0.0;
            if (P.ab) ab += P.ab[c];
        }
    sw = wave_sum(sw); ss = wave_sum(ss); wet = wave_sum(wet); ab = wave_sum(ab);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sh[0][w] = sw; sh[1][w] = ss; sh[2][w] = wet; sh[3][w] = ab; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < SUM_THREADS / 64; ++k) {
            sw += sh[0][k]; ss += sh[1][k]; wet += sh[2][k]; ab += sh[3][k];
        }
        part[4 * blockIdx.x + 0] = sw;
        part[4 * blockIdx.x + 1] = ss;
        part[4 * blockIdx.x + 2] = wet;
        part[4 * blockIdx.x + 3] = ab;
    }
}

// Sum of npart partial quadruples and of the boundary accumulators, in a fixed order.
__global__ void __launch_bounds__(SUM_THREADS) k_sums2(const double *__restrict__ part, int npart,
                                                       const double *__restrict__ bnd, int nb,
                                                       double *__restrict__ out)
{
    __shared__ double sh[6][SUM_THREADS / 64];
    double a = 0, b = 0, c = 0, d = 0, e = 0, f = 0;
    for (int k = threadIdx.x; k < npart; k += SUM_THREADS) {
        a += part[4 * k]; b += part[4 * k + 1]; c += part[4 * k + 2]; f += part[4 * k + 3];
    }
    for (int k = threadIdx.x; k < nb; k += SUM_THREADS) { d += bnd[k]; e += bnd[nb + k]; }
    a = wave_sum(a); b = wave_sum(b); c = wave_sum(c); d = wave_sum(d); e = wave_sum(e); f = wave_sum(f);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = a; sh[1][w] = b; sh[2][w] = c; sh[3][w] = d; sh[4][w] = e; sh[5][w] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < SUM_THREADS / 64; ++k) {
            a += sh[0][k]; b += sh[1][k]; c += sh[2][k]; d += sh[3][k]; e += sh[4][k]; f += sh[5][k];
        }
        out[0] = a; out[1] = b; out[2] = c; out[3] = d; out[4] = e; out[5] = f;
    }
}

}  // namespace

// ===========================================================================
// Host side
// ===========================================================================

struct sw_ctx {
    sw_grid grid{};
    sw_params par{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int nx = 0, ny = 0, pitch = 0;
    size_t plane = 0;                // floats per pitched plane
    float *buf = nullptr;            // all pitched planes in one allocation
    float *H[2]{}, *qx[2]{}, *qy[2]{}, *b[2]{};
    float *QLx = nullptr, *QLy = nullptr;
    float *jx[2]{}, *jy[2]{}, *jm[2]{};  // J0 and |J0| per buffer level
    float *rb = nullptr;             // bed residual of the compensated Exner update
    float *nM = nullptr, *d50 = nullptr, *psi = nullptr, *qb = nullptr, *srcw = nullptr;
    float nM_s = 0.0f, d50_s = 5e-4f, psi_s = 0.4f;
    // forcing: rainfall, absorption (per-cell plane or scalar), Coriolis, wind
    double rain = 0.0, coriolis = 0.0, wind_x = 0.0, wind_y = 0.0, wind_coef = 0.0;
    float *beta = nullptr;
    float beta_s = 0.0f;
    double *ab = nullptr;            // absorbed depth per cell (FP64, pitched), with absorption
    float *rh = nullptr;             // depth residual of the compensated rainfall, with rain
    float *faces = nullptr;          // unfused face arrays
    double *bnd = nullptr;           // boundary accumulators: water [2(nx+ny)], sediment [2(nx+ny)]
    double *part = nullptr;          // sum partials
    double *sums = nullptr;          // sum results (device)
    Ctrl *ctrl = nullptr;
    int64_t k = 0;                   // steps since the state was set
    int64_t step0 = 0;               // step counter offset (sw_set_time)
    double t0 = 0.0;                 // time at k = 0
    bool have_state = false, dirty = true;
    unsigned *bound_slot = nullptr;  // NSLOT x 4 maxima of sw_step_bound
    StepRec *steplog = nullptr;      // the step log ring (kStepLog records)
    int has_inflow = 0;
    double q_base = 0, q_peak = 0, t_peak = 0, t_sigma = 1;
    double qb_total = 0.0;
    int nsum_blocks = 0, sum_rows = 1;
    int ntx = 0, nty = 0;            // tile grid of the tiled kernels
    uint8_t *tflags = nullptr;       // act[2][ntiles], synced[ntiles], force[ntiles]
    hipStream_t cap = nullptr;       // private stream used only to capture graphs
    // pinned host staging of one plane (hipHostMalloc, on first use): every
    // transfer of a field between the host and the device goes through it,
    // so the runtime never has to pin pageable user memory on the fly
    float *stage = nullptr;
    size_t stage_bytes = 0;
    // asynchronous Save: a device snapshot of the state, copied to pinned host
    // memory on a second stream while the steps go on
    float *snap = nullptr;           // 4 pitched planes h, hu, hv, b
    Ctrl *snap_ctrl = nullptr;       // the control block at the snapshot (device)
    float *snap_host = nullptr;      // pinned: 4 dense planes, then the control block
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_snap = nullptr, ev_copied = nullptr;
    bool save_pending = false;
    int64_t save_k = 0;
    hipGraphExec_t gexec = nullptr;  // two tiled steps (even k, then odd k)
    hipGraphExec_t gexec_long = nullptr;  // kLongPairs such pairs
    bool graph_ok = false;           // false once a kernel argument changed (soil, sources, shape)
    int64_t graph_builds = 0;        // graph pairs captured and instantiated so far
    uint64_t args_gen = 0;           // bumped whenever a kernel argument changes
    std::vector<int32_t> forced_in, forced_qb;  // inflow / bed-source cells (flat indices)
    int shape = kDefaultShape;       // index into kShapes
    size_t max_tiles = 0;            // tile count of the smallest shape (flag capacity)
    uint4 *tmax = nullptr;           // per-tile Eq. 7 maxima, two rings of max_tiles
    int *sched = nullptr;            // work lists of the strip kernels (layout: sched_layout)
    int max_chunks = 0;              // list segments of the largest tile grid
    int graph_fixed = 0;
    double graph_dt = 0.0;
    std::string err;
};

namespace {

int fail(sw_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                              \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail((ctx), SW_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

KPar make_kpar(const sw_ctx *c)
{
    KPar P{};
    P.nx = c->nx; P.ny = c->ny; P.pitch = c->pitch;
    P.bcW = c->grid.bc[0]; P.bcE = c->grid.bc[1]; P.bcS = c->grid.bc[2]; P.bcN = c->grid.bc[3];
    P.dx = (float)c->grid.dx;
    P.inv_dx = (float)(1.0 / c->grid.dx);
    P.g = (float)c->par.g;
    P.eps = (float)c->par.eps_dry;
    P.eps4 = (float)(c->par.eps_dry * c->par.eps_dry * c->par.eps_dry * c->par.eps_dry);
    P.h_sed = (float)c->par.h_sed;
    P.s_rel_m1 = (float)(c->par.s_rel - 1.0);
    P.C_J = (float)c->par.C_J; P.C_Sh = (float)c->par.C_Sh;
    P.A_G = (float)c->par.A_G; P.m_exp = (float)c->par.m_exp;
    P.half_g_inv_dx = (float)(c->par.g / (2.0 * c->grid.dx));
    P.sed_law = c->par.sed_law;
    P.nM = c->nM; P.nM_s = c->nM_s;
    P.d50 = c->d50; P.d50_s = c->d50_s;
    P.psi = c->psi; P.psi_s = c->psi_s;
    P.qb = c->qb;
    P.srcw = c->has_inflow ? c->srcw : nullptr;
    P.rb = (c->par.sed_law != SW_SED_NONE || c->qb) ? c->rb : nullptr;
    // limiter as the bounds of its slope ratio (beta, theta, gamma)
    P.lim_b = P.lim_t = P.lim_g = 1.0f;
    if (c->par.limiter == SW_LIM_MC) { P.lim_b = 2.0f; P.lim_t = 2.0f; P.lim_g = 0.5f; }
    if (c->par.limiter == SW_LIM_SUPERBEE) { P.lim_b = 2.0f; P.lim_t = 2.0f; P.lim_g = 1.0f; }
    P.speeds = c->par.hll_speeds;
    P.rain = (float)c->rain;
    P.beta = c->beta;
    P.beta_s = c->beta_s;
    P.ab = c->ab;
    P.rh = c->rh;
    P.cor = (float)c->coriolis;
    const double wm = std::sqrt(c->wind_x * c->wind_x + c->wind_y * c->wind_y);
    P.wsx = (float)(c->wind_coef * wm * c->wind_x);
    P.wsy = (float)(c->wind_coef * wm * c->wind_y);
    P.inv_hsed = (float)(1.0 / c->par.h_sed);
    P.force = (c->coriolis != 0.0 || P.wsx != 0.0f || P.wsy != 0.0f) ? 1 : 0;
    P.variant = (c->par.limiter != SW_LIM_MINMOD || c->par.hll_speeds != SW_HLL_DAVIS) ? 1 : 0;
    P.force2 = (c->par.flags & SW_FLAG_FORCE2) ? 1 : 0;
    return P;
}

StepArgs make_step_args(const sw_ctx *c, int fixed, double dt)
{
    StepArgs A{};
    A.mode_fixed = fixed;
    A.dt_fixed = dt;
    A.dx = c->grid.dx; A.cfl = c->par.cfl; A.dt_max = c->par.dt_max; A.dt_min = c->par.dt_min;
    A.has_inflow = c->has_inflow;
    A.q_base = c->q_base; A.q_peak = c->q_peak; A.t_peak = c->t_peak; A.t_sigma = c->t_sigma;
    A.qb_total = c->qb_total;
    A.rain_area = c->rain * (double)c->nx * (double)c->ny * c->grid.dx * c->grid.dx;
    A.log = c->steplog;
    return A;
}

// The staging holds at least `bytes` (and at least one plane) afterwards.
int ensure_stage(sw_ctx *c, size_t bytes)
{
    bytes = std::max(bytes, c->plane * sizeof(float));
    if (c->stage_bytes >= bytes) return SW_OK;
    if (c->stage) (void)hipHostFree(c->stage);
    if (c->copy_stream) (void)hipStreamSynchronize(c->copy_stream);
    (void)hipFree(c->snap);
    (void)hipFree(c->snap_ctrl);
    if (c->snap_host) (void)hipHostFree(c->snap_host);
    if (c->ev_snap) (void)hipEventDestroy(c->ev_snap);
    if (c->ev_copied) (void)hipEventDestroy(c->ev_copied);
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    c->stage = nullptr;
    c->stage_bytes = 0;
    HIPCHK(c, hipHostMalloc((void **)&c->stage, bytes, hipHostMallocDefault));
    c->stage_bytes = bytes;
    return SW_OK;
}

// Host bytes -> device, through the pinned staging (at most one plane).
int stage_to_device(sw_ctx *c, void *dst, const void *src, size_t bytes)
{
    int rc = ensure_stage(c, bytes);
    if (rc) return rc;
    std::memcpy(c->stage, src, bytes);
    HIPCHK(c, hipMemcpyAsync(dst, c->stage, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SW_OK;
}

// Device bytes -> host (ordered after the work on the stream), through the staging.
int stage_to_host(sw_ctx *c, void *dst, const void *src, size_t bytes)
{
    int rc = ensure_stage(c, bytes);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(c->stage, src, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::memcpy(dst, c->stage, bytes);
    return SW_OK;
}

// Copy a user [ny][nx] array (host or device) into a pitched device plane.
int upload_plane(sw_ctx *c, float *dst, const float *src, int ptr_kind)
{
    if (ptr_kind == SW_PTR_HOST) {
        int rc = ensure_stage(c, 0);
        if (rc) return rc;
        std::memcpy(c->stage, src, (size_t)c->nx * c->ny * sizeof(float));
        HIPCHK(c, hipMemcpy2DAsync(dst, c->pitch * sizeof(float), c->stage, c->nx * sizeof(float),
                                   c->nx * sizeof(float), c->ny, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else if (ptr_kind == SW_PTR_DEVICE) {
        HIPCHK(c, hipMemcpy2DAsync(dst, c->pitch * sizeof(float), src, c->nx * sizeof(float),
                                   c->nx * sizeof(float), c->ny, hipMemcpyDeviceToDevice, c->stream));
    } else {
        return fail(c, SW_ERR_ARG, "ptr_kind must be SW_PTR_HOST or SW_PTR_DEVICE");
    }
    return SW_OK;
}

int download_plane(sw_ctx *c, float *dst, const float *src, int ptr_kind)
{
    if (ptr_kind != SW_PTR_HOST && ptr_kind != SW_PTR_DEVICE)
        return fail(c, SW_ERR_ARG, "ptr_kind must be SW_PTR_HOST or SW_PTR_DEVICE");
    if (ptr_kind == SW_PTR_DEVICE) {
        HIPCHK(c, hipMemcpy2DAsync(dst, c->nx * sizeof(float), src, c->pitch * sizeof(float),
                                   c->nx * sizeof(float), c->ny, hipMemcpyDeviceToDevice, c->stream));
        return SW_OK;
    }
    int rc = ensure_stage(c, 0);
    if (rc) return rc;
    HIPCHK(c, hipMemcpy2DAsync(c->stage, c->nx * sizeof(float), src, c->pitch * sizeof(float),
                               c->nx * sizeof(float), c->ny, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::memcpy(dst, c->stage, (size_t)c->nx * c->ny * sizeof(float));
    return SW_OK;
}

dim3 cell_grid(const sw_ctx *c) { return dim3((c->nx + BX - 1) / BX, (c->ny + BY - 1) / BY); }

size_t ntiles(const sw_ctx *c) { return (size_t)c->ntx * c->nty; }

// Tiles per K3 workgroup (list segment) for nt tiles: at least 256, at most
// 32 LT (one 32-bit mask per thread), and at most 64 segments where possible.
int list_chunk(int nt) { return std::min(32 * LT, std::max(256, (nt + 63) / 64)); }
// Threads of the workgroup that lists a segment of chunk tiles: one tile per
// thread up to LT threads (small segments: short dependency chains in many
// small workgroups; large ones: at most 32 tiles per thread).
int list_threads(int chunk) { return std::min(LT, std::max(256, (chunk + 63) / 64 * 64)); }

// Offsets (in ints) of the parts of the work-list buffer.
struct SchedLayout {
    size_t totals, cnt_l, cnt_e, pre_l, pre_e, part, lag, eul, total;
};
SchedLayout sched_layout(int nchunks, size_t tiles)
{
    SchedLayout L;
    L.totals = 0;
    L.cnt_l = 4;
    L.cnt_e = L.cnt_l + nchunks;
    L.pre_l = L.cnt_e + nchunks;
    L.pre_e = L.pre_l + nchunks + 1;
    L.part = (L.pre_e + nchunks + 1 + 3) / 4 * 4;  // uint4 aligned
    L.lag = L.part + 4 * (size_t)nchunks;
    L.eul = L.lag + tiles;
    L.total = L.eul + tiles;
    return L;
}
uint8_t *act_flags(const sw_ctx *c, int par) { return c->tflags + par * c->max_tiles; }
uint8_t *synced_flags(const sw_ctx *c) { return c->tflags + 2 * c->max_tiles; }
uint8_t *force_flags(const sw_ctx *c) { return c->tflags + 3 * c->max_tiles; }

size_t tile_of(const sw_ctx *c, int cell)
{
    int i = cell % c->nx, j = cell / c->nx;
    return (size_t)(j / kShapes[c->shape].ty) * c->ntx + (size_t)(i / kShapes[c->shape].tx);
}

// Tiles that must never be skipped: they hold inflow or bed-source cells.
int upload_force(sw_ctx *c)
{
    std::vector<uint8_t> f(ntiles(c), 0);
    for (int32_t q : c->forced_in) f[tile_of(c, q)] = 1;
    for (int32_t q : c->forced_qb) f[tile_of(c, q)] = 1;
    return stage_to_device(c, force_flags(c), f.data(), f.size());
}

void set_shape(sw_ctx *c, int shape)
{
    c->shape = shape;
    c->ntx = (c->nx + kShapes[shape].tx - 1) / kShapes[shape].tx;
    c->nty = (c->ny + kShapes[shape].ty - 1) / kShapes[shape].ty;
    c->dirty = true;
    c->graph_ok = false;
    c->args_gen++;
}

Inst make_inst(const sw_ctx *c, const StepArgs &A)
{
    Inst I{};
    I.P = make_kpar(c);
    I.A = A;
    I.ctrl = c->ctrl;
    for (int s = 0; s < 2; ++s) {
        I.H[s] = c->H[s]; I.qx[s] = c->qx[s]; I.qy[s] = c->qy[s]; I.b[s] = c->b[s];
        I.act[s] = act_flags(c, s);
    }
    I.QLx = c->QLx;
    for (int s = 0; s < 2; ++s) {
        I.jx[s] = c->jx[s];
        I.jy[s] = c->jy[s];
        I.jm[s] = c->jm[s];
    }
    I.QLy = c->QLy;
    I.bnd = c->bnd;
    I.synced = synced_flags(c);
    I.force = force_flags(c);
    I.tmax[0] = c->tmax;
    I.tmax[1] = c->tmax + c->max_tiles;
    I.ntx = c->ntx;
    I.nty = c->nty;
    // rain wets every tile: no tile may be skipped
    I.hgs = ((c->par.flags & SW_FLAG_HGS) && !(c->rain > 0.0)) ? 1 : 0;
    const int nt = c->ntx * c->nty;
    I.chunk = list_chunk(nt);
    I.nchunk = (nt + I.chunk - 1) / I.chunk;
    SchedLayout L = sched_layout(c->max_chunks, c->max_tiles);
    int *sb = c->sched;
    I.totals = sb + L.totals;
    I.cnt_l = sb + L.cnt_l;
    I.cnt_e = sb + L.cnt_e;
    I.pre_l = sb + L.pre_l;
    I.pre_e = sb + L.pre_e;
    I.part = (uint4 *)(sb + L.part);
    I.lag = sb + L.lag;
    I.eul = sb + L.eul;
    return I;
}

// Launch one tiled stage for the context's tile shape.
enum Stage { kPrepare, kDt, kLagrange, kEuler, kCount };

template <int TX, int TY>
void launch_stage_t(Stage st, hipStream_t s, const Inst &I, int par, dim3 g)
{
    if (st == kPrepare) hipLaunchKernelGGL((k_prepare_t<TX, TY>), g, dim3(NT), 0, s, I, par);
    else if (st == kDt) hipLaunchKernelGGL(k_dt_t, dim3(1), dim3(RT), 0, s, I, par);
    else if (st == kCount) hipLaunchKernelGGL(k_count_t, dim3(1), dim3(RT), 0, s, I, par, TX, TY);
    else if (st == kLagrange) hipLaunchKernelGGL((k_lagrange_t<TX, TY>), g, dim3(NT), 0, s, I, par);
    else hipLaunchKernelGGL((k_euler_t<TX, TY>), g, dim3(NT), 0, s, I, par);
}

template <int TX, int TY>
void launch_batch_t(Stage st, hipStream_t s, const Inst *insts, int nmem, const int *table,
                    int ntab, int par)
{
    if (st == kDt) hipLaunchKernelGGL(k_dt_b, dim3(nmem), dim3(RT), 0, s, insts, par);
    else if (st == kLagrange)
        hipLaunchKernelGGL((k_lagrange_b<TX, TY>), dim3(ntab), dim3(NT), 0, s, insts, table, par);
    else hipLaunchKernelGGL((k_euler_b<TX, TY>), dim3(ntab), dim3(NT), 0, s, insts, table, par);
}

// Strip ensembles: K3a over the (member, segment) table dtab, the stage
// kernels over the (member, local workgroup) table, both on work lists.
template <int S, bool CS>
void launch_batch_s(Stage st, hipStream_t s, const Inst *insts, const int *table, int ntab,
                    const int *dtab, int ndtab, int lthr, int par, bool var, bool f2)
{
    if (st == kDt) hipLaunchKernelGGL(k_dt_lists_b, dim3(ndtab), dim3(lthr), 0, s, insts, dtab, par);
    else if (st == kLagrange && f2)
        hipLaunchKernelGGL((k_lagrange_slb<S, CS, true>), dim3(ntab), dim3(NT), 0, s, insts, table, par);
    else if (st == kLagrange)
        hipLaunchKernelGGL((k_lagrange_slb<S, CS, false>), dim3(ntab), dim3(NT), 0, s, insts, table, par);
    else if (var)
        hipLaunchKernelGGL((k_euler_slb<S, CS, true>), dim3(ntab), dim3(NT), 0, s, insts, table, par);
    else hipLaunchKernelGGL((k_euler_slb<S, CS, false>), dim3(ntab), dim3(NT), 0, s, insts, table, par);
}

template <int S>
void launch_batch_s(Stage st, hipStream_t s, const Inst *insts, const int *table, int ntab,
                    const int *dtab, int ndtab, int lthr, int par, bool cs, bool var, bool f2)
{
    if (cs) launch_batch_s<S, true>(st, s, insts, table, ntab, dtab, ndtab, lthr, par, var, f2);
    else launch_batch_s<S, false>(st, s, insts, table, ntab, dtab, ndtab, lthr, par, var, f2);
}

// cs: some member has a per-cell soil or source plane; var: some member runs
// another limiter or wave-speed estimate than minmod + Davis (the general
// kernel gives those members the default's bits).  Tile shapes take the
// (member, bx, by) table; strips the stage and K3a tables.
void launch_batch(int shape, Stage st, hipStream_t s, const Inst *insts, int nmem,
                  const int *table, int ntab, const int *dtab, int ndtab, int lthr, int par,
                  bool cs, bool var, bool f2)
{
    switch (shape) {
    case 0: launch_batch_t<64, 8>(st, s, insts, nmem, table, ntab, par); break;
    case 1: launch_batch_t<64, 4>(st, s, insts, nmem, table, ntab, par); break;
    case 2: launch_batch_t<64, 16>(st, s, insts, nmem, table, ntab, par); break;
    case 3: launch_batch_t<128, 4>(st, s, insts, nmem, table, ntab, par); break;
    case 4: launch_batch_s<8>(st, s, insts, table, ntab, dtab, ndtab, lthr, par, cs, var, f2); break;
    case 5: launch_batch_s<16>(st, s, insts, table, ntab, dtab, ndtab, lthr, par, cs, var, f2); break;
    default: launch_batch_s<32>(st, s, insts, table, ntab, dtab, ndtab, lthr, par, cs, var, f2); break;
    }
}

// Whether a grid's kernels must read per-cell soil or source planes.
bool cell_soil(const KPar &P) { return P.nM || P.d50 || P.psi || P.srcw || P.qb || P.beta; }

// Strip shapes: the prepare pass runs one workgroup per tile; K3 builds the
// work lists; the stage kernels run one wavefront per list entry.
// A stage kernel launch; with events e0/e1 (measurement), the launch itself
// records its start and end time stamps in them (hipExtLaunchKernelGGL).
template <typename K>
void launch_timed(K kern, dim3 g, hipStream_t s, hipEvent_t e0, hipEvent_t e1, const Inst &I,
                  int par)
{
    if (e0) hipExtLaunchKernelGGL(kern, g, dim3(NT), 0, s, e0, e1, 0, I, par);
    else hipLaunchKernelGGL(kern, g, dim3(NT), 0, s, I, par);
}

template <int S>
void launch_strip_t(Stage st, hipStream_t s, const Inst &I, int par, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 gt(I.ntx, I.nty);
    // one wavefront per possible entry; with dry tiles skipped, at most
    // kMaxStageGroups workgroups (the stage kernels then take longer lists in
    // passes).  Without skipping every tile is listed, no workgroup idles and
    // the single-pass kernels (fewer registers held across the pass loop)
    // take the whole grid.
    const int need = (I.ntx * I.nty + SWAVES - 1) / SWAVES;
    const bool big = need > kMaxStageGroups;
    const bool passes = I.hgs && big;
    const int gl = passes ? kMaxStageGroups : need;
    const int gll = passes ? gl
                    : big  ? (I.ntx * ((I.nty + kLagGroup - 1) / kLagGroup) + SWAVES - 1) / SWAVES
                           : (kLagHalves * I.ntx * I.nty + SWAVES - 1) / SWAVES;
    const bool cs = cell_soil(I.P);
    auto lag1 = passes ? (cs ? k_lagrange_sl<S, true, 2, false> : k_lagrange_sl<S, false, 2, false>)
                : big  ? (cs ? k_lagrange_sl<S, true, 3, false> : k_lagrange_sl<S, false, 3, false>)
                       : (cs ? k_lagrange_sl<S, true, 1, false> : k_lagrange_sl<S, false, 1, false>);
    auto lag2 = passes ? (cs ? k_lagrange_sl<S, true, 2, true> : k_lagrange_sl<S, false, 2, true>)
                : big  ? (cs ? k_lagrange_sl<S, true, 3, true> : k_lagrange_sl<S, false, 3, true>)
                       : (cs ? k_lagrange_sl<S, true, 1, true> : k_lagrange_sl<S, false, 1, true>);
    auto lag = I.P.force2 ? lag2 : lag1;
    auto eul = I.P.variant
                   ? (passes ? (cs ? k_euler_sl<S, true, 2, true> : k_euler_sl<S, false, 2, true>)
                             : (cs ? k_euler_sl<S, true, 1, true> : k_euler_sl<S, false, 1, true>))
                   : (passes ? (cs ? k_euler_sl<S, true, 2, false> : k_euler_sl<S, false, 2, false>)
                             : (cs ? k_euler_sl<S, true, 1, false> : k_euler_sl<S, false, 1, false>));
    if (st == kPrepare) hipLaunchKernelGGL((k_prepare_t<SX, S>), gt, dim3(NT), 0, s, I, par);
    else if (st == kDt)
        hipLaunchKernelGGL(k_dt_lists, dim3(I.nchunk), dim3(list_threads(I.chunk)), 0, s, I, par);
    else if (st == kCount) hipLaunchKernelGGL(k_count_t, dim3(1), dim3(RT), 0, s, I, par, SX, S);
    else if (st == kLagrange) launch_timed(lag, dim3(gll), s, e0, e1, I, par);
    else launch_timed(eul, dim3(gl), s, e0, e1, I, par);
}

// e0/e1 (optional): time stamps of a Lagrangian or Euler launch on strips.
void launch_stage(int shape, Stage st, hipStream_t s, const Inst &I, int par,
                  hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    dim3 g(I.ntx, I.nty);
    switch (shape) {
    case 0: launch_stage_t<64, 8>(st, s, I, par, g); break;
    case 1: launch_stage_t<64, 4>(st, s, I, par, g); break;
    case 2: launch_stage_t<64, 16>(st, s, I, par, g); break;
    case 3: launch_stage_t<128, 4>(st, s, I, par, g); break;
    case 4: launch_strip_t<8>(st, s, I, par, e0, e1); break;
    case 5: launch_strip_t<16>(st, s, I, par, e0, e1); break;
    default: launch_strip_t<32>(st, s, I, par, e0, e1); break;
    }
}

// Recompute the Eq. 7 maxima and the wet-tile flags of the current state
// (after any set_* or a tile-shape change), and mark every tile's two buffers
// as possibly different.
int prepare(sw_ctx *c)
{
    int cur = (int)(c->k & 1);
    int rc = upload_force(c);
    if (rc) return rc;
    HIPCHK(c, hipMemsetAsync(c->ctrl->slot[cur], 0, sizeof(c->ctrl->slot[0]), c->stream));
    HIPCHK(c, hipMemsetAsync(synced_flags(c), 0, c->max_tiles, c->stream));
    Inst I = make_inst(c, make_step_args(c, 0, 0.0));
    launch_stage(c->shape, kPrepare, c->stream, I, cur);
    if (c->par.flags & SW_FLAG_UNFUSED) {
        KPar P = make_kpar(c);
        hipLaunchKernelGGL(k_prepare, cell_grid(c), dim3(BX, BY), 0, c->stream, P, c->ctrl, cur,
                           c->H[cur], c->qx[cur], c->qy[cur], c->b[cur]);
    }
    HIPCHK(c, hipGetLastError());
    // the captured graphs stay valid: a new state, bed or time lands in the
    // same planes and control block, so the kernel arguments are unchanged
    c->dirty = false;
    return SW_OK;
}

int read_ctrl(sw_ctx *c, Ctrl *h)
{
    return stage_to_host(c, h, c->ctrl, sizeof(Ctrl));
}

// Index of the buffer holding the current state (the start of the failing
// step if the device raised an error).
int current_buffer(sw_ctx *c, const Ctrl &h) { return h.err ? (h.err_k & 1) : (int)(c->k & 1); }

void enqueue_tiled_step(sw_ctx *c, hipStream_t st, int par, const KPar &P, const StepArgs &A)
{
    (void)P;
    Inst I = make_inst(c, A);
    launch_stage(c->shape, kDt, st, I, par);
    launch_stage(c->shape, kLagrange, st, I, par);
    launch_stage(c->shape, kEuler, st, I, par);
}

void enqueue_unfused_step(sw_ctx *c, int par, const KPar &P, const StepArgs &A)
{
    dim3 g = cell_grid(c), blk(BX, BY);
    dim3 gf((c->nx + 1 + BX - 1) / BX, (c->ny + 1 + BY - 1) / BY);
    size_t nfx = (size_t)(c->nx + 1) * c->ny, nfy = (size_t)c->nx * (c->ny + 1);
    FaceView F;
    F.xH = c->faces; F.xn = F.xH + nfx; F.xt = F.xn + nfx; F.xJ = F.xt + nfx;
    F.yH = F.xJ + nfx; F.yn = F.yH + nfy; F.yt = F.yn + nfy; F.yJ = F.yt + nfy;
    StateView S{c->H[par], c->qx[par], c->qy[par], c->b[par]};
    LagView L{c->QLx, c->QLy};
    OutView O{c->H[par ^ 1], c->qx[par ^ 1], c->qy[par ^ 1], c->b[par ^ 1]};
    hipLaunchKernelGGL(k_dt, dim3(1), dim3(64), 0, c->stream, c->ctrl, par, A);
    hipLaunchKernelGGL(k_lagrange, g, blk, 0, c->stream, P, c->ctrl, par, S, c->QLx, c->QLy);
    hipLaunchKernelGGL(k_faces, gf, blk, 0, c->stream, P, c->ctrl, S, L, F);
    hipLaunchKernelGGL(k_update, g, blk, 0, c->stream, P, c->ctrl, par, S, L, F, O, c->bnd);
}

// Capture the two-step graph (even step, then odd step) for the current inputs.
// Step pairs in the long graph: one graph launch per 16 steps, so the gap
// between two graph launches is paid once per 16 steps instead of every
// second step.
constexpr int kLongPairs = 8;

int capture_pairs(sw_ctx *c, const KPar &P, const StepArgs &A, int pairs, hipGraphExec_t *out)
{
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    for (int q = 0; q < pairs; ++q) {
        enqueue_tiled_step(c, c->cap, 0, P, A);
        enqueue_tiled_step(c, c->cap, 1, P, A);
    }
    HIPCHK(c, hipStreamEndCapture(c->cap, &g));
    hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, SW_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return SW_OK;
}

int ensure_graph(sw_ctx *c, const KPar &P, const StepArgs &A)
{
    if (c->graph_ok && c->graph_fixed == A.mode_fixed && c->graph_dt == A.dt_fixed) return SW_OK;
    for (hipGraphExec_t *x : {&c->gexec, &c->gexec_long})
        if (*x) {
            (void)hipGraphExecDestroy(*x);
            *x = nullptr;
        }
    if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    int rc = capture_pairs(c, P, A, 1, &c->gexec);
    if (!rc) rc = capture_pairs(c, P, A, kLongPairs, &c->gexec_long);
    if (rc) return rc;
    c->graph_ok = true;
    c->graph_builds++;
    c->graph_fixed = A.mode_fixed;
    c->graph_dt = A.dt_fixed;
    return SW_OK;
}

int launch_steps(sw_ctx *c, int32_t nsteps, int fixed, double dt)
{
    if (!c) return SW_ERR_ARG;
    if (nsteps < 0) return fail(c, SW_ERR_ARG, "nsteps must be >= 0");
    if (!c->have_state) return fail(c, SW_ERR_STATE, "advance before sw_set_state");
    if (fixed && !(dt > 0.0)) return fail(c, SW_ERR_ARG, "fixed dt must be > 0");
    if (c->dirty) {
        int rc = prepare(c);
        if (rc) return rc;
    }
    KPar P = make_kpar(c);
    StepArgs A = make_step_args(c, fixed, dt);
    if (c->par.flags & SW_FLAG_UNFUSED) {
        for (int32_t s = 0; s < nsteps; ++s) {
            enqueue_unfused_step(c, (int)(c->k & 1), P, A);
            HIPCHK(c, hipGetLastError());
            c->k++;
        }
        return SW_OK;
    }
    const bool use_graph = !(c->par.flags & SW_FLAG_NO_GRAPH);
    int32_t left = nsteps;
    if (left > 0 && (c->k & 1)) {  // align to an even step for the two-step graph
        enqueue_tiled_step(c, c->stream, 1, P, A);
        HIPCHK(c, hipGetLastError());
        c->k++;
        left--;
    }
    if (use_graph && left >= 2) {
        int rc = ensure_graph(c, P, A);
        if (rc) return rc;
        for (; left >= 2 * kLongPairs; left -= 2 * kLongPairs) {
            HIPCHK(c, hipGraphLaunch(c->gexec_long, c->stream));
            c->k += 2 * kLongPairs;
        }
        for (; left >= 2; left -= 2) {
            HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
            c->k += 2;
        }
    }
    for (; left > 0; --left) {
        enqueue_tiled_step(c, c->stream, (int)(c->k & 1), P, A);
        HIPCHK(c, hipGetLastError());
        c->k++;
    }
    return SW_OK;
}

// A copy of a context's current state (fields, bed residual, boundary
// accumulators, control block and step index) on the device, to put back
// after trial steps (the autotuners).
struct StateKeep {
    float *planes = nullptr;
    double *bnd = nullptr;
    Ctrl ctrl{};
    int64_t k0 = 0;
};

int keep_save(sw_ctx *c, StateKeep &kp)
{
    int rc = read_ctrl(c, &kp.ctrl);
    if (rc) return rc;
    if (kp.ctrl.err) return fail(c, kp.ctrl.err, "trial steps with a pending device error");
    kp.k0 = c->k;
    const int cur = (int)(kp.k0 & 1);
    const size_t nb = 4 * (size_t)(c->nx + c->ny);
    HIPCHK(c, hipMalloc(&kp.planes, 5 * c->plane * sizeof(float)));
    HIPCHK(c, hipMalloc(&kp.bnd, nb * sizeof(double)));
    const float *src[5] = {c->H[cur], c->qx[cur], c->qy[cur], c->b[cur], c->rb};
    for (int f = 0; f < 5; ++f)
        HIPCHK(c, hipMemcpyAsync(kp.planes + f * c->plane, src[f], c->plane * sizeof(float),
                                 hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(kp.bnd, c->bnd, nb * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SW_OK;
}

// Put the kept state back (the next advance runs the set-up pass).
int keep_restore(sw_ctx *c, const StateKeep &kp)
{
    const int cur = (int)(kp.k0 & 1);
    const size_t nb = 4 * (size_t)(c->nx + c->ny);
    float *dst[5] = {c->H[cur], c->qx[cur], c->qy[cur], c->b[cur], c->rb};
    for (int f = 0; f < 5; ++f)
        HIPCHK(c, hipMemcpyAsync(dst[f], kp.planes + f * c->plane, c->plane * sizeof(float),
                                 hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->bnd, kp.bnd, nb * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    int rc = stage_to_device(c, c->ctrl, &kp.ctrl, sizeof(Ctrl));
    if (rc) return rc;
    c->k = kp.k0;
    c->dirty = true;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SW_OK;
}

void keep_free(StateKeep &kp)
{
    (void)hipFree(kp.planes);
    (void)hipFree(kp.bnd);
    kp.planes = nullptr;
    kp.bnd = nullptr;
}

}  // namespace

extern "C" {

void sw_default_params(sw_params *p)
{
    if (!p) return;
    p->g = 9.81;
    p->cfl = 0.3;
    p->eps_dry = 1e-5;
    p->h_sed = 1e-2;
    p->dt_max = 1.0;
    p->dt_min = 1e-9;
    p->s_rel = 2.65;
    p->C_J = 2.0;
    p->C_Sh = 5.0;
    p->A_G = 1e-3;
    p->m_exp = 2.0;
    p->sed_law = SW_SED_EQ4;
    p->flags = SW_FLAG_HGS;
    p->limiter = SW_LIM_MINMOD;
    p->hll_speeds = SW_HLL_DAVIS;
}

int sw_create(const sw_grid *grid, const sw_params *params, void *hip_stream, sw_ctx **out)
{
    if (!grid || !params || !out) return SW_ERR_ARG;
    *out = nullptr;
    if (grid->nx < 1 || grid->ny < 1 || !(grid->dx > 0.0)) return SW_ERR_ARG;
    // the strip kernels address a plane with one 32-bit byte offset from its
    // base: a pitched plane must stay below 4 GiB (2^30 cells)
    if ((int64_t)((grid->nx + 63) / 64 * 64) * grid->ny * 4 >= ((int64_t)1 << 32)) return SW_ERR_ARG;
    for (int s = 0; s < 4; ++s)
        if (grid->bc[s] != SW_BC_WALL && grid->bc[s] != SW_BC_OPEN) return SW_ERR_ARG;
    if (params->sed_law < SW_SED_NONE || params->sed_law > SW_SED_EQ4) return SW_ERR_ARG;
    if (!(params->cfl > 0.0) || !(params->g > 0.0) || !(params->eps_dry > 0.0)) return SW_ERR_ARG;
    if (params->limiter < SW_LIM_MINMOD || params->limiter > SW_LIM_SUPERBEE) return SW_ERR_ARG;
    if (params->hll_speeds != SW_HLL_DAVIS && params->hll_speeds != SW_HLL_TWO_RAREFACTION)
        return SW_ERR_ARG;
    // the second-order force is built into the strip kernels only
    if ((params->flags & SW_FLAG_FORCE2) && (params->flags & SW_FLAG_UNFUSED)) return SW_ERR_ARG;
    sw_ctx *c = new sw_ctx();
    c->grid = *grid;
    c->par = *params;
    c->nx = grid->nx;
    c->ny = grid->ny;
    c->pitch = (grid->nx + 63) / 64 * 64;
    c->plane = (size_t)c->pitch * c->ny;
    auto bail = [&](hipError_t e, const char *what) {
        std::string m = std::string(what) + ": " + hipGetErrorString(e);
        sw_destroy(c);
        fprintf(stderr, "sw_create: %s\n", m.c_str());
        return SW_ERR_HIP;
    };
    hipError_t e;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess)
            return bail(e, "hipStreamCreate");
        c->own_stream = true;
    }
    // planes: 2 x (H, qx, qy, b), QLx, QLy, 2 x (J0x, J0y, |J0|), bed residual
    const int nplanes = 17;
    if ((e = hipMalloc(&c->buf, nplanes * c->plane * sizeof(float))) != hipSuccess)
        return bail(e, "hipMalloc(state)");
    if ((e = hipMemsetAsync(c->buf, 0, nplanes * c->plane * sizeof(float), c->stream)) != hipSuccess)
        return bail(e, "hipMemset(state)");
    for (int s = 0; s < 2; ++s) {
        c->H[s] = c->buf + (4 * s + 0) * c->plane;
        c->qx[s] = c->buf + (4 * s + 1) * c->plane;
        c->qy[s] = c->buf + (4 * s + 2) * c->plane;
        c->b[s] = c->buf + (4 * s + 3) * c->plane;
    }
    c->QLx = c->buf + 8 * c->plane;
    c->QLy = c->buf + 9 * c->plane;
    for (int s = 0; s < 2; ++s) {
        c->jx[s] = c->buf + (10 + 3 * s) * c->plane;
        c->jy[s] = c->buf + (11 + 3 * s) * c->plane;
        c->jm[s] = c->buf + (12 + 3 * s) * c->plane;
    }
    c->rb = c->buf + 16 * c->plane;
    if (c->par.flags & SW_FLAG_UNFUSED) {  // face arrays of the unfused sequence only
        size_t nf = 4 * ((size_t)(c->nx + 1) * c->ny + (size_t)c->nx * (c->ny + 1));
        if ((e = hipMalloc(&c->faces, nf * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc(faces)");
        if ((e = hipMemsetAsync(c->faces, 0, nf * sizeof(float), c->stream)) != hipSuccess) return bail(e, "hipMemset(faces)");
    }
    size_t nb = 4 * (size_t)(c->nx + c->ny);
    if ((e = hipMalloc(&c->bnd, nb * sizeof(double))) != hipSuccess) return bail(e, "hipMalloc(bnd)");
    if ((e = hipMalloc(&c->steplog, kStepLog * sizeof(StepRec))) != hipSuccess)
        return bail(e, "hipMalloc(step log)");
    if ((e = hipMemsetAsync(c->bnd, 0, nb * sizeof(double), c->stream)) != hipSuccess) return bail(e, "hipMemset(bnd)");
    c->sum_rows = std::max(1, (int)((c->ny + 1023) / 1024));
    c->nsum_blocks = (c->ny + c->sum_rows - 1) / c->sum_rows;
    if ((e = hipMalloc(&c->part, (4 * (size_t)c->nsum_blocks + 8) * sizeof(double))) != hipSuccess)
        return bail(e, "hipMalloc(part)");
    c->sums = c->part + 4 * (size_t)c->nsum_blocks;
    for (int sh = 0; sh < kNumShapes; ++sh) {
        set_shape(c, sh);
        c->max_tiles = std::max(c->max_tiles, ntiles(c));
        const int nt = (int)ntiles(c), ch = list_chunk(nt);
        c->max_chunks = std::max(c->max_chunks, (nt + ch - 1) / ch);
    }
    set_shape(c, kDefaultShape);
    if ((e = hipMalloc(&c->tflags, 4 * c->max_tiles)) != hipSuccess) return bail(e, "hipMalloc(tiles)");
    if ((e = hipMemsetAsync(c->tflags, 0, 4 * c->max_tiles, c->stream)) != hipSuccess) return bail(e, "hipMemset(tiles)");
    if ((e = hipMalloc(&c->tmax, 2 * c->max_tiles * sizeof(uint4))) != hipSuccess) return bail(e, "hipMalloc(tmax)");
    const size_t nsched = sched_layout(c->max_chunks, c->max_tiles).total;
    if ((e = hipMalloc(&c->sched, nsched * sizeof(int))) != hipSuccess) return bail(e, "hipMalloc(sched)");
    if ((e = hipMemsetAsync(c->sched, 0, nsched * sizeof(int), c->stream)) != hipSuccess) return bail(e, "hipMemset(sched)");
    if ((e = hipMemsetAsync(c->tmax, 0, 2 * c->max_tiles * sizeof(uint4), c->stream)) != hipSuccess) return bail(e, "hipMemset(tmax)");
    if ((e = hipMalloc(&c->ctrl, sizeof(Ctrl))) != hipSuccess) return bail(e, "hipMalloc(ctrl)");
    if ((e = hipMemsetAsync(c->ctrl, 0, sizeof(Ctrl), c->stream)) != hipSuccess) return bail(e, "hipMemset(ctrl)");
    // every clear above is ordered on the context's stream (which may be a
    // non-blocking stream that does not wait for the null stream); creation
    // returns once they are done
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return bail(e, "hipStreamSynchronize");
    *out = c;
    return SW_OK;
}

int sw_destroy(sw_ctx *c)
{
    if (!c) return SW_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->buf);
    (void)hipFree(c->faces);
    (void)hipFree(c->bnd);
    (void)hipFree(c->part);
    (void)hipFree(c->ctrl);
    (void)hipFree(c->bound_slot);
    (void)hipFree(c->steplog);
    (void)hipFree(c->nM);
    (void)hipFree(c->d50);
    (void)hipFree(c->psi);
    (void)hipFree(c->qb);
    (void)hipFree(c->srcw);
    (void)hipFree(c->beta);
    (void)hipFree(c->ab);
    (void)hipFree(c->rh);
    (void)hipFree(c->tflags);
    (void)hipFree(c->tmax);
    (void)hipFree(c->sched);
    if (c->stage) (void)hipHostFree(c->stage);
    if (c->copy_stream) (void)hipStreamSynchronize(c->copy_stream);
    (void)hipFree(c->snap);
    (void)hipFree(c->snap_ctrl);
    if (c->snap_host) (void)hipHostFree(c->snap_host);
    if (c->ev_snap) (void)hipEventDestroy(c->ev_snap);
    if (c->ev_copied) (void)hipEventDestroy(c->ev_copied);
    if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->gexec_long) (void)hipGraphExecDestroy(c->gexec_long);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return SW_OK;
}

int sw_set_bed(sw_ctx *c, const float *b, int ptr_kind)
{
    if (!c) return SW_ERR_ARG;
    if (!b) return fail(c, SW_ERR_ARG, "bed pointer is NULL");
    int cur = (int)(c->k & 1);
    int rc = upload_plane(c, c->b[cur], b, ptr_kind);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(c->b[cur ^ 1], c->b[cur], c->plane * sizeof(float),
                             hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->rb, 0, c->plane * sizeof(float), c->stream));
    c->dirty = true;
    return SW_OK;
}

static int set_soil_field(sw_ctx *c, float **dst, const float *src, int ptr_kind)
{
    if (!src) {
        (void)hipFree(*dst);
        *dst = nullptr;
        return SW_OK;
    }
    if (!*dst) {
        HIPCHK(c, hipMalloc(dst, c->plane * sizeof(float)));
        HIPCHK(c, hipMemsetAsync(*dst, 0, c->plane * sizeof(float), c->stream));
    }
    return upload_plane(c, *dst, src, ptr_kind);
}

int sw_set_soil(sw_ctx *c, const float *manning, float manning_scalar, const float *d50,
                float d50_scalar, const float *psi, float psi_scalar, int ptr_kind)
{
    if (!c) return SW_ERR_ARG;
    if (!psi && !(psi_scalar >= 0.0f && psi_scalar < 1.0f))
        return fail(c, SW_ERR_ARG, "porosity must lie in [0, 1)");
    if (!d50 && !(d50_scalar > 0.0f)) return fail(c, SW_ERR_ARG, "d50 must be > 0");
    if (!manning && !(manning_scalar >= 0.0f)) return fail(c, SW_ERR_ARG, "Manning n must be >= 0");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int rc;
    if ((rc = set_soil_field(c, &c->nM, manning, ptr_kind))) return rc;
    if ((rc = set_soil_field(c, &c->d50, d50, ptr_kind))) return rc;
    if ((rc = set_soil_field(c, &c->psi, psi, ptr_kind))) return rc;
    c->nM_s = manning_scalar;
    c->d50_s = d50_scalar;
    c->psi_s = psi_scalar;
    c->dirty = true;
    c->graph_ok = false;
    c->args_gen++;  // soil pointers and scalars are kernel arguments
    return SW_OK;
}

int sw_set_state(sw_ctx *c, const float *h, const float *hu, const float *hv, int ptr_kind)
{
    if (!c) return SW_ERR_ARG;
    if (!h || !hu || !hv) return fail(c, SW_ERR_ARG, "state pointer is NULL");
    // host-side check and clean-up of the initial state
    size_t n = (size_t)c->nx * c->ny;
    std::vector<float> H(n), U(n), V(n);
    if (ptr_kind != SW_PTR_HOST && ptr_kind != SW_PTR_DEVICE)
        return fail(c, SW_ERR_ARG, "ptr_kind must be SW_PTR_HOST or SW_PTR_DEVICE");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    {
        const float *src[3] = {h, hu, hv};
        float *dst[3] = {H.data(), U.data(), V.data()};
        for (int f = 0; f < 3; ++f) {
            if (ptr_kind == SW_PTR_HOST) {
                std::memcpy(dst[f], src[f], n * sizeof(float));
            } else {
                int rc = stage_to_host(c, dst[f], src[f], n * sizeof(float));
                if (rc) return rc;
            }
        }
    }
    for (size_t q = 0; q < n; ++q) {
        if (!(H[q] >= 0.0f) || !std::isfinite(H[q]) || !std::isfinite(U[q]) || !std::isfinite(V[q]))
            return fail(c, SW_ERR_ARG, "initial depth must be finite and >= 0, discharges finite");
        if (H[q] == 0.0f) { H[q] = 0.0f; U[q] = 0.0f; V[q] = 0.0f; }
    }
    // keep the bed of the current state (the start of a failed step after a
    // device error), restart the step ring at k = 0
    Ctrl hc;
    int rc0 = read_ctrl(c, &hc);
    if (rc0) return rc0;
    int cur = current_buffer(c, hc);
    if (cur != 0)
        HIPCHK(c, hipMemcpyAsync(c->b[0], c->b[cur], c->plane * sizeof(float),
                                 hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->b[1], c->b[0], c->plane * sizeof(float), hipMemcpyDeviceToDevice,
                             c->stream));
    c->k = 0;
    int rc;
    if ((rc = upload_plane(c, c->H[0], H.data(), SW_PTR_HOST))) return rc;
    if ((rc = upload_plane(c, c->qx[0], U.data(), SW_PTR_HOST))) return rc;
    if ((rc = upload_plane(c, c->qy[0], V.data(), SW_PTR_HOST))) return rc;
    HIPCHK(c, hipMemsetAsync(c->QLx, 0, 2 * c->plane * sizeof(float), c->stream));
    HIPCHK(c, hipMemsetAsync(c->bnd, 0, 4 * (size_t)(c->nx + c->ny) * sizeof(double), c->stream));
    if (c->ab) HIPCHK(c, hipMemsetAsync(c->ab, 0, c->plane * sizeof(double), c->stream));
    if (c->rh) HIPCHK(c, hipMemsetAsync(c->rh, 0, c->plane * sizeof(float), c->stream));
    Ctrl h0{};
    h0.t[0] = c->t0;
    {
        const int rc_ = stage_to_device(c, c->ctrl, &h0, sizeof(Ctrl));
        if (rc_) return rc_;
    }
    c->have_state = true;
    c->dirty = true;
    return SW_OK;
}

int sw_set_inflow(sw_ctx *c, const int32_t *cell_idx, const float *weight, int32_t n,
                  double q_base, double q_peak, double t_peak, double t_sigma)
{
    if (!c) return SW_ERR_ARG;
    if (n < 0) return fail(c, SW_ERR_ARG, "n must be >= 0");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->graph_ok = false;
    c->args_gen++;  // the hydrograph and weight plane are kernel arguments
    if (n == 0) {
        c->has_inflow = 0;
        c->forced_in.clear();
        c->dirty = true;
        return upload_force(c);
    }
    if (!cell_idx || !weight) return fail(c, SW_ERR_ARG, "inflow arrays are NULL");
    double wsum = 0.0;
    for (int32_t q = 0; q < n; ++q) {
        if (cell_idx[q] < 0 || cell_idx[q] >= c->nx * c->ny)
            return fail(c, SW_ERR_ARG, "inflow cell index out of range");
        if (!(weight[q] >= 0.0f)) return fail(c, SW_ERR_ARG, "inflow weights must be >= 0");
        wsum += weight[q];
    }
    if (!(wsum > 0.0)) return fail(c, SW_ERR_ARG, "inflow weights sum to zero");
    std::vector<float> w((size_t)c->plane, 0.0f);
    std::vector<double> acc((size_t)c->nx * c->ny, 0.0);
    for (int32_t q = 0; q < n; ++q) acc[cell_idx[q]] += (double)weight[q] / wsum;
    double dx2 = c->grid.dx * c->grid.dx;
    for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) w[(size_t)j * c->pitch + i] = (float)(acc[(size_t)j * c->nx + i] / dx2);
    if (!c->srcw) HIPCHK(c, hipMalloc(&c->srcw, c->plane * sizeof(float)));
    int rcw = stage_to_device(c, c->srcw, w.data(), c->plane * sizeof(float));
    if (rcw) return rcw;
    c->has_inflow = 1;
    c->q_base = q_base; c->q_peak = q_peak; c->t_peak = t_peak; c->t_sigma = t_sigma;
    c->forced_in.assign(cell_idx, cell_idx + n);
    c->dirty = true;
    return upload_force(c);
}

int sw_set_sed_sources(sw_ctx *c, const float *qb_plus, const float *qb_minus, int ptr_kind)
{
    if (!c) return SW_ERR_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->graph_ok = false;
    c->args_gen++;  // the source plane and its total are kernel arguments
    if (!qb_plus && !qb_minus) {
        (void)hipFree(c->qb);
        c->qb = nullptr;
        c->qb_total = 0.0;
        c->forced_qb.clear();
        c->dirty = true;
        return upload_force(c);
    }
    size_t n = (size_t)c->nx * c->ny;
    std::vector<float> p(n, 0.0f), m(n, 0.0f), d((size_t)c->plane, 0.0f);
    if (ptr_kind != SW_PTR_HOST && ptr_kind != SW_PTR_DEVICE)
        return fail(c, SW_ERR_ARG, "ptr_kind must be SW_PTR_HOST or SW_PTR_DEVICE");
    for (int f = 0; f < 2; ++f) {
        const float *src = f == 0 ? qb_plus : qb_minus;
        float *dst = f == 0 ? p.data() : m.data();
        if (!src) continue;
        if (ptr_kind == SW_PTR_HOST) {
            std::memcpy(dst, src, n * sizeof(float));
        } else {
            int rc = stage_to_host(c, dst, src, n * sizeof(float));
            if (rc) return rc;
        }
    }
    double tot = 0.0;
    c->forced_qb.clear();
    for (int j = 0; j < c->ny; ++j)
        for (int i = 0; i < c->nx; ++i) {
            float v = p[(size_t)j * c->nx + i] - m[(size_t)j * c->nx + i];
            if (!std::isfinite(v)) return fail(c, SW_ERR_ARG, "bed sources must be finite");
            d[(size_t)j * c->pitch + i] = v;
            tot += (double)v;
            if (v != 0.0f) c->forced_qb.push_back(j * c->nx + i);
        }
    if (!c->qb) HIPCHK(c, hipMalloc(&c->qb, c->plane * sizeof(float)));
    int rcq = stage_to_device(c, c->qb, d.data(), c->plane * sizeof(float));
    if (rcq) return rcq;
    c->qb_total = tot * c->grid.dx * c->grid.dx;
    c->dirty = true;
    return upload_force(c);
}

int sw_set_forcing(sw_ctx *c, double rain, const float *beta, float beta_scalar, double coriolis,
                   double wind_x, double wind_y, double wind_coef, int ptr_kind)
{
    if (!c) return SW_ERR_ARG;
    if (!(rain >= 0.0) || !std::isfinite(rain)) return fail(c, SW_ERR_ARG, "rain must be finite and >= 0");
    if (!beta && !(beta_scalar >= 0.0f && std::isfinite(beta_scalar)))
        return fail(c, SW_ERR_ARG, "absorption coefficient must be finite and >= 0");
    if (!std::isfinite(coriolis) || !std::isfinite(wind_x) || !std::isfinite(wind_y) ||
        !(wind_coef >= 0.0) || !std::isfinite(wind_coef))
        return fail(c, SW_ERR_ARG, "Coriolis and wind parameters must be finite, wind_coef >= 0");
    if (beta && ptr_kind == SW_PTR_HOST)
        for (size_t q = 0; q < (size_t)c->nx * c->ny; ++q)
            if (!(beta[q] >= 0.0f) || !std::isfinite(beta[q]))
                return fail(c, SW_ERR_ARG, "absorption coefficients must be finite and >= 0");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int rc = set_soil_field(c, &c->beta, beta, ptr_kind);
    if (rc) return rc;
    c->beta_s = beta ? 0.0f : beta_scalar;
    const bool absorbs = beta != nullptr || beta_scalar > 0.0f;
    if (absorbs && !c->ab) {
        HIPCHK(c, hipMalloc(&c->ab, c->plane * sizeof(double)));
        HIPCHK(c, hipMemsetAsync(c->ab, 0, c->plane * sizeof(double), c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else if (!absorbs && c->ab) {
        (void)hipFree(c->ab);
        c->ab = nullptr;
    }
    if (rain > 0.0 && !c->rh) {
        HIPCHK(c, hipMalloc(&c->rh, c->plane * sizeof(float)));
        HIPCHK(c, hipMemsetAsync(c->rh, 0, c->plane * sizeof(float), c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else if (!(rain > 0.0) && c->rh) {
        (void)hipFree(c->rh);
        c->rh = nullptr;
    }
    c->rain = rain;
    c->coriolis = coriolis;
    c->wind_x = wind_x;
    c->wind_y = wind_y;
    c->wind_coef = wind_coef;
    c->dirty = true;
    c->graph_ok = false;
    c->args_gen++;  // the forcing constants and planes are kernel arguments
    return SW_OK;
}

int sw_set_time(sw_ctx *c, double t, int64_t step)
{
    if (!c) return SW_ERR_ARG;
    Ctrl h;
    int rc = read_ctrl(c, &h);
    if (rc) return rc;
    h.t[c->k & 1] = t;
    {
        const int rc_ = stage_to_device(c, c->ctrl, &h, sizeof(Ctrl));
        if (rc_) return rc_;
    }
    c->t0 = t;
    c->step0 = step - c->k;
    return SW_OK;
}

int sw_replace_state(sw_ctx *c, const float *h, const float *hu, const float *hv, const float *b,
                     double t, int64_t step)
{
    if (!c) return SW_ERR_ARG;
    if (!h || !hu || !hv || !b) return fail(c, SW_ERR_ARG, "state pointer is NULL");
    int rc;
    c->k = 0;
    if ((rc = upload_plane(c, c->H[0], h, SW_PTR_DEVICE))) return rc;
    if ((rc = upload_plane(c, c->qx[0], hu, SW_PTR_DEVICE))) return rc;
    if ((rc = upload_plane(c, c->qy[0], hv, SW_PTR_DEVICE))) return rc;
    if ((rc = upload_plane(c, c->b[0], b, SW_PTR_DEVICE))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->b[1], c->b[0], c->plane * sizeof(float), hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipMemsetAsync(c->rb, 0, c->plane * sizeof(float), c->stream));
    HIPCHK(c, hipMemsetAsync(c->QLx, 0, 2 * c->plane * sizeof(float), c->stream));
    HIPCHK(c, hipMemsetAsync(c->bnd, 0, 4 * (size_t)(c->nx + c->ny) * sizeof(double), c->stream));
    if (c->ab) HIPCHK(c, hipMemsetAsync(c->ab, 0, c->plane * sizeof(double), c->stream));
    if (c->rh) HIPCHK(c, hipMemsetAsync(c->rh, 0, c->plane * sizeof(float), c->stream));
    Ctrl h0{};
    h0.t[0] = t;
    {
        const int rc_ = stage_to_device(c, c->ctrl, &h0, sizeof(Ctrl));
        if (rc_) return rc_;
    }
    c->t0 = t;
    c->step0 = step;
    c->have_state = true;
    c->dirty = true;
    return SW_OK;
}

int sw_get_grid(const sw_ctx *c, sw_grid *out)
{
    if (!c || !out) return SW_ERR_ARG;
    *out = c->grid;
    return SW_OK;
}

int sw_advance(sw_ctx *c, int32_t nsteps) { return launch_steps(c, nsteps, 0, 0.0); }

int sw_advance_fixed_dt(sw_ctx *c, int32_t nsteps, double dt) { return launch_steps(c, nsteps, 1, dt); }

int sw_advance_profiled(sw_ctx *c, int32_t nsteps, double *avg_ms)
{
    if (!c || !avg_ms) return SW_ERR_ARG;
    if (nsteps < 1) return fail(c, SW_ERR_ARG, "nsteps must be >= 1");
    if (c->par.flags & SW_FLAG_UNFUSED)
        return fail(c, SW_ERR_ARG, "kernel timing covers the tiled path only");
    if (!c->have_state) return fail(c, SW_ERR_STATE, "advance before sw_set_state");
    if (c->dirty) {
        int rc = prepare(c);
        if (rc) return rc;
    }
    Inst I = make_inst(c, make_step_args(c, 0, 0.0));
    // strips: each stage launch records its own start and end (the kernel's
    // execution, as a kernel trace reports it); tile shapes: events between launches
    const bool ext = is_strip(c->shape);
    std::vector<hipEvent_t> ev(4 * (size_t)nsteps, nullptr);
    for (auto &e : ev) HIPCHK(c, hipEventCreate(&e));
    for (int32_t s = 0; s < nsteps; ++s) {
        int par = (int)(c->k & 1);
        hipEvent_t *e = &ev[4 * (size_t)s];
        launch_stage(c->shape, kDt, c->stream, I, par);
        if (ext) {
            launch_stage(c->shape, kLagrange, c->stream, I, par, e[0], e[1]);
            launch_stage(c->shape, kEuler, c->stream, I, par, e[2], e[3]);
        } else {
            HIPCHK(c, hipEventRecord(e[0], c->stream));
            launch_stage(c->shape, kLagrange, c->stream, I, par);
            HIPCHK(c, hipEventRecord(e[1], c->stream));
            HIPCHK(c, hipEventRecord(e[2], c->stream));
            launch_stage(c->shape, kEuler, c->stream, I, par);
            HIPCHK(c, hipEventRecord(e[3], c->stream));
        }
        launch_stage(c->shape, kCount, c->stream, I, par);
        HIPCHK(c, hipGetLastError());
        c->k++;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double tl = 0.0, te = 0.0;
    for (int32_t s = 0; s < nsteps; ++s) {
        float a = 0.0f, b = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&a, ev[4 * (size_t)s], ev[4 * (size_t)s + 1]));
        HIPCHK(c, hipEventElapsedTime(&b, ev[4 * (size_t)s + 2], ev[4 * (size_t)s + 3]));
        tl += a;
        te += b;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    avg_ms[0] = tl / nsteps;
    avg_ms[1] = te / nsteps;
    return SW_OK;
}

int sw_set_tile_shape(sw_ctx *c, int32_t tile_x, int32_t tile_y)
{
    if (!c) return SW_ERR_ARG;
    for (int sh = 0; sh < kNumShapes; ++sh)
        if (kShapes[sh].tx == tile_x && kShapes[sh].ty == tile_y) {
            if ((c->par.flags & SW_FLAG_FORCE2) && !is_strip(sh))
                return fail(c, SW_ERR_ARG, "the second-order force runs on strip shapes only");
            HIPCHK(c, hipStreamSynchronize(c->stream));
            set_shape(c, sh);
            return SW_OK;
        }
    return fail(c, SW_ERR_ARG, "unknown tile shape");
}

int sw_autotune(sw_ctx *c, int32_t nsteps, int32_t *tile_x, int32_t *tile_y)
{
    if (!c) return SW_ERR_ARG;
    if (nsteps < 1) return fail(c, SW_ERR_ARG, "nsteps must be >= 1");
    if (!c->have_state) return fail(c, SW_ERR_STATE, "autotune before sw_set_state");
    if (c->par.flags & SW_FLAG_UNFUSED) return fail(c, SW_ERR_ARG, "the unfused path has no tiles");
    StateKeep kp;
    int rc = keep_save(c, kp);
    if (rc) {
        keep_free(kp);
        return rc;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int best = c->shape;
    float best_ms = 0.0f;
    bool timed = false;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = fail(c, SW_ERR_HIP, "hipEventCreate");
    for (int sh = 0; sh < kNumShapes && !rc; ++sh) {
        if ((c->par.flags & SW_FLAG_FORCE2) && !is_strip(sh)) continue;
        set_shape(c, sh);
        if ((rc = prepare(c))) break;
        Inst I = make_inst(c, make_step_args(c, 0, 0.0));
        if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = fail(c, SW_ERR_HIP, "hipEventRecord"); break; }
        for (int32_t s = 0; s < nsteps; ++s) {
            int par = (int)(c->k & 1);
            launch_stage(sh, kDt, c->stream, I, par);
            launch_stage(sh, kLagrange, c->stream, I, par);
            launch_stage(sh, kEuler, c->stream, I, par);
            c->k++;
        }
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(c, SW_ERR_HIP, "kernel timing failed");
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (!timed || ms < best_ms) { best_ms = ms; best = sh; timed = true; }
        if ((rc = keep_restore(c, kp))) break;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (!rc) rc = keep_restore(c, kp);
    keep_free(kp);
    if (rc) return rc;
    set_shape(c, best);
    if (tile_x) *tile_x = kShapes[best].tx;
    if (tile_y) *tile_y = kShapes[best].ty;
    return SW_OK;
}

int sw_sync(sw_ctx *c)
{
    if (!c) return SW_ERR_ARG;
    Ctrl h;
    int rc = read_ctrl(c, &h);
    if (rc) return rc;
    if (h.err) return fail(c, h.err, "device error raised at step " + std::to_string(h.err_k));
    return SW_OK;
}

int sw_get_fields(sw_ctx *c, float *h, float *hu, float *hv, float *b, int ptr_kind)
{
    if (!c) return SW_ERR_ARG;
    Ctrl hc;
    int rc = read_ctrl(c, &hc);
    if (rc) return rc;
    int cur = current_buffer(c, hc);
    if (h && (rc = download_plane(c, h, c->H[cur], ptr_kind))) return rc;
    if (hu && (rc = download_plane(c, hu, c->qx[cur], ptr_kind))) return rc;
    if (hv && (rc = download_plane(c, hv, c->qy[cur], ptr_kind))) return rc;
    if (b && (rc = download_plane(c, b, c->b[cur], ptr_kind))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (hc.err) return fail(c, hc.err, "device error raised at step " + std::to_string(hc.err_k));
    return SW_OK;
}

int sw_step_bound(sw_ctx *c, double *dt)
{
    if (!c || !dt) return SW_ERR_ARG;
    if (!c->have_state) return fail(c, SW_ERR_STATE, "sw_step_bound before sw_set_state");
    Ctrl hc;
    int rc = read_ctrl(c, &hc);
    if (rc) return rc;
    if (hc.err) return fail(c, hc.err, "device error raised at step " + std::to_string(hc.err_k));
    const int cur = current_buffer(c, hc);
    const size_t bytes = NSLOT * 4 * sizeof(unsigned);
    if (!c->bound_slot) HIPCHK(c, hipMalloc(&c->bound_slot, bytes));
    HIPCHK(c, hipMemsetAsync(c->bound_slot, 0, bytes, c->stream));
    KPar P = make_kpar(c);
    hipLaunchKernelGGL(k_bound, cell_grid(c), dim3(BX, BY), 0, c->stream, P,
                       (unsigned(*)[4])c->bound_slot, c->H[cur], c->qx[cur], c->qy[cur], c->b[cur]);
    HIPCHK(c, hipGetLastError());
    unsigned m[NSLOT][4];
    if ((rc = stage_to_host(c, m, c->bound_slot, bytes))) return rc;
    unsigned a = 0, b = 0, d = 0, bad = 0;
    for (int q = 0; q < NSLOT; ++q) {
        a = std::max(a, m[q][0]); b = std::max(b, m[q][1]); d = std::max(d, m[q][2]);
        bad = std::max(bad, m[q][3]);
    }
    if (bad) return fail(c, SW_ERR_NONFINITE, "sw_step_bound: a field is not finite");
    float fa, fb, fd;
    std::memcpy(&fa, &a, 4); std::memcpy(&fb, &b, 4); std::memcpy(&fd, &d, 4);
    // the K3 reading of Eq. 7 (cell size h = dx), capped at dt_max
    const double h = c->grid.dx, vp = fa, vs = fb, D = fd;
    const double t0 = vp > 0.0 ? h / (2.0 * vp) : INFINITY;
    const double t1 = vs > 0.0 ? h / vs : INFINITY;
    const double t2 = D > 0.0 ? h * h / (2.0 * D) : INFINITY;
    const double bound = c->par.cfl * std::min(t0, std::min(t1, t2));
    *dt = bound < c->par.dt_max ? bound : c->par.dt_max;
    return SW_OK;
}

int sw_get_step_log(sw_ctx *c, int32_t n, sw_step_record *out, int32_t *count)
{
    if (!c || n < 0 || (n > 0 && !out)) return SW_ERR_ARG;
    Ctrl hc;
    int rc = read_ctrl(c, &hc);
    if (rc) return rc;
    const int taken = hc.kdev;  // steps published since the state was set
    const int m = std::min(std::min(n, taken), kStepLog);
    if (count) *count = m;
    if (m == 0) return SW_OK;
    std::vector<StepRec> ring(kStepLog);
    if ((rc = stage_to_host(c, ring.data(), c->steplog, kStepLog * sizeof(StepRec)))) return rc;
    for (int q = 0; q < m; ++q) {  // oldest first
        const StepRec &r = ring[(taken - m + q) & (kStepLog - 1)];
        sw_step_record &o = out[q];
        o.step = c->step0 + r.step;
        o.t = r.t; o.dt = r.dt; o.vp = r.vp; o.vs = r.vs; o.D = r.D; o.inflow = r.q;
        o.binding = r.binding; o.reserved = 0;
    }
    return SW_OK;
}

int sw_get_sums(sw_ctx *c, sw_sums *out)
{
    if (!c || !out) return SW_ERR_ARG;
    Ctrl hc;
    int rc = read_ctrl(c, &hc);
    if (rc) return rc;
    int cur = current_buffer(c, hc);
    KPar P = make_kpar(c);
    hipLaunchKernelGGL(k_sums1, dim3(c->nsum_blocks), dim3(SUM_THREADS), 0, c->stream, P,
                       c->H[cur], c->b[cur], c->part, c->sum_rows);
    int nb = 2 * (c->nx + c->ny);
    hipLaunchKernelGGL(k_sums2, dim3(1), dim3(SUM_THREADS), 0, c->stream, c->part, c->nsum_blocks,
                       c->bnd, nb, c->sums);
    HIPCHK(c, hipGetLastError());
    double s[6];
    std::vector<uint8_t> act(ntiles(c));
    if ((rc = stage_to_host(c, s, c->sums, sizeof(s)))) return rc;
    if ((rc = stage_to_host(c, act.data(), act_flags(c, cur), act.size()))) return rc;
    int64_t nact = 0;
    for (size_t t = 0; t < act.size(); ++t) nact += act[t] ? 1 : 0;
    double dx2 = c->grid.dx * c->grid.dx;
    int64_t kk = hc.err ? hc.err_k : c->k;
    memset(out, 0, sizeof(*out));
    out->t = hc.t[kk & 1];
    out->last_dt = hc.last_dt;
    out->water_volume = s[0] * dx2;
    out->sediment_volume = s[1] * dx2;
    out->wet_cells = (int64_t)s[2];
    out->water_boundary_out = s[3];
    out->sed_boundary_out = s[4];
    out->water_source_in = hc.in_w;
    out->sed_source_in = hc.in_s;
    out->vp = hc.vp; out->vs = hc.vs; out->D = hc.D;
    out->step = c->step0 + kk;
    out->active_tiles = (c->par.flags & SW_FLAG_UNFUSED) ? -1 : nact;
    out->cells_lagrange = (int64_t)hc.work[0];
    out->cells_euler = (int64_t)hc.work[1];
    out->binding_term = hc.binding;
    out->error = hc.err;
    out->graph_builds = c->graph_builds;
    out->water_rain_in = hc.in_rain;
    out->water_absorbed = s[5] * dx2;
    return SW_OK;
}

int sw_save_begin(sw_ctx *c)
{
    if (!c) return SW_ERR_ARG;
    if (!c->have_state) return fail(c, SW_ERR_STATE, "save before sw_set_state");
    if (c->save_pending) return fail(c, SW_ERR_STATE, "the previous save was not collected");
    const size_t dense = (size_t)c->nx * c->ny;
    if (!c->snap) {
        HIPCHK(c, hipMalloc(&c->snap, 4 * c->plane * sizeof(float)));
        HIPCHK(c, hipMalloc(&c->snap_ctrl, sizeof(Ctrl)));
        HIPCHK(c, hipHostMalloc((void **)&c->snap_host, 4 * dense * sizeof(float) + sizeof(Ctrl),
                                hipHostMallocDefault));
        HIPCHK(c, hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_snap, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_copied, hipEventDisableTiming));
    }
    // on the solver's stream, after the queued steps: a device copy of the
    // current level (the steps after it may overwrite that level)
    const int cur = (int)(c->k & 1);
    const float *src[4] = {c->H[cur], c->qx[cur], c->qy[cur], c->b[cur]};
    for (int f = 0; f < 4; ++f)
        HIPCHK(c, hipMemcpyAsync(c->snap + f * c->plane, src[f], c->plane * sizeof(float),
                                 hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->snap_ctrl, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipEventRecord(c->ev_snap, c->stream));
    // on the copy stream: the snapshot to pinned host memory
    HIPCHK(c, hipStreamWaitEvent(c->copy_stream, c->ev_snap, 0));
    for (int f = 0; f < 4; ++f)
        HIPCHK(c, hipMemcpy2DAsync(c->snap_host + f * dense, c->nx * sizeof(float),
                                   c->snap + f * c->plane, c->pitch * sizeof(float),
                                   c->nx * sizeof(float), c->ny, hipMemcpyDeviceToHost,
                                   c->copy_stream));
    HIPCHK(c, hipMemcpyAsync(c->snap_host + 4 * dense, c->snap_ctrl, sizeof(Ctrl),
                             hipMemcpyDeviceToHost, c->copy_stream));
    HIPCHK(c, hipEventRecord(c->ev_copied, c->copy_stream));
    c->save_pending = true;
    c->save_k = c->k;
    return SW_OK;
}

int sw_save_wait(sw_ctx *c, float *h, float *hu, float *hv, float *b, double *t, int64_t *step)
{
    if (!c) return SW_ERR_ARG;
    if (!c->save_pending) return fail(c, SW_ERR_STATE, "no save in flight");
    HIPCHK(c, hipEventSynchronize(c->ev_copied));
    c->save_pending = false;
    const size_t dense = (size_t)c->nx * c->ny;
    float *dst[4] = {h, hu, hv, b};
    for (int f = 0; f < 4; ++f)
        if (dst[f]) std::memcpy(dst[f], c->snap_host + f * dense, dense * sizeof(float));
    Ctrl hc;
    std::memcpy(&hc, c->snap_host + 4 * dense, sizeof(Ctrl));
    if (t) *t = hc.t[c->save_k & 1];
    if (step) *step = c->step0 + c->save_k;
    if (hc.err) return fail(c, hc.err, "device error raised at step " + std::to_string(hc.err_k));
    return SW_OK;
}

// Checkpoint blob: a fixed header, the dense planes h, hu, hv, b and the bed
// residual of the current state, then the boundary accumulators.
struct CkptHeader {
    char magic[8];           // "CSPHCKP1"
    int32_t nx, ny, ctrl_bytes, nb;
    int64_t step;            // step counter of the saved state
    double t;                // model time of the saved state
    int32_t par;             // buffer parity of the saved ring entries
    int32_t extra;           // bit 0: absorbed depths (FP64 plane), bit 1: rainfall residual plane follow
    Ctrl ctrl;               // device control block (time ring, source balances, maxima)
};

static size_t ckpt_bytes(const sw_ctx *c)
{
    const size_t n = (size_t)c->nx * c->ny, nb = 4 * (size_t)(c->nx + c->ny);
    return sizeof(CkptHeader) + 5 * n * sizeof(float) + nb * sizeof(double) +
           (c->ab ? c->plane * sizeof(double) : 0) + (c->rh ? c->plane * sizeof(float) : 0);
}

int sw_checkpoint_size(const sw_ctx *c, int64_t *bytes)
{
    if (!c || !bytes) return SW_ERR_ARG;
    *bytes = (int64_t)ckpt_bytes(c);
    return SW_OK;
}

int sw_checkpoint_save(sw_ctx *c, void *buf, int64_t bytes)
{
    if (!c || !buf) return SW_ERR_ARG;
    if (bytes < (int64_t)ckpt_bytes(c)) return fail(c, SW_ERR_ARG, "checkpoint buffer too small");
    if (!c->have_state) return fail(c, SW_ERR_STATE, "checkpoint before sw_set_state");
    CkptHeader h;
    std::memset(&h, 0, sizeof(h));
    int rc = read_ctrl(c, &h.ctrl);
    if (rc) return rc;
    if (h.ctrl.err) return fail(c, SW_ERR_STATE, "checkpoint with a pending device error");
    std::memcpy(h.magic, "CSPHCKP1", 8);
    h.nx = c->nx;
    h.ny = c->ny;
    h.ctrl_bytes = (int32_t)sizeof(Ctrl);
    h.nb = 4 * (c->nx + c->ny);
    h.par = (int32_t)(c->k & 1);
    h.extra = (c->ab ? 1 : 0) | (c->rh ? 2 : 0);
    h.step = c->step0 + c->k;
    h.t = h.ctrl.t[h.par];
    char *out = (char *)buf;
    std::memcpy(out, &h, sizeof(h));
    out += sizeof(h);
    const size_t n = (size_t)c->nx * c->ny;
    const int cur = h.par;
    const float *planes[5] = {c->H[cur], c->qx[cur], c->qy[cur], c->b[cur], c->rb};
    for (int f = 0; f < 5; ++f, out += n * sizeof(float))
        if ((rc = download_plane(c, (float *)out, planes[f], SW_PTR_HOST))) return rc;
    if ((rc = stage_to_host(c, out, c->bnd, (size_t)h.nb * sizeof(double)))) return rc;
    out += (size_t)h.nb * sizeof(double);
    if (c->ab && (rc = stage_to_host(c, out, c->ab, c->plane * sizeof(double)))) return rc;
    if (c->ab) out += c->plane * sizeof(double);
    if (c->rh) rc = stage_to_host(c, out, c->rh, c->plane * sizeof(float));
    return rc;
}

int sw_checkpoint_load(sw_ctx *c, const void *buf, int64_t bytes)
{
    if (!c || !buf) return SW_ERR_ARG;
    if (bytes < (int64_t)sizeof(CkptHeader)) return fail(c, SW_ERR_ARG, "checkpoint too short");
    CkptHeader h;
    std::memcpy(&h, buf, sizeof(h));
    if (std::memcmp(h.magic, "CSPHCKP1", 8) != 0 || h.ctrl_bytes != (int32_t)sizeof(Ctrl))
        return fail(c, SW_ERR_ARG, "not a checkpoint of this library");
    if (h.nx != c->nx || h.ny != c->ny || h.nb != 4 * (c->nx + c->ny))
        return fail(c, SW_ERR_ARG, "checkpoint of another grid");
    if (bytes < (int64_t)ckpt_bytes(c)) return fail(c, SW_ERR_ARG, "checkpoint too short");
    if (h.extra != ((c->ab ? 1 : 0) | (c->rh ? 2 : 0)))
        return fail(c, SW_ERR_ARG, "checkpoint of a context with other rain or absorption settings");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const char *in = (const char *)buf + sizeof(h);
    const size_t n = (size_t)c->nx * c->ny;
    c->k = 0;
    float *planes[5] = {c->H[0], c->qx[0], c->qy[0], c->b[0], c->rb};
    int rc;
    for (int f = 0; f < 5; ++f, in += n * sizeof(float))
        if ((rc = upload_plane(c, planes[f], (const float *)in, SW_PTR_HOST))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->b[1], c->b[0], c->plane * sizeof(float), hipMemcpyDeviceToDevice,
                             c->stream));
    HIPCHK(c, hipMemsetAsync(c->QLx, 0, 2 * c->plane * sizeof(float), c->stream));
    if ((rc = stage_to_device(c, c->bnd, in, (size_t)h.nb * sizeof(double)))) return rc;
    in += (size_t)h.nb * sizeof(double);
    if (c->ab && (rc = stage_to_device(c, c->ab, in, c->plane * sizeof(double)))) return rc;
    if (c->ab) in += c->plane * sizeof(double);
    if (c->rh && (rc = stage_to_device(c, c->rh, in, c->plane * sizeof(float)))) return rc;
    // the saved control block with its ring entries moved to parity 0
    Ctrl k0 = h.ctrl;
    std::memset(k0.slot, 0, sizeof(k0.slot));
    k0.t[0] = h.t;
    k0.t[1] = h.t;
    k0.dt[0] = h.ctrl.dt[h.par];
    k0.qmid[0] = h.ctrl.qmid[h.par];
    k0.kdev = 0;
    k0.err = 0;
    k0.err_k = 0;
    if ((rc = stage_to_device(c, c->ctrl, &k0, sizeof(Ctrl)))) return rc;
    c->t0 = h.t;
    c->step0 = h.step;
    c->have_state = true;
    c->dirty = true;
    return SW_OK;
}

const char *sw_last_error(const sw_ctx *c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

// ===========================================================================
// Allocation-free advance: the kernels of sw_advance on the default strip
// shape, with every buffer they need (both state levels, the Lagrangian
// momentum, the J0 planes, the bed residual, the boundary accumulators, tile
// flags and maxima, work lists, control block) carved from one file-scope
// device array.  Loading, set-up and readback are kernels too (no memset or
// memcpy nodes), so the whole call can be captured into a HIP graph.
// ===========================================================================

static __device__ __align__(256) unsigned char scratch[SW_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
// Device address of `scratch` on each GPU (hipGetSymbolAddress, taken once
// per device with that device current): host code never passes the array's
// own name to a kernel or a runtime call.
unsigned char *g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Offsets (bytes, 256-aligned) of the parts of the array for one grid.
struct NoallocLayout {
    size_t planes, bnd, tflags, tmax, sched, ctrl, total;
    int pitch, ntx, nty, chunks;
    size_t plane, tiles;
};

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

NoallocLayout noalloc_layout(int nx, int ny)
{
    NoallocLayout L{};
    L.pitch = (nx + 63) / 64 * 64;
    L.plane = (size_t)L.pitch * ny;
    L.ntx = (nx + kShapes[kDefaultShape].tx - 1) / kShapes[kDefaultShape].tx;
    L.nty = (ny + kShapes[kDefaultShape].ty - 1) / kShapes[kDefaultShape].ty;
    L.tiles = (size_t)L.ntx * L.nty;
    const int ch = list_chunk((int)L.tiles);
    L.chunks = ((int)L.tiles + ch - 1) / ch;
    L.planes = 0;
    L.bnd = up256(17 * L.plane * sizeof(float));
    L.tflags = L.bnd + up256(4 * (size_t)(nx + ny) * sizeof(double));
    L.tmax = L.tflags + up256(4 * L.tiles);
    L.sched = L.tmax + up256(2 * L.tiles * sizeof(uint4));
    L.ctrl = L.sched + up256(sched_layout(L.chunks, L.tiles).total * sizeof(int));
    L.total = L.ctrl + up256(sizeof(Ctrl));
    return L;
}

// Zero a 4-byte-word range of the array (grid-stride).
__global__ void k_noalloc_zero(uint32_t *p, size_t n)
{
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (size_t)gridDim.x * blockDim.x)
        p[q] = 0u;
}

// Fresh control block with the model time t0.
__global__ void k_noalloc_ctrl(Ctrl *ctrl, double t0)
{
    uint32_t *w = reinterpret_cast<uint32_t *>(ctrl);
    for (size_t q = threadIdx.x; q < sizeof(Ctrl) / 4; q += blockDim.x) w[q] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) ctrl->t[0] = t0;
}

// The caller's dense [ny][nx] state and bed into the pitched planes of level
// 0 (the bed into both levels); a cell with zero depth gets zero discharge.
// A negative or non-finite depth, or a non-finite discharge or bed, raises
// SW_ERR_ARG in the control block before step 0, so no step runs.
__global__ void k_noalloc_load(KPar P, Ctrl *ctrl, const float *__restrict__ h,
                               const float *__restrict__ hu, const float *__restrict__ hv,
                               const float *__restrict__ b, float *H, float *Qx, float *Qy,
                               float *B0, float *B1)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= P.nx) return;
    const size_t s = (size_t)j * P.nx + i, d = (size_t)j * P.pitch + i;
    float hh = h[s], u = hu[s], v = hv[s];
    const float bb = b[s];
    if (!(hh >= 0.0f) || !isfinite(hh) || !isfinite(u) || !isfinite(v) || !isfinite(bb))
        ctrl->err = SW_ERR_ARG;  // the same value from every failing lane; err_k stays 0
    if (hh == 0.0f) { hh = 0.0f; u = 0.0f; v = 0.0f; }
    H[d] = hh; Qx[d] = u; Qy[d] = v; B0[d] = bb; B1[d] = bb;
}

// The current state (level nsteps & 1, or the start of the failing step after
// a device error) back into the caller's dense arrays; the model time and the
// error code into the optional device outputs.
__global__ void k_noalloc_store(KPar P, const Ctrl *__restrict__ ctrl, int nsteps, Inst I,
                                float *h, float *hu, float *hv, float *b, double *t_out,
                                int32_t *err_out)
{
    const int cur = ctrl->err ? (ctrl->err_k & 1) : (nsteps & 1);
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i == 0 && j == 0) {
        if (t_out) *t_out = ctrl->t[cur];
        if (err_out) *err_out = ctrl->err;
    }
    if (i >= P.nx) return;
    const size_t s = (size_t)j * P.nx + i, d = (size_t)j * P.pitch + i;
    h[s] = I.H[cur][d]; hu[s] = I.qx[cur][d]; hv[s] = I.qy[cur][d]; b[s] = I.b[cur][d];
}

// Message for the caller's buffer (no heap allocation on any path).
int noalloc_fail(char *errbuf, int32_t errbuf_len, int code, const char *fmt, ...)
{
    if (errbuf && errbuf_len > 0) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(errbuf, (size_t)errbuf_len, fmt, ap);
        va_end(ap);
    }
    return code;
}

// The array's address on the current device (looked up on the first call).
int noalloc_scratch(unsigned char **out, char *errbuf, int32_t errbuf_len)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return noalloc_fail(errbuf, errbuf_len, SW_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return noalloc_fail(errbuf, errbuf_len, SW_ERR_ARG, "device %d beyond the library's table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return noalloc_fail(errbuf, errbuf_len, SW_ERR_HIP, "hipGetSymbolAddress(scratch): %s",
                                hipGetErrorString(e));
        g_scratch[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch[dev];
    return SW_OK;
}

}  // namespace

extern "C" {

int sw_advance_noalloc(const sw_grid *grid, const sw_params *params, float manning, float d50,
                       float psi, float *h, float *hu, float *hv, float *b, int32_t nsteps,
                       double dt_fixed, double t0, double *t_out, int32_t *err_out,
                       void *hip_stream, char *errbuf, int32_t errbuf_len)
{
    auto bad = [&](const char *m) { return noalloc_fail(errbuf, errbuf_len, SW_ERR_ARG, "%s", m); };
    if (errbuf && errbuf_len > 0) errbuf[0] = '\0';
    if (!grid || !params) return bad("grid or params is NULL");
    if (!h || !hu || !hv || !b) return bad("a field pointer is NULL");
    if (grid->nx < 1 || grid->ny < 1 || !(grid->dx > 0.0)) return bad("nx, ny must be >= 1 and dx > 0");
    if (grid->nx > (1 << 24) || grid->ny > (1 << 24)) return bad("grid larger than the scratch array");
    for (int s = 0; s < 4; ++s)
        if (grid->bc[s] != SW_BC_WALL && grid->bc[s] != SW_BC_OPEN) return bad("unknown boundary kind");
    if (params->sed_law < SW_SED_NONE || params->sed_law > SW_SED_EQ4) return bad("unknown sediment law");
    if (params->limiter < SW_LIM_MINMOD || params->limiter > SW_LIM_SUPERBEE) return bad("unknown limiter");
    if (params->hll_speeds != SW_HLL_DAVIS && params->hll_speeds != SW_HLL_TWO_RAREFACTION)
        return bad("unknown wave-speed estimate");
    if (!(params->cfl > 0.0) || !(params->g > 0.0) || !(params->eps_dry > 0.0))
        return bad("cfl, g and eps_dry must be > 0");
    if (params->flags & SW_FLAG_UNFUSED) return bad("the unfused sequence is not available here");
    if (!(manning >= 0.0f) || !(d50 > 0.0f) || !(psi >= 0.0f && psi < 1.0f))
        return bad("manning >= 0, d50 > 0 and 0 <= psi < 1 are required");
    if (nsteps < 0) return bad("nsteps must be >= 0");
    if (!(dt_fixed >= 0.0) || !std::isfinite(dt_fixed) || !std::isfinite(t0))
        return bad("dt_fixed must be finite and >= 0, t0 finite");
    const NoallocLayout L = noalloc_layout(grid->nx, grid->ny);
    if (L.total > (size_t)SW_NOALLOC_SCRATCH_BYTES)
        return noalloc_fail(errbuf, errbuf_len, SW_ERR_ARG,
                            "a %d x %d grid needs %zu bytes of scratch, more than the %zu the "
                            "library holds", grid->nx, grid->ny, L.total,
                            (size_t)SW_NOALLOC_SCRATCH_BYTES);
    unsigned char *base = nullptr;
    int rc = noalloc_scratch(&base, errbuf, errbuf_len);
    if (rc) return rc;

    // a context on the stack whose buffers all lie in the array (nothing of
    // it is allocated: its strings and vectors stay empty)
    sw_ctx c;
    c.grid = *grid;
    c.par = *params;
    c.stream = (hipStream_t)hip_stream;
    c.nx = grid->nx;
    c.ny = grid->ny;
    c.pitch = L.pitch;
    c.plane = L.plane;
    c.buf = reinterpret_cast<float *>(base + L.planes);
    for (int s = 0; s < 2; ++s) {
        c.H[s] = c.buf + (4 * s + 0) * c.plane;
        c.qx[s] = c.buf + (4 * s + 1) * c.plane;
        c.qy[s] = c.buf + (4 * s + 2) * c.plane;
        c.b[s] = c.buf + (4 * s + 3) * c.plane;
    }
    c.QLx = c.buf + 8 * c.plane;
    c.QLy = c.buf + 9 * c.plane;
    for (int s = 0; s < 2; ++s) {
        c.jx[s] = c.buf + (10 + 3 * s) * c.plane;
        c.jy[s] = c.buf + (11 + 3 * s) * c.plane;
        c.jm[s] = c.buf + (12 + 3 * s) * c.plane;
    }
    c.rb = c.buf + 16 * c.plane;
    c.nM_s = manning;
    c.d50_s = d50;
    c.psi_s = psi;
    c.bnd = reinterpret_cast<double *>(base + L.bnd);
    c.tflags = base + L.tflags;
    c.tmax = reinterpret_cast<uint4 *>(base + L.tmax);
    c.sched = reinterpret_cast<int *>(base + L.sched);
    c.ctrl = reinterpret_cast<Ctrl *>(base + L.ctrl);
    c.shape = kDefaultShape;
    c.ntx = L.ntx;
    c.nty = L.nty;
    c.max_tiles = L.tiles;
    c.max_chunks = L.chunks;
    c.t0 = t0;

    // set-up: clear the bed residual, balances, flags, maxima and lists; a
    // fresh control block; the caller's state into level 0
    hipStream_t st = c.stream;
    struct Range {
        void *p;
        size_t bytes;
    } clear[] = {{c.rb, c.plane * sizeof(float)},
                 {c.bnd, 4 * (size_t)(c.nx + c.ny) * sizeof(double)},
                 {c.tflags, 4 * L.tiles},
                 {c.tmax, 2 * L.tiles * sizeof(uint4)},
                 {c.sched, sched_layout(L.chunks, L.tiles).total * sizeof(int)}};
    for (const Range &r : clear) {
        const size_t words = (r.bytes + 3) / 4;
        const int blocks = (int)std::min<size_t>(1024, (words + 255) / 256);
        hipLaunchKernelGGL(k_noalloc_zero, dim3(std::max(blocks, 1)), dim3(256), 0, st,
                           static_cast<uint32_t *>(r.p), words);
    }
    hipLaunchKernelGGL(k_noalloc_ctrl, dim3(1), dim3(256), 0, st, c.ctrl, t0);
    const KPar P = make_kpar(&c);
    const dim3 rows((c.nx + 255) / 256, c.ny);
    hipLaunchKernelGGL(k_noalloc_load, rows, dim3(256), 0, st, P, c.ctrl, h, hu, hv, b, c.H[0],
                       c.qx[0], c.qy[0], c.b[0], c.b[1]);
    const StepArgs A = make_step_args(&c, dt_fixed > 0.0 ? 1 : 0, dt_fixed);
    const Inst I = make_inst(&c, A);
    launch_stage(c.shape, kPrepare, st, I, 0);
    for (int32_t s = 0; s < nsteps; ++s) enqueue_tiled_step(&c, st, s & 1, P, A);
    hipLaunchKernelGGL(k_noalloc_store, rows, dim3(256), 0, st, P, c.ctrl, nsteps, I, h, hu, hv,
                       b, t_out, err_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return noalloc_fail(errbuf, errbuf_len, SW_ERR_HIP, "kernel launch: %s", hipGetErrorString(e));
    return SW_OK;
}

}  // extern "C"

// ===========================================================================
// Ensembles: several grids advanced together, one launch per stage per step.
// ===========================================================================

struct swb_ctx {
    std::vector<sw_ctx *> mem;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    Inst *d_insts = nullptr;
    int *d_table = nullptr;          // stage table, then (strips) the K3a table
    int ntab = 0, ndtab = 0;
    int lthr = LT;  // threads of a K3a workgroup (the widest member segment's)
    int shape = kDefaultShape;
    bool cs = false;  // some member reads per-cell soil or source planes
    bool var = false; // some member runs a limiter or wave-speed estimate other than minmod + Davis
    bool f2 = false;  // the members run the second-order Lagrangian force
    hipGraphExec_t gexec = nullptr;
    hipGraphExec_t gexec_long = nullptr;
    bool built = false;
    std::vector<uint64_t> gen;  // each member's args_gen when the tables were built
    std::string err;
};

namespace {

int bfail(swb_ctx *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    return code;
}

#define BHIPCHK(b, call)                                                                   \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return bfail((b), SW_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Instance table and tile table for the current member inputs and shape.
int batch_build(swb_ctx *b)
{
    const int n = (int)b->mem.size();
    std::vector<Inst> insts(n);
    std::vector<int> table, dtable;
    int lthr = 256;
    b->cs = false;
    b->var = false;
    b->f2 = (b->mem[0]->par.flags & SW_FLAG_FORCE2) != 0;
    for (int m = 0; m < n; ++m) {
        sw_ctx *c = b->mem[m];
        if (c->shape != b->shape) set_shape(c, b->shape);
        if (c->dirty) {
            int rc = prepare(c);
            if (rc) return bfail(b, rc, "member " + std::to_string(m) + ": " + c->err);
        }
        insts[m] = make_inst(c, make_step_args(c, 0, 0.0));
        b->cs = b->cs || cell_soil(insts[m].P);
        b->var = b->var || insts[m].P.variant;
        if (is_strip(b->shape)) {  // one entry per workgroup of SWAVES list entries
            const int blocks = (c->ntx * c->nty + SWAVES - 1) / SWAVES;
            for (int w = 0; w < blocks; ++w) {
                table.push_back(m);
                table.push_back(w);
            }
            for (int k = 0; k < insts[m].nchunk; ++k) {
                dtable.push_back(m);
                dtable.push_back(k);
            }
            lthr = std::max(lthr, list_threads(insts[m].chunk));
        } else {  // one entry per tile
            for (int by = 0; by < c->nty; ++by)
                for (int bx = 0; bx < c->ntx; ++bx) {
                    table.push_back(m);
                    table.push_back(bx);
                    table.push_back(by);
                }
        }
    }
    const int per = is_strip(b->shape) ? 2 : 3;
    b->ntab = (int)(table.size() / per);
    b->ndtab = (int)(dtable.size() / 2);
    b->lthr = lthr;
    b->gen.resize(n);
    for (int m = 0; m < n; ++m) b->gen[m] = b->mem[m]->args_gen;
    table.insert(table.end(), dtable.begin(), dtable.end());
    (void)hipFree(b->d_insts);
    (void)hipFree(b->d_table);
    b->d_insts = nullptr;
    b->d_table = nullptr;
    BHIPCHK(b, hipMalloc(&b->d_insts, n * sizeof(Inst)));
    BHIPCHK(b, hipMalloc(&b->d_table, table.size() * sizeof(int)));
    {  // through a pinned temporary (no on-the-fly pinning of the host vectors)
        const size_t bi = n * sizeof(Inst), bt = table.size() * sizeof(int);
        char *tmp = nullptr;
        BHIPCHK(b, hipHostMalloc((void **)&tmp, bi + bt, hipHostMallocDefault));
        std::memcpy(tmp, insts.data(), bi);
        std::memcpy(tmp + bi, table.data(), bt);
        hipError_t e1 = hipMemcpyAsync(b->d_insts, tmp, bi, hipMemcpyHostToDevice, b->stream);
        hipError_t e2 = hipMemcpyAsync(b->d_table, tmp + bi, bt, hipMemcpyHostToDevice, b->stream);
        hipError_t e3 = hipStreamSynchronize(b->stream);
        (void)hipHostFree(tmp);
        BHIPCHK(b, e1);
        BHIPCHK(b, e2);
        BHIPCHK(b, e3);
    }
    if (b->gexec_long) {
        (void)hipGraphExecDestroy(b->gexec_long);
        b->gexec_long = nullptr;
    }
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    b->built = true;
    return SW_OK;
}

void batch_step(swb_ctx *b, hipStream_t st, int par)
{
    const int n = (int)b->mem.size();
    const int *dtab = b->d_table + 2 * b->ntab;
    launch_batch(b->shape, kDt, st, b->d_insts, n, b->d_table, b->ntab, dtab, b->ndtab, b->lthr, par,
                 b->cs, b->var, b->f2);
    launch_batch(b->shape, kLagrange, st, b->d_insts, n, b->d_table, b->ntab, dtab, b->ndtab, b->lthr, par,
                 b->cs, b->var, b->f2);
    launch_batch(b->shape, kEuler, st, b->d_insts, n, b->d_table, b->ntab, dtab, b->ndtab, b->lthr, par,
                 b->cs, b->var, b->f2);
}

// The member tables and graphs hold every member's kernel arguments: they are
// rebuilt when one of them changed (soil, sources, shape).  A member with a
// new state, bed or time only needs its set-up pass.
bool batch_needs_build(const swb_ctx *b)
{
    if (!b->built) return true;
    for (size_t m = 0; m < b->mem.size(); ++m)
        if (b->mem[m]->args_gen != b->gen[m] || b->mem[m]->shape != b->shape) return true;
    return false;
}

}  // namespace

extern "C" {

int swb_create(int32_t n, sw_ctx *const *members, swb_ctx **out)
{
    if (!out || n < 1 || !members) return SW_ERR_ARG;
    *out = nullptr;
    for (int32_t m = 0; m < n; ++m) {
        if (!members[m]) return SW_ERR_ARG;
        if (members[m]->stream != members[0]->stream) return SW_ERR_ARG;
        if (members[m]->par.flags & SW_FLAG_UNFUSED) return SW_ERR_ARG;
        // one Lagrangian kernel serves every member: one force order
        if ((members[m]->par.flags ^ members[0]->par.flags) & SW_FLAG_FORCE2) return SW_ERR_ARG;
        for (int32_t q = 0; q < m; ++q)
            if (members[q] == members[m]) return SW_ERR_ARG;
    }
    swb_ctx *b = new swb_ctx();
    b->mem.assign(members, members + n);
    b->stream = members[0]->stream;
    *out = b;
    return SW_OK;
}

int swb_destroy(swb_ctx *b)
{
    if (!b) return SW_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->gexec_long) (void)hipGraphExecDestroy(b->gexec_long);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    (void)hipFree(b->d_insts);
    (void)hipFree(b->d_table);
    delete b;
    return SW_OK;
}

int swb_set_tile_shape(swb_ctx *b, int32_t tile_x, int32_t tile_y)
{
    if (!b) return SW_ERR_ARG;
    for (int sh = 0; sh < kNumShapes; ++sh)
        if (kShapes[sh].tx == tile_x && kShapes[sh].ty == tile_y) {
            if ((b->mem[0]->par.flags & SW_FLAG_FORCE2) && !is_strip(sh))
                return bfail(b, SW_ERR_ARG, "the second-order force runs on strip shapes only");
            BHIPCHK(b, hipStreamSynchronize(b->stream));
            b->shape = sh;
            b->built = false;
            return SW_OK;
        }
    return bfail(b, SW_ERR_ARG, "unknown tile shape");
}

int swb_advance(swb_ctx *b, int32_t nsteps)
{
    if (!b) return SW_ERR_ARG;
    if (nsteps < 0) return bfail(b, SW_ERR_ARG, "nsteps must be >= 0");
    const int par0 = (int)(b->mem[0]->k & 1);
    for (size_t m = 0; m < b->mem.size(); ++m) {
        if (!b->mem[m]->have_state)
            return bfail(b, SW_ERR_STATE, "member " + std::to_string(m) + " has no state");
        if ((int)(b->mem[m]->k & 1) != par0)
            return bfail(b, SW_ERR_STATE, "members are at steps of different parity");
    }
    if (batch_needs_build(b)) {
        int rc = batch_build(b);
        if (rc) return rc;
    }
    for (size_t m = 0; m < b->mem.size(); ++m)
        if (b->mem[m]->dirty) {
            int rc = prepare(b->mem[m]);
            if (rc) return bfail(b, rc, "member " + std::to_string(m) + ": " + b->mem[m]->err);
        }
    int32_t left = nsteps;
    auto advance_members = [&](int s) {
        for (sw_ctx *c : b->mem) c->k += s;
    };
    if (left > 0 && (b->mem[0]->k & 1)) {
        batch_step(b, b->stream, 1);
        BHIPCHK(b, hipGetLastError());
        advance_members(1);
        left--;
    }
    if (left >= 2) {
        if (!b->gexec) {  // graphs of one and of kLongPairs step pairs
            if (!b->cap) BHIPCHK(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
            for (int pairs : {1, kLongPairs}) {
                hipGraph_t g = nullptr;
                BHIPCHK(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
                for (int q = 0; q < pairs; ++q) {
                    batch_step(b, b->cap, 0);
                    batch_step(b, b->cap, 1);
                }
                BHIPCHK(b, hipStreamEndCapture(b->cap, &g));
                hipError_t e = hipGraphInstantiate(pairs == 1 ? &b->gexec : &b->gexec_long, g, nullptr,
                                                   nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess)
                    return bfail(b, SW_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
        }
        for (; left >= 2 * kLongPairs; left -= 2 * kLongPairs) {
            BHIPCHK(b, hipGraphLaunch(b->gexec_long, b->stream));
            advance_members(2 * kLongPairs);
        }
        for (; left >= 2; left -= 2) {
            BHIPCHK(b, hipGraphLaunch(b->gexec, b->stream));
            advance_members(2);
        }
    }
    for (; left > 0; --left) {
        batch_step(b, b->stream, (int)(b->mem[0]->k & 1));
        BHIPCHK(b, hipGetLastError());
        advance_members(1);
    }
    return SW_OK;
}

int swb_sync(swb_ctx *b)
{
    if (!b) return SW_ERR_ARG;
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    for (size_t m = 0; m < b->mem.size(); ++m) {
        int rc = sw_sync(b->mem[m]);
        if (rc) return bfail(b, rc, "member " + std::to_string(m) + ": " + b->mem[m]->err);
    }
    return SW_OK;
}

const char *swb_last_error(const swb_ctx *b) { return b ? b->err.c_str() : "null batch"; }

int swb_autotune(swb_ctx *b, int32_t nsteps, int32_t *tile_x, int32_t *tile_y)
{
    if (!b) return SW_ERR_ARG;
    if (nsteps < 1) return bfail(b, SW_ERR_ARG, "nsteps must be >= 1");
    const int n = (int)b->mem.size();
    const int par0 = (int)(b->mem[0]->k & 1);
    for (int m = 0; m < n; ++m) {
        if (!b->mem[m]->have_state)
            return bfail(b, SW_ERR_STATE, "member " + std::to_string(m) + " has no state");
        if ((int)(b->mem[m]->k & 1) != par0)
            return bfail(b, SW_ERR_STATE, "members are at steps of different parity");
    }
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    std::vector<StateKeep> keep(n);
    int rc = SW_OK;
    for (int m = 0; m < n && !rc; ++m)
        if ((rc = keep_save(b->mem[m], keep[m]))) rc = bfail(b, rc, "member " + std::to_string(m) + ": " + b->mem[m]->err);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = bfail(b, SW_ERR_HIP, "hipEventCreate");
    const int shape0 = b->shape;
    int best = shape0;
    float best_ms = 0.0f;
    bool timed = false;
    for (int sh = 0; sh < kNumShapes && !rc; ++sh) {
        if ((b->mem[0]->par.flags & SW_FLAG_FORCE2) && !is_strip(sh)) continue;
        b->shape = sh;
        b->built = false;
        if ((rc = batch_build(b))) break;
        for (int m = 0; m < n && !rc; ++m)
            if (b->mem[m]->dirty && (rc = prepare(b->mem[m])))
                rc = bfail(b, rc, "member " + std::to_string(m) + ": " + b->mem[m]->err);
        if (rc) break;
        if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = bfail(b, SW_ERR_HIP, "hipEventRecord"); break; }
        for (int32_t s = 0; s < nsteps; ++s) {
            batch_step(b, b->stream, (int)(b->mem[0]->k & 1));
            for (sw_ctx *c : b->mem) c->k++;
        }
        if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = bfail(b, SW_ERR_HIP, "kernel timing failed");
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (!timed || ms < best_ms) { best_ms = ms; best = sh; timed = true; }
        for (int m = 0; m < n && !rc; ++m)
            if ((rc = keep_restore(b->mem[m], keep[m])))
                rc = bfail(b, rc, "member " + std::to_string(m) + ": " + b->mem[m]->err);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (int m = 0; m < n; ++m) {
        if (!rc && keep[m].planes && (rc = keep_restore(b->mem[m], keep[m])))
            rc = bfail(b, rc, "member " + std::to_string(m) + ": " + b->mem[m]->err);
        keep_free(keep[m]);
    }
    b->shape = rc ? shape0 : best;
    b->built = false;
    if (rc) return rc;
    if (tile_x) *tile_x = kShapes[best].tx;
    if (tile_y) *tile_y = kShapes[best].ty;
    return SW_OK;
}

// Per-member access through the batch: the members are ordinary contexts, so
// each call forwards to the member's own entry point (and its error text is
// copied into the batch's).
static int bmember(swb_ctx *b, int32_t m, sw_ctx **c)
{
    if (!b) return SW_ERR_ARG;
    if (m < 0 || m >= (int32_t)b->mem.size()) return bfail(b, SW_ERR_ARG, "member index out of range");
    *c = b->mem[m];
    return SW_OK;
}
static int bforward(swb_ctx *b, sw_ctx *c, int rc)
{
    if (rc) b->err = c->err;
    return rc;
}

int swb_get_fields(swb_ctx *b, int32_t m, float *h, float *hu, float *hv, float *bed, int ptr_kind)
{
    sw_ctx *c = nullptr;
    int rc = bmember(b, m, &c);
    return rc ? rc : bforward(b, c, sw_get_fields(c, h, hu, hv, bed, ptr_kind));
}

int swb_get_sums(swb_ctx *b, int32_t m, sw_sums *out)
{
    sw_ctx *c = nullptr;
    int rc = bmember(b, m, &c);
    return rc ? rc : bforward(b, c, sw_get_sums(c, out));
}

int swb_set_state(swb_ctx *b, int32_t m, const float *h, const float *hu, const float *hv,
                  int ptr_kind)
{
    sw_ctx *c = nullptr;
    int rc = bmember(b, m, &c);
    return rc ? rc : bforward(b, c, sw_set_state(c, h, hu, hv, ptr_kind));
}

int swb_set_bed(swb_ctx *b, int32_t m, const float *bed, int ptr_kind)
{
    sw_ctx *c = nullptr;
    int rc = bmember(b, m, &c);
    return rc ? rc : bforward(b, c, sw_set_bed(c, bed, ptr_kind));
}

int swb_set_soil(swb_ctx *b, int32_t m, const float *manning, float manning_scalar, const float *d50,
                 float d50_scalar, const float *psi, float psi_scalar, int ptr_kind)
{
    sw_ctx *c = nullptr;
    int rc = bmember(b, m, &c);
    return rc ? rc
              : bforward(b, c, sw_set_soil(c, manning, manning_scalar, d50, d50_scalar, psi,
                                           psi_scalar, ptr_kind));
}

int swb_set_inflow(swb_ctx *b, int32_t m, const int32_t *cell_idx, const float *weight, int32_t n,
                   double q_base, double q_peak, double t_peak, double t_sigma)
{
    sw_ctx *c = nullptr;
    int rc = bmember(b, m, &c);
    return rc ? rc
              : bforward(b, c, sw_set_inflow(c, cell_idx, weight, n, q_base, q_peak, t_peak, t_sigma));
}

int swb_set_sed_sources(swb_ctx *b, int32_t m, const float *qb_plus, const float *qb_minus,
                        int ptr_kind)
{
    sw_ctx *c = nullptr;
    int rc = bmember(b, m, &c);
    return rc ? rc : bforward(b, c, sw_set_sed_sources(c, qb_plus, qb_minus, ptr_kind));
}

}  // extern "C"
