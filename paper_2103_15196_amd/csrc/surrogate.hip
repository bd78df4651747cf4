// surrogate.hip -- the learned surrogate of the CSPH-TVD step on gfx950: 3x3
// convolutions on the matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands,
// FP32 accumulation), training kernels (input and weight gradients on the
// matrix cores, Adam in FP32) and the surrogate step with its mass check and
// plain-solver fall back.
//
// Layouts.  Activations are BF16, channels last ("NHWC"): [img][y][x][C] with
// C = 8 for the 5-channel input (channels 5..7 zero) and C = 48 for the
// hidden layers.  A convolution is an implicit GEMM: output pixel m (16 per
// MFMA block, consecutive along x), output channel n (16 per block) and the
// reduction index k = tap * C + c over the 9 taps (ky, kx) and C channels,
// padded to a multiple of 32.  Lane l of a wavefront holds A[l % 16][8 (l/16)
// .. +7] (8 channels of one pixel at one tap: a 16-byte load), B[8 (l/16) ..
// +7][l % 16] and D[4 (l/16) .. +3][l % 16] (checked on the GPU).  Weights are
// packed once per update into exactly these per-lane B fragments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "csph.h"
#include "surrogate.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int MAXW = 48;      // widest layer
constexpr int CIN0 = 8;       // stored channels of the 5-channel input
constexpr int NT = 256;       // threads per workgroup
constexpr int NWAVE = NT / 64;

__device__ __forceinline__ unsigned short bf16_bits(float f)
{
    // round to nearest even (NaN kept quiet)
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// One layer's geometry: stored input channels (8 or 48), valid input and
// output channels, output channel blocks of 16, reduction chunks of 32.
struct Geo {
    int cs, cin, cout, nb, kc;
};

// ---------------------------------------------------------------------------
// Weight packing: B[k][n] = Wf[n][c][ky][kx] for k = (3 ky + kx) cs + c, in the
// per-lane fragment order [nb][kc][lane][8].  flip: the weights of the
// transposed convolution (input gradient), Wf[n][c][ky][kx] = W[c][n][2-ky][2-kx].
// ---------------------------------------------------------------------------
// One packing job: a layer's weights into the forward or transposed fragment
// order; the launch takes up to kPackJobs of them, one per row of its grid.
struct PackJob {
    const float *W;
    unsigned short *out;
    Geo g;
    int flip, wcin;
};
constexpr int kPackJobs = 16;
struct PackTable {
    PackJob j[kPackJobs];
};
__global__ void k_pack(PackTable t)
{
    const PackJob &J = t.j[blockIdx.y];
    const Geo g = J.g;
    const int total = g.nb * g.kc * 64 * 8;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        const int j = q & 7, lane = (q >> 3) & 63, f = q >> 9;
        const int kc = f % g.kc, nb = f / g.kc;
        const int k = 32 * kc + 8 * (lane >> 4) + j, n = 16 * nb + (lane & 15);
        const int tap = k / g.cs, c = k % g.cs;
        float v = 0.0f;
        if (tap < 9 && c < g.cin && n < g.cout) {
            const int ky = tap / 3, kx = tap % 3;
            // W is [wcout][wcin][3][3]
            v = J.flip ? J.W[((c * J.wcin + n) * 3 + (2 - ky)) * 3 + (2 - kx)]
                       : J.W[((n * J.wcin + c) * 3 + ky) * 3 + kx];
        }
        J.out[q] = bf16_bits(v);
    }
}

// ---------------------------------------------------------------------------
// Convolution on the matrix cores.  A workgroup of CW = 8 wavefronts owns a
// strip of TW = 64 output pixels of one image and marches down a segment of
// rows, 8 output rows per step (one per wavefront, two wavefronts per SIMD).
// Each step stages the 10 input rows they need (64 + 2 pixels, zero outside
// the image) in LDS
// with coalesced 16-byte loads; the layer's packed weights are staged once.
// A wavefront computes its 64 pixels (4 M blocks of 16) x all output
// channels (NB blocks of 16): per reduction chunk it reads 4 A fragments and
// NB B fragments from LDS and issues 4 NB MFMAs, so every fragment read
// feeds several MFMAs.  CS, the stored input channels, is 8 (KC = 3) for the
// input layer and 48 (KC = 14) otherwise.
// mode 0: bias + ReLU -> BF16 NHWC (out_c channels stored)
// mode 1: bias, no activation -> FP32 planar [img][cout][ny][nx]
// mode 2: input gradient: no bias, times (mask > 0) -> BF16 NHWC (mask: the
//         BF16 activation the gradient flows into, mask_c channels per pixel)
// ---------------------------------------------------------------------------
constexpr int TW = 64;     // output pixels per tile row
constexpr int CW = 8;      // wavefronts (output rows per step) of a convolution workgroup
constexpr int CT = 64 * CW;

// LDS of one convolution workgroup: packed weights, the staged input rows
// and the waves' output tiles
template <int NB, int KC>
constexpr int conv_lds_bytes()
{
    constexpr int PXU = (KC == 3 ? CIN0 : MAXW) * 2 / 16;
    constexpr int SU = (CW + 2) * (TW + 2) * PXU, OU = TW * NB * 2;
    return 16 * (NB * KC * 64 + SU + CW * OU);
}

template <int NB, int KC>
__global__ void __launch_bounds__(CT) k_conv(const unsigned short *__restrict__ in, Geo g,
                                             const unsigned short *__restrict__ wpk,
                                             const float *__restrict__ bias, int mode,
                                             const unsigned short *__restrict__ mask, int mask_c,
                                             void *__restrict__ out, int out_c, int nx, int ny,
                                             int cseg)
{
    constexpr int CS = KC == 3 ? CIN0 : MAXW;
    constexpr int PXU = CS * 2 / 16;            // uint4 per staged pixel
    constexpr int ROWU = (TW + 2) * PXU;        // uint4 per staged row
    constexpr int SROWS = CW + 2;               // staged rows per step
    constexpr int SU = SROWS * ROWU;            // staged uint4 per step
    constexpr int PER = (SU + CT - 1) / CT;     // staged uint4 per thread
    constexpr int OU = TW * NB * 2;             // uint4 of one wave's BF16 output tile
    __shared__ uint4 sw[NB * KC * 64];
    __shared__ uint4 sx[SU];       // staged input rows
    __shared__ uint4 st[CW * OU];  // the waves' output tiles (one region per wave)
    const uint4 *w4 = reinterpret_cast<const uint4 *>(wpk);
    for (int q = threadIdx.x; q < NB * KC * 64; q += CT) sw[q] = w4[q];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int x0 = blockIdx.x * TW, img = blockIdx.z;
    const int ys = blockIdx.y * cseg, ye = min(ny, ys + cseg);
    const unsigned short *base = in + (long)img * ny * nx * CS;
    // the input rows of the next step are loaded into registers while the
    // current step computes
    uint4 pre[PER];
    auto fetch = [&](int y0) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int q = threadIdx.x + j * CT;
            const int r = q / ROWU, rem = q - r * ROWU;
            const int px = rem / PXU, part = rem - px * PXU;
            const int yy = y0 - 1 + r, xx = x0 - 1 + px;
            pre[j] = make_uint4(0u, 0u, 0u, 0u);
            if (q < SU && (unsigned)yy < (unsigned)ny && (unsigned)xx < (unsigned)nx)
                pre[j] = *reinterpret_cast<const uint4 *>(base + ((long)yy * nx + xx) * CS + part * 8);
        }
    };
    // BF16 NHWC outputs of exactly NB * 16 channels leave through LDS as
    // whole 16-byte pixel chunks: a wave writes its tile into its own region
    // of st after its MFMAs and stores it to memory in the next step, before
    // that step's input loads are issued (a wait for the loads then finds the
    // stores, which the same counter tracks, long done)
    const bool tile_out = mode != 1 && out_c == NB * 16 && (mode == 0 || mask_c == out_c);
    auto flush = [&](int y) {
        if (y >= ye) return;
        unsigned short *ob = static_cast<unsigned short *>(out);
        for (int q = lane; q < OU; q += 64) {
            const int px = q / (NB * 2), part = q - px * (NB * 2);
            const int xx = x0 + px;
            if (xx >= nx) continue;
            const long pix = ((long)img * ny + y) * nx + xx;
            uint4 v = st[wv * OU + q];
            if (mode == 2) {  // the gradient flows only where the activation is > 0
                const uint4 mk = *reinterpret_cast<const uint4 *>(mask + pix * mask_c + part * 8);
                unsigned vv[4] = {v.x, v.y, v.z, v.w};
                const unsigned mm[4] = {mk.x, mk.y, mk.z, mk.w};
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const bool lo = bf16_float((unsigned short)(mm[h] & 0xffffu)) > 0.0f;
                    const bool hi = bf16_float((unsigned short)(mm[h] >> 16)) > 0.0f;
                    vv[h] &= (lo ? 0x0000ffffu : 0u) | (hi ? 0xffff0000u : 0u);
                }
                v = make_uint4(vv[0], vv[1], vv[2], vv[3]);
            }
            *reinterpret_cast<uint4 *>(ob + pix * out_c + part * 8) = v;
        }
    };
    int pending = -1;  // row of the tile waiting in st (tile_out), or -1
    fetch(ys);
    for (int y0 = ys; y0 < ye; y0 += CW) {
        __syncthreads();  // the previous step is done with sx
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int q = threadIdx.x + j * CT;
            if (q < SU) sx[q] = pre[j];
        }
        __syncthreads();
        if (pending >= 0) flush(pending);
        if (y0 + CW < ye) fetch(y0 + CW);
        floatx4 acc[4][NB];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int b = 0; b < NB; ++b) acc[mb][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            // the padding rows k >= 9 CS of the packed weights are zero, so a
            // lane past the last tap may read any finite activation: it reads
            // tap 8 (no branch around the fragment reads)
            const int k = 32 * kc + 8 * kg;
            const int tap = min(k / CS, 8), c = k - (k / CS) * CS;
            const int ty = tap / 3, tx = tap - 3 * ty;
            bf16x8 bv[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const uint4 wv4 = sw[(b * KC + kc) * 64 + lane];
                __builtin_memcpy(&bv[b], &wv4, 16);
            }
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const uint4 a = sx[(wv + ty) * ROWU + (mb * 16 + m + tx) * PXU + c / 8];
                bf16x8 av;
                __builtin_memcpy(&av, &a, 16);
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[mb][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv[b], acc[mb][b], 0, 0, 0);
            }
        }
        // lane holds, in M block mb, output pixels x0 + 16 mb + 4 kg + i
        // (i = 0..3) of row y, channel 16 b + m
        const int y = y0 + wv;
        if (tile_out) {
            unsigned short *so = reinterpret_cast<unsigned short *>(st + wv * OU);
#pragma unroll
            for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int n = 16 * b + m;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        float v = acc[mb][b][i];
                        if (mode == 0) v = n < g.cout ? fmaxf(v + bias[min(n, g.cout - 1)], 0.0f) : 0.0f;
                        so[(16 * mb + 4 * kg + i) * (NB * 16) + n] = bf16_bits(v);
                    }
                }
            pending = y;
            continue;
        }
        if (y >= ye) continue;
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int n = 16 * b + m;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int xx = x0 + 16 * mb + 4 * kg + i;
                    if (xx >= nx || n >= g.cout) continue;
                    const long pix = ((long)img * ny + y) * nx + xx;
                    float v = acc[mb][b][i];
                    if (mode == 0) {
                        v = fmaxf(v + bias[n], 0.0f);
                        static_cast<unsigned short *>(out)[pix * out_c + n] = bf16_bits(v);
                    } else if (mode == 1) {
                        v += bias[n];
                        static_cast<float *>(out)[(((long)img * g.cout + n) * ny + y) * nx + xx] = v;
                    } else {
                        if (!(bf16_float(mask[pix * mask_c + n]) > 0.0f)) v = 0.0f;
                        static_cast<unsigned short *>(out)[pix * out_c + n] = bf16_bits(v);
                    }
                }
            }
    }
    if (pending >= 0) flush(pending);
}

// Planar FP32 [img][cin][ny][nx] -> BF16 NHWC with cs stored channels.
__global__ void k_to_nhwc(const float *__restrict__ x, int cin, int cs, long npix_img, int nimg,
                          unsigned short *__restrict__ out)
{
    const long total = npix_img * nimg;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < total;
         p += (long)gridDim.x * blockDim.x) {
        const long img = p / npix_img, q = p % npix_img;
        for (int c = 0; c < cs; ++c)
            out[p * cs + c] = c < cin ? bf16_bits(x[(img * cin + c) * npix_img + q]) : 0;
    }
}

// Loss and its gradient: d = y - t; loss partial sums of d^2 (FP64); the
// gradient 2 d / N stored BF16 NHWC (cs channels) for the backward pass.
__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ t, int cout, int cs,
                      long npix_img, int nimg, double inv_n, unsigned short *__restrict__ g,
                      double *__restrict__ part)
{
    __shared__ double red[NWAVE];
    double s = 0.0;
    const long total = npix_img * nimg;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < total;
         p += (long)gridDim.x * blockDim.x) {
        const long img = p / npix_img, q = p - img * npix_img;
        // the pixel's cs BF16 values (cout gradients, zeros after them) leave
        // as 16-byte chunks (cs is a stored width: a multiple of 8)
        uint4 *gp = reinterpret_cast<uint4 *>(g + p * cs);
        for (int c8 = 0; c8 < cs; c8 += 8) {
            unsigned short v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int c = c8 + k;
                float gv = 0.0f;
                if (c < cout) {
                    const long i = (img * cout + c) * npix_img + q;
                    const float d = y[i] - t[i];
                    s += (double)d * (double)d;
                    gv = (float)(2.0 * inv_n * (double)d);
                }
                v[k] = bf16_bits(gv);
            }
            uint4 u;
            __builtin_memcpy(&u, v, 16);
            gp[c8 / 8] = u;
        }
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NWAVE; ++w) s += red[w];
        part[blockIdx.x] = s;
    }
}

// Weight and bias gradients of one layer on the matrix cores:
//   dW[n][c][ky][kx] = sum over pixels p of dz[p][n] x[p + (ky-1, kx-1)][c],
//   db[n] = sum over p of dz[p][n],
// a GEMM D[n][j] = sum_p A[n][p] B[p][j] with j = 9 c + 3 ky + kx (so D is
// W's gradient in parameter order), M = cout, N = 9 cin, and the pixels as
// the reduction (BF16 products, FP32 accumulation, split over workgroups).
//
// Work item: R consecutive rows of one 64-pixel column strip of one image.
// Its steps s = 0, 1 stage the input rows ya - 1 and ya; step s >= 2 stages
// input row y + 1 and the dz row y = ya + s - 2, then adds the products of
// row y.  The input rows sit in a ring of three LDS slots (image row gy in
// slot (gy + 1) mod 3), so every input row is loaded and staged once per
// item.  Both operands are staged transposed, pixels contiguous, so an A or
// B fragment (8 consecutive pixels of one row n or column j) is one aligned
// 16-byte LDS read:
//   sdz[n][i]                 = dz at (y, x0 + i),
//   sx[9 c + 3 slot + kx][i]  = x at (gy, x0 + i + kx - 1)
// (consecutive columns j read rows 4 banks apart: no bank conflicts).  The
// bias gradient is one more GEMM column, j = 9 cin, whose B rows are ones
// (three LDS rows of ones, one per slot, staged once).  A staging task is
// 8 pixels x 4 channels: 8-byte channels-last buffer loads from a resource
// spanning one image row (10 pixels for the input, whose three horizontal
// shifts need the neighbours; a pixel outside the image takes an offset
// beyond the resource, which the hardware answers with zeros), a transpose
// of BF16 pairs in registers and 16-byte LDS stores.  Two loader
// groups of threads (tid < 256, tid >= 256) take the steps alternately, each
// loading the step after next while the products run, so two steps of loads
// are in flight.  Wavefront w owns the column blocks w, w + DWW, ... and all
// row blocks; it holds the step's A fragments in registers and reads the
// two B fragments of a column block before its MFMAs (each B fragment feeds
// NBM MFMAs).  Each workgroup writes its partials (one slice per workgroup,
// summed in a fixed order by k_dw_sum).
constexpr int DWX = 64;                                  // pixels per strip
constexpr int DWP = DWX + 8;                             // padded LDS row (bf16): 144 bytes
constexpr int DWW = 8;                                   // wavefronts of a workgroup
constexpr int DWT = 64 * DWW;
constexpr int DWJ = ((9 * MAXW + 16) / 16 + DWW - 1) / DWW;  // column blocks per wavefront (+ bias)
constexpr int DW_ONES = 9 * MAXW;                        // first of the three rows of ones
constexpr unsigned DW_OOB = 0x80000000u;                 // an offset beyond every resource
// fourth word of a raw buffer resource: data format 32 bits (4 in bits 15..18),
// stride 0, so an offset at or past the resource's byte count reads zero
constexpr int DW_RSRC_W3 = 4 << 15;
constexpr int DW_ZT = 96;                                // first dz task within a loader group
static_assert(DWT == 2 * 256, "two loader groups of 256 threads");
static_assert(8 * (MAXW / 4) <= DW_ZT && DW_ZT + 8 * (MAXW / 4) <= 256,
              "a group holds the input tasks of 48 channels, then the dz tasks of 48 channels");

// BF16 pairs (low half of a with low half of b), (high half of a with high
// of b): one byte permute each (selector bytes 0-3 pick bytes of a, 4-7 bytes of b)
__device__ __forceinline__ unsigned pair_lo(unsigned a, unsigned b) { return __builtin_amdgcn_perm(b, a, 0x05040100u); }
__device__ __forceinline__ unsigned pair_hi(unsigned a, unsigned b) { return __builtin_amdgcn_perm(b, a, 0x07060302u); }
// channel e (0..3) of a 4-channel chunk, pixels a (low half) and b (high half)
__device__ __forceinline__ unsigned pair_ch(const uint2 &a, const uint2 &b, int e)
{
    const unsigned wa = e < 2 ? a.x : a.y, wb = e < 2 ? b.x : b.y;
    return (e & 1) ? pair_hi(wa, wb) : pair_lo(wa, wb);
}

// One step of a work item (uniform across the workgroup).
struct DwStep {
    long it;                  // item index
    int s, nrow;              // step, rows of the item
    int img, x0, ya;          // image, first pixel of the strip, first row
};

template <int NBM>  // row blocks: ceil(cout / 16)
__global__ void __launch_bounds__(DWT) __attribute__((amdgpu_waves_per_eu(4))) k_dw(
    const unsigned short *__restrict__ x, int cs, int cin, const unsigned short *__restrict__ dz, int dcs,
    int cout, int nimg, int nx, int ny, float *__restrict__ part)
{
    __shared__ __attribute__((aligned(16))) unsigned short sdz[MAXW][DWP];
    __shared__ __attribute__((aligned(16))) unsigned short sx[9 * MAXW + 9][DWP];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 15, kg = lane >> 4;
    const int jcols = 9 * cin, nbj = (jcols + 16) / 16;  // + the bias column
    const int ncx = (cin + 3) / 4, ncz = (cout + 3) / 4;  // 4-channel groups
    // loader role: group grp stages the steps of its parity; within it,
    // l < 8 ncx is the input task (g, cg), DW_ZT <= l < DW_ZT + 8 ncz the
    // dz task (g, cg); g = group of 8 pixels, cg = group of 4 channels
    const int grp = tid >> 8, l = tid & 255;
    const bool tx = l < 8 * ncx, tz = l >= DW_ZT && l < DW_ZT + 8 * ncz;
    const int tl = tz ? l - DW_ZT : l;
    const int tg = tl & 7, tcg = tl >> 3;
    // this lane's GEMM columns: sx row 9 c + kx + 3 slot(ky), kept as
    // 4 (9 c + kx) + ky; the bias column reads the rows of ones
    int col[DWJ];
#pragma unroll
    for (int t = 0; t < DWJ; ++t) {
        const int j = 16 * (wv + DWW * t) + m;
        const int jj = min(j, jcols - 1);
        const int c = jj / 9, tap = jj - 9 * c, ky = tap / 3, kx = tap - 3 * ky;
        col[t] = j == jcols ? 4 * DW_ONES : 4 * (9 * c + kx) + ky;
    }
    // rows of sdz and sx that are read but never staged hold zeros (their
    // products land only in D entries that are not written)
    for (int q = tid; q < MAXW * DWP / 8; q += DWT) reinterpret_cast<uint4 *>(&sdz[0][0])[q] = make_uint4(0u, 0u, 0u, 0u);
    for (int q = tid; q < (9 * MAXW + 9) * DWP / 8; q += DWT) {
        const unsigned one = q >= DW_ONES * DWP / 8 ? 0x3f803f80u : 0u;  // BF16 1.0 pairs
        reinterpret_cast<uint4 *>(&sx[0][0])[q] = make_uint4(one, one, one, one);
    }
    floatx4 acc[DWJ][NBM];
#pragma unroll
    for (int t = 0; t < DWJ; ++t)
#pragma unroll
        for (int b = 0; b < NBM; ++b) acc[t][b] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};

    // work items: R rows of a strip, about one item per workgroup
    const int xblocks = (nx + DWX - 1) / DWX;
    const long strips = (long)nimg * xblocks;
    const long G = gridDim.x;
    const int R = (int)max(1L, (strips * ny + G - 1) / G);
    const int cps = (ny + R - 1) / R;
    const long items = strips * cps;
    auto first = [&](long it, DwStep &st) -> bool {
        if (it >= items) return false;
        const int q = (int)(it % cps);
        const long sp = it / cps;
        st.it = it;
        st.s = 0;
        st.ya = q * R;
        st.nrow = min(R, ny - st.ya);
        st.x0 = (int)(sp % xblocks) * DWX;
        st.img = (int)(sp / xblocks);
        return true;
    };
    auto next = [&](DwStep &st) -> bool {
        if (++st.s < st.nrow + 2) return true;
        return first(st.it + G, st);
    };

    // the loads of one step, into registers
    uint2 v[10];
    auto fetch = [&](const DwStep &st) {
        if (tx) {  // pixels x0 + 8 g - 1 .. x0 + 8 g + 8 of input row ya + s - 1 (zeros outside)
            const int gy = st.ya + st.s - 1;
            const bool rowok = (unsigned)gy < (unsigned)ny;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(x + ((long)st.img * ny + (rowok ? gy : 0)) * nx * cs), (short)0,
                rowok ? nx * cs * 2 : 0, DW_RSRC_W3);
            const int p0 = st.x0 + 8 * tg - 1;
#pragma unroll
            for (int e = 0; e < 10; ++e) {
                const int px = p0 + e;
                const unsigned off = (unsigned)px < (unsigned)nx ? (unsigned)(px * cs + 4 * tcg) * 2u : DW_OOB;
                const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
                v[e] = make_uint2(w[0], w[1]);
            }
        } else if (tz && st.s >= 2) {  // pixels x0 + 8 g .. x0 + 8 g + 7 of dz row ya + s - 2
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(dz + ((long)st.img * ny + st.ya + st.s - 2) * nx * dcs), (short)0, nx * dcs * 2,
                DW_RSRC_W3);
            const int p0 = st.x0 + 8 * tg;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int px = p0 + e;
                const unsigned off = px < nx ? (unsigned)(px * dcs + 4 * tcg) * 2u : DW_OOB;
                const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
                v[e] = make_uint2(w[0], w[1]);
            }
        }
    };

    DwStep cur, ahead;  // the step being computed; the last step whose loads were issued
    bool has = first(blockIdx.x, cur);
    ahead = cur;
    bool hasa = has && next(ahead);
    if (grp == 0 && has) fetch(cur);
    if (grp == 1 && hasa) fetch(ahead);
    for (int k = 0; has; ++k) {
        const bool mine = grp == (k & 1);
        __syncthreads();  // the previous step is done with the slots it read
        if (mine) {
            if (tx) {
                // sx[9 c + 3 slot + kx][8 g + i] = pixel x0 + 8 g + i + kx - 1 = v[i + kx]
                const int slot = (cur.ya + cur.s) % 3;  // (gy + 1) mod 3
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = 4 * tcg + e;
                    uint4 *row = reinterpret_cast<uint4 *>(&sx[9 * c + 3 * slot][8 * tg]);
                    const unsigned p0 = pair_ch(v[0], v[1], e), p2 = pair_ch(v[2], v[3], e),
                                   p4 = pair_ch(v[4], v[5], e), p6 = pair_ch(v[6], v[7], e),
                                   p8 = pair_ch(v[8], v[9], e);
                    row[0] = make_uint4(p0, p2, p4, p6);  // kx = 0
                    row[DWP / 8] = make_uint4(pair_ch(v[1], v[2], e), pair_ch(v[3], v[4], e),
                                              pair_ch(v[5], v[6], e), pair_ch(v[7], v[8], e));
                    row[2 * DWP / 8] = make_uint4(p2, p4, p6, p8);  // kx = 2
                }
            } else if (tz && cur.s >= 2) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    *reinterpret_cast<uint4 *>(&sdz[4 * tcg + e][8 * tg]) =
                        make_uint4(pair_ch(v[0], v[1], e), pair_ch(v[2], v[3], e),
                                   pair_ch(v[4], v[5], e), pair_ch(v[6], v[7], e));
            }
        }
        __syncthreads();
        {  // this group loads the step after next
            DwStep n2 = ahead;
            const bool h2 = hasa && next(n2);
            if (mine && h2) fetch(n2);
            ahead = n2;
            hasa = h2;
        }
        if (cur.s >= 2) {  // products of row y = ya + s - 2 (input rows y - 1 .. y + 1)
            const int ym = (cur.ya + cur.s - 2) % 3;  // tap ky reads slot (y + ky) mod 3
            // byte offsets of this lane's fragments; the A fragments of both
            // 32-pixel chunks stay in registers, each column block reads its
            // two B fragments before its MFMAs
            const char *sxb = reinterpret_cast<const char *>(&sx[0][0]);
            const char *szb = reinterpret_cast<const char *>(&sdz[0][0]);
            const unsigned aoff = (unsigned)m * (2u * DWP) + 16u * kg;
            bf16x8 a[NBM][2];
#pragma unroll
            for (int b = 0; b < NBM; ++b)
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const uint4 w = *reinterpret_cast<const uint4 *>(szb + aoff + b * 16 * (2 * DWP) + 64 * ks);
                    __builtin_memcpy(&a[b][ks], &w, 16);
                }
#pragma unroll
            for (int t = 0; t < DWJ; ++t) {
                if (wv + DWW * t >= nbj) break;
                int slot = ym + (col[t] & 3);
                slot = slot >= 3 ? slot - 3 : slot;
                const unsigned boff = (unsigned)((col[t] >> 2) + 3 * slot) * (2u * DWP) + 16u * kg;
                const uint4 w0 = *reinterpret_cast<const uint4 *>(sxb + boff);
                const uint4 w1 = *reinterpret_cast<const uint4 *>(sxb + boff + 64);
                bf16x8 b0, b1;
                __builtin_memcpy(&b0, &w0, 16);
                __builtin_memcpy(&b1, &w1, 16);
#pragma unroll
                for (int b = 0; b < NBM; ++b)
                    acc[t][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[b][0], b0, acc[t][b], 0, 0, 0);
#pragma unroll
                for (int b = 0; b < NBM; ++b)
                    acc[t][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[b][1], b1, acc[t][b], 0, 0, 0);
            }
        }
        has = next(cur);
    }
    // lane holds D[16 b + 4 kg + i][16 jb + m], i = 0..3; column jcols is the bias
    float *mine = part + (long)blockIdx.x * (cout * jcols + cout);
#pragma unroll
    for (int t = 0; t < DWJ; ++t) {
        const int jb = wv + DWW * t;
        if (jb >= nbj) break;
        const int j = 16 * jb + m;
#pragma unroll
        for (int b = 0; b < NBM; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int n = 16 * b + 4 * kg + i;
                if (n < cout && j < jcols) mine[n * jcols + j] = acc[t][b][i];
                if (n < cout && j == jcols) mine[cout * jcols + n] = acc[t][b][i];
            }
    }
}

// Sum of the per-workgroup partial gradients (fixed order) into grad.
// The weight gradient as the sum of the workgroups' partial slices, in a
// fixed order (the same bits every run): a 256-thread workgroup takes 64
// consecutive entries; its four wavefronts sum the partials p = q, q + 4,
// q + 8, ... (q the wavefront) with coalesced loads, and the four sums are
// added in wavefront order.
constexpr int DWS_COLS = 64;
__global__ void __launch_bounds__(256) k_dw_sum(const float *__restrict__ part, int nparts, int len,
                                                float *__restrict__ grad)
{
    __shared__ float red[4][DWS_COLS];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int i = blockIdx.x * DWS_COLS + lane;
    float s = 0.0f;
    if (i < len) {
#pragma unroll 8
        for (int p = q; p < nparts; p += 4) s += part[(long)p * len + i];
    }
    red[q][lane] = s;
    __syncthreads();
    if (q == 0 && i < len) grad[i] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Adam with bias correction (Kingma & Ba 2015), FP32.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, long n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Surrogate inputs from a solver state: x = scale * (h, hu, hv, b, h > 0).
__global__ void k_inputs(const float *__restrict__ f, long n, float s0, float s1, float s2,
                         float s3, float s4, unsigned short *__restrict__ out)
{
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n;
         p += (long)gridDim.x * blockDim.x) {
        const float h = f[p], qx = f[n + p], qy = f[2 * n + p], b = f[3 * n + p];
        out[p * CIN0 + 0] = bf16_bits(s0 * h);
        out[p * CIN0 + 1] = bf16_bits(s1 * qx);
        out[p * CIN0 + 2] = bf16_bits(s2 * qy);
        out[p * CIN0 + 3] = bf16_bits(s3 * b);
        out[p * CIN0 + 4] = bf16_bits(h > 0.0f ? s4 : 0.0f);
        for (int c = 5; c < CIN0; ++c) out[p * CIN0 + c] = 0;
    }
}

// New state = old + out_scale * prediction (depth clamped at 0, momentum 0 on
// dry cells); FP64 partial sums of the old and new depth and bed.
__global__ void k_apply(const float *__restrict__ f, const float *__restrict__ o, long n, float s0,
                        float s1, float s2, float s3, float *__restrict__ nf,
                        double *__restrict__ part)
{
    __shared__ double r[4][NWAVE];
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n;
         p += (long)gridDim.x * blockDim.x) {
        const float h = f[p];
        float hn = h + s0 * o[p];
        if (!(hn > 0.0f)) hn = 0.0f;
        const float qx = hn > 0.0f ? f[n + p] + s1 * o[n + p] : 0.0f;
        const float qy = hn > 0.0f ? f[2 * n + p] + s2 * o[2 * n + p] : 0.0f;
        const float bn = f[3 * n + p] + s3 * o[3 * n + p];
        nf[p] = hn;
        nf[n + p] = qx;
        nf[2 * n + p] = qy;
        nf[3 * n + p] = bn;
        a += (double)h;
        b += (double)hn;
        c += (double)f[3 * n + p];
        d += (double)bn;
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off);
        b += __shfl_down(b, off);
        c += __shfl_down(c, off);
        d += __shfl_down(d, off);
    }
    if ((threadIdx.x & 63) == 0) {
        r[0][threadIdx.x >> 6] = a; r[1][threadIdx.x >> 6] = b;
        r[2][threadIdx.x >> 6] = c; r[3][threadIdx.x >> 6] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NWAVE; ++w) { a += r[0][w]; b += r[1][w]; c += r[2][w]; d += r[3][w]; }
        part[4 * blockIdx.x] = a;
        part[4 * blockIdx.x + 1] = b;
        part[4 * blockIdx.x + 2] = c;
        part[4 * blockIdx.x + 3] = d;
    }
}

// Largest |u[p] - v[p]| over n values (per workgroup; exact in FP32).
__global__ void k_maxdiff(const float *__restrict__ u, const float *__restrict__ v, long n,
                          float *__restrict__ part)
{
    __shared__ float r[NWAVE];
    float m = 0.0f;
    for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < n;
         p += (long)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(u[p] - v[p]));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_down(m, off));
    if ((threadIdx.x & 63) == 0) r[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NWAVE; ++w) m = fmaxf(m, r[w]);
        part[blockIdx.x] = m;
    }
}

// Gather of images idx[0..nb) of a planar set [npairs][c][npix] into [nb][c][npix].
__global__ void k_gather(const float *__restrict__ src, const int *__restrict__ idx, int nb, int c,
                         long npix, float *__restrict__ dst)
{
    const long per = (long)c * npix, total = per * nb;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < total;
         q += (long)gridDim.x * blockDim.x) {
        const long i = q / per, r = q - i * per;
        dst[q] = src[(long)idx[i] * per + r];
    }
}

}  // namespace

// ===========================================================================
// Host side
// ===========================================================================

struct sws_net {
    hipStream_t stream = nullptr;
    int L = 0;
    std::vector<int> ch;            // widths, L + 1
    std::vector<Geo> fwd, bwd;      // per layer (bwd: transposed convolution)
    std::vector<long> woff, boff;   // offsets of W_l, b_l in the parameter vector
    long nparam = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // params, grads, Adam moments
    std::vector<unsigned short *> wpk, wpk_t;                      // packed forward / transposed weights
    long adam_t = 0;
    float in_scale[5] = {1, 1, 1, 1, 1}, out_scale[4] = {1, 1, 1, 1};
    bool packed = false;
    // scratch (grown on demand)
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    // pinned host staging (hipHostMalloc, grown on demand): every transfer
    // between user host memory and the device goes through it
    void *hstage = nullptr;
    size_t hstage_bytes = 0;
    std::string err;
};

namespace {

int sfail(sws_net *n, int code, const std::string &msg)
{
    if (n) n->err = msg;
    return code;
}

#define SHIP(n, call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return sfail((n), SW_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int stored(int c) { return c <= CIN0 ? CIN0 : MAXW; }

Geo make_geo(int cin, int cout)
{
    Geo g;
    g.cs = stored(cin);
    g.cin = cin;
    g.cout = cout;
    g.nb = (cout + 15) / 16;
    g.kc = (9 * g.cs + 31) / 32;
    return g;
}

size_t packed_len(const Geo &g) { return (size_t)g.nb * g.kc * 64 * 8; }

int grid_for(long n) { return (int)std::min<long>(4096, std::max<long>(1, (n + NT - 1) / NT)); }

constexpr int kConvCUs = 256;           // compute units of the MI355X
constexpr int kLdsPerCU = 160 * 1024;   // LDS bytes per compute unit

// One workgroup per (64-pixel strip, row segment, image).  The segments are
// as tall as leaves every workgroup the chip holds at once one of them (a
// multiple of CW rows): each workgroup loads its weights and first input rows
// once, so fewer, taller segments spend less time on that.
template <int NB, int KC>
void conv_t(hipStream_t s, const unsigned short *in, Geo g, const unsigned short *w,
            const float *bias, int mode, const unsigned short *mask, int mask_c, void *out,
            int out_c, int nimg, int nx, int ny)
{
    const long cols = (long)((nx + TW - 1) / TW) * nimg;
    const long steps = (ny + CW - 1) / CW;
    const long slots = (long)kConvCUs * std::max(1, kLdsPerCU / conv_lds_bytes<NB, KC>());
    const int cseg = CW * (int)std::max<long>(1, (cols * steps + slots - 1) / slots);
    const dim3 grid((nx + TW - 1) / TW, (ny + cseg - 1) / cseg, nimg);
    hipLaunchKernelGGL((k_conv<NB, KC>), grid, dim3(CT), 0, s, in, g, w, bias, mode, mask,
                       mask_c, out, out_c, nx, ny, cseg);
}

// Dispatch on (output blocks, reduction chunks): KC = 3 for the 8-channel
// input, 14 for 48 stored channels.
int conv(sws_net *n, const unsigned short *in, const Geo &g, const unsigned short *w,
         const float *bias, int mode, const unsigned short *mask, int mask_c, void *out, int out_c,
         int nimg, int nx, int ny)
{
    if (g.cs != (g.kc == 3 ? CIN0 : MAXW)) return sfail(n, SW_ERR_ARG, "unsupported layer shape");
    hipStream_t s = n->stream;
    if (g.kc == 3 && g.nb == 3) conv_t<3, 3>(s, in, g, w, bias, mode, mask, mask_c, out, out_c, nimg, nx, ny);
    else if (g.kc == 3 && g.nb == 1) conv_t<1, 3>(s, in, g, w, bias, mode, mask, mask_c, out, out_c, nimg, nx, ny);
    else if (g.kc == 3 && g.nb == 2) conv_t<2, 3>(s, in, g, w, bias, mode, mask, mask_c, out, out_c, nimg, nx, ny);
    else if (g.kc == 14 && g.nb == 3) conv_t<3, 14>(s, in, g, w, bias, mode, mask, mask_c, out, out_c, nimg, nx, ny);
    else if (g.kc == 14 && g.nb == 2) conv_t<2, 14>(s, in, g, w, bias, mode, mask, mask_c, out, out_c, nimg, nx, ny);
    else if (g.kc == 14 && g.nb == 1) conv_t<1, 14>(s, in, g, w, bias, mode, mask, mask_c, out, out_c, nimg, nx, ny);
    else return sfail(n, SW_ERR_ARG, "unsupported layer shape");
    SHIP(n, hipGetLastError());
    return SW_OK;
}

int pack_all(sws_net *n)
{
    std::vector<PackJob> jobs;
    for (int l = 0; l < n->L; ++l) {
        jobs.push_back(PackJob{n->p + n->woff[l], n->wpk[l], n->fwd[l], 0, n->ch[l]});
        if (l > 0)  // the input gradient of layer 0 is never needed
            jobs.push_back(PackJob{n->p + n->woff[l], n->wpk_t[l], n->bwd[l], 1, n->ch[l]});
    }
    for (size_t j0 = 0; j0 < jobs.size(); j0 += kPackJobs) {
        PackTable t{};
        const int nj = (int)std::min<size_t>(kPackJobs, jobs.size() - j0);
        long most = 1;
        for (int j = 0; j < nj; ++j) {
            t.j[j] = jobs[j0 + j];
            most = std::max<long>(most, (long)packed_len(jobs[j0 + j].g));
        }
        hipLaunchKernelGGL(k_pack, dim3(grid_for(most), nj), dim3(NT), 0, n->stream, t);
    }
    SHIP(n, hipGetLastError());
    n->packed = true;
    return SW_OK;
}

int ensure_scratch(sws_net *n, size_t bytes)
{
    if (bytes <= n->scratch_bytes) return SW_OK;
    SHIP(n, hipStreamSynchronize(n->stream));
    (void)hipFree(n->scratch);
    n->scratch = nullptr;
    n->scratch_bytes = 0;
    SHIP(n, hipMalloc(&n->scratch, bytes));
    // channels a layer narrower than its stored width never writes must read as 0
    SHIP(n, hipMemsetAsync(n->scratch, 0, bytes, n->stream));
    n->scratch_bytes = bytes;
    return SW_OK;
}

// Scratch layout for nimg images of npix pixels: activations of every layer
// (BF16 NHWC, kept for the backward pass), the FP32 output, two gradient
// buffers, weight-gradient partials and reduction partials.
struct Scratch {
    std::vector<unsigned short *> act;  // act[l]: input of layer l (stored channels)
    float *out;
    unsigned short *ga, *gb;
    float *dwpart;
    double *red;
    size_t bytes;
};
constexpr int DW_GRID = 512;
constexpr int RED_GRID = 1024;

Scratch layout(const sws_net *n, long npix, char *base)
{
    Scratch s;
    size_t off = 0;
    auto take = [&](size_t b) {
        char *p = base ? base + off : nullptr;
        off += (b + 255) / 256 * 256;
        return p;
    };
    for (int l = 0; l < n->L; ++l)
        s.act.push_back((unsigned short *)take((size_t)npix * stored(n->ch[l]) * 2));
    s.out = (float *)take((size_t)npix * 4 * sizeof(float));
    s.ga = (unsigned short *)take((size_t)npix * MAXW * 2);
    s.gb = (unsigned short *)take((size_t)npix * MAXW * 2);
    s.dwpart = (float *)take((size_t)DW_GRID * (MAXW * MAXW * 9 + MAXW) * sizeof(float));
    s.red = (double *)take((size_t)4 * RED_GRID * sizeof(double));
    s.bytes = off;
    return s;
}

int forward_into(sws_net *n, const Scratch &s, int nimg, int nx, int ny)
{
    for (int l = 0; l < n->L; ++l) {
        const bool last = l == n->L - 1;
        int rc = conv(n, s.act[l], n->fwd[l], n->wpk[l], n->p + n->boff[l], last ? 1 : 0, nullptr,
                      0, last ? (void *)s.out : (void *)s.act[l + 1],
                      last ? 0 : stored(n->ch[l + 1]), nimg, nx, ny);
        if (rc) return rc;
    }
    return SW_OK;
}

int ensure_hstage(sws_net *n, size_t bytes)
{
    if (n->hstage_bytes >= bytes) return SW_OK;
    if (n->hstage) (void)hipHostFree(n->hstage);
    n->hstage = nullptr;
    n->hstage_bytes = 0;
    SHIP(n, hipHostMalloc(&n->hstage, bytes, hipHostMallocDefault));
    n->hstage_bytes = bytes;
    return SW_OK;
}

// User memory (host or device) -> device, stream-ordered; a host source goes
// through the pinned staging and is done when this returns.
int copy_in(sws_net *n, void *dst, const void *src, size_t bytes, int ptr_kind)
{
    if (ptr_kind != SW_PTR_HOST && ptr_kind != SW_PTR_DEVICE)
        return sfail(n, SW_ERR_ARG, "ptr_kind must be SW_PTR_HOST or SW_PTR_DEVICE");
    if (ptr_kind == SW_PTR_DEVICE) {
        SHIP(n, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, n->stream));
        return SW_OK;
    }
    int rc = ensure_hstage(n, bytes);
    if (rc) return rc;
    std::memcpy(n->hstage, src, bytes);
    SHIP(n, hipMemcpyAsync(dst, n->hstage, bytes, hipMemcpyHostToDevice, n->stream));
    SHIP(n, hipStreamSynchronize(n->stream));
    return SW_OK;
}

// Device -> user memory (host or device), after the work on the stream; synchronises.
int copy_out(sws_net *n, void *dst, const void *src, size_t bytes, int ptr_kind)
{
    if (ptr_kind != SW_PTR_HOST && ptr_kind != SW_PTR_DEVICE)
        return sfail(n, SW_ERR_ARG, "ptr_kind must be SW_PTR_HOST or SW_PTR_DEVICE");
    if (ptr_kind == SW_PTR_DEVICE) {
        SHIP(n, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, n->stream));
        SHIP(n, hipStreamSynchronize(n->stream));
        return SW_OK;
    }
    int rc = ensure_hstage(n, bytes);
    if (rc) return rc;
    SHIP(n, hipMemcpyAsync(n->hstage, src, bytes, hipMemcpyDeviceToHost, n->stream));
    SHIP(n, hipStreamSynchronize(n->stream));
    std::memcpy(dst, n->hstage, bytes);
    return SW_OK;
}

}  // namespace

extern "C" {

int sws_create(const int32_t *channels, int32_t nlayers, void *hip_stream, sws_net **out)
{
    if (!channels || !out || nlayers < 2) return SW_ERR_ARG;
    *out = nullptr;
    if (channels[0] != 5 || channels[nlayers] != 4) return SW_ERR_ARG;
    for (int l = 0; l <= nlayers; ++l)
        if (channels[l] < 1 || channels[l] > MAXW) return SW_ERR_ARG;
    sws_net *n = new sws_net();
    n->stream = (hipStream_t)hip_stream;
    n->L = nlayers;
    n->ch.assign(channels, channels + nlayers + 1);
    long off = 0;
    for (int l = 0; l < nlayers; ++l) {
        n->fwd.push_back(make_geo(n->ch[l], n->ch[l + 1]));
        // the transposed convolution reads gradient buffers of MAXW channels per
        // pixel, except the loss gradient of the last layer's outputs, which
        // keeps their stored width (8 channels: 3 reduction chunks, not 14)
        Geo t = make_geo(n->ch[l + 1], n->ch[l]);
        if (l + 1 < nlayers) {
            t.cs = MAXW;
            t.kc = (9 * MAXW + 31) / 32;
        }
        n->bwd.push_back(t);
        n->woff.push_back(off);
        off += (long)n->ch[l + 1] * n->ch[l] * 9;
        n->boff.push_back(off);
        off += n->ch[l + 1];
    }
    n->nparam = off;
    auto bail = [&](hipError_t e) {
        sws_destroy(n);
        (void)e;
        return SW_ERR_HIP;
    };
    hipError_t e;
    for (float **q : {&n->p, &n->g, &n->m, &n->v}) {
        if ((e = hipMalloc(q, off * sizeof(float))) != hipSuccess) return bail(e);
        if ((e = hipMemsetAsync(*q, 0, off * sizeof(float), n->stream)) != hipSuccess) return bail(e);
    }
    // ordered on the net's stream (possibly non-blocking), done before returning
    if ((e = hipStreamSynchronize(n->stream)) != hipSuccess) return bail(e);
    for (int l = 0; l < nlayers; ++l) {
        unsigned short *a = nullptr, *b = nullptr;
        if ((e = hipMalloc(&a, packed_len(n->fwd[l]) * 2)) != hipSuccess) return bail(e);
        n->wpk.push_back(a);
        if ((e = hipMalloc(&b, packed_len(n->bwd[l]) * 2)) != hipSuccess) return bail(e);
        n->wpk_t.push_back(b);
    }
    *out = n;
    return SW_OK;
}

int sws_destroy(sws_net *n)
{
    if (!n) return SW_OK;
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    else (void)hipDeviceSynchronize();
    for (float *q : {n->p, n->g, n->m, n->v}) (void)hipFree(q);
    for (auto *q : n->wpk) (void)hipFree(q);
    for (auto *q : n->wpk_t) (void)hipFree(q);
    (void)hipFree(n->scratch);
    if (n->hstage) (void)hipHostFree(n->hstage);
    delete n;
    return SW_OK;
}

int sws_param_count(const sws_net *n, int64_t *count)
{
    if (!n || !count) return SW_ERR_ARG;
    *count = n->nparam;
    return SW_OK;
}

int sws_set_params(sws_net *n, const float *params, int ptr_kind)
{
    if (!n || !params) return SW_ERR_ARG;
    int rc = copy_in(n, n->p, params, n->nparam * sizeof(float), ptr_kind);
    if (rc) return rc;
    SHIP(n, hipMemsetAsync(n->m, 0, n->nparam * sizeof(float), n->stream));
    SHIP(n, hipMemsetAsync(n->v, 0, n->nparam * sizeof(float), n->stream));
    n->adam_t = 0;
    return pack_all(n);
}

int sws_get_params(sws_net *n, float *params, int ptr_kind)
{
    if (!n || !params) return SW_ERR_ARG;
    if (ptr_kind != SW_PTR_HOST && ptr_kind != SW_PTR_DEVICE)
        return sfail(n, SW_ERR_ARG, "ptr_kind must be SW_PTR_HOST or SW_PTR_DEVICE");
    return copy_out(n, params, n->p, n->nparam * sizeof(float), ptr_kind);
}

int sws_set_scales(sws_net *n, const float in_scale[5], const float out_scale[4])
{
    if (!n || !in_scale || !out_scale) return SW_ERR_ARG;
    std::memcpy(n->in_scale, in_scale, sizeof n->in_scale);
    std::memcpy(n->out_scale, out_scale, sizeof n->out_scale);
    return SW_OK;
}

int sws_forward(sws_net *n, const float *x, float *y, int32_t nimg, int32_t nx, int32_t ny,
                int ptr_kind)
{
    if (!n || !x || !y || nimg < 1 || nx < 1 || ny < 1) return SW_ERR_ARG;
    if (ptr_kind != SW_PTR_HOST && ptr_kind != SW_PTR_DEVICE)
        return sfail(n, SW_ERR_ARG, "ptr_kind must be SW_PTR_HOST or SW_PTR_DEVICE");
    if (!n->packed) {
        int rc = pack_all(n);
        if (rc) return rc;
    }
    const long npix = (long)nimg * nx * ny;
    const size_t xin = (size_t)npix * 5 * sizeof(float), yout = (size_t)npix * 4 * sizeof(float);
    const size_t need = layout(n, npix, nullptr).bytes + xin;
    int rc = ensure_scratch(n, need);
    if (rc) return rc;
    Scratch s = layout(n, npix, (char *)n->scratch);
    float *xd = (float *)((char *)n->scratch + s.bytes);
    rc = copy_in(n, xd, x, xin, ptr_kind);
    if (rc) return rc;
    hipLaunchKernelGGL(k_to_nhwc, dim3(grid_for(npix)), dim3(NT), 0, n->stream, xd, 5, CIN0,
                       (long)nx * ny, nimg, s.act[0]);
    rc = forward_into(n, s, nimg, nx, ny);
    if (rc) return rc;
    return copy_out(n, y, s.out, yout, ptr_kind);
}

}  // extern "C"

namespace {

// The weight-gradient kernel reads each image row through a buffer resource
// whose size (48 BF16 channels per pixel) is a 31-bit byte count.
bool train_width_ok(sws_net *n, int32_t nx)
{
    if ((long)nx * MAXW * 2 <= 0x7fffffffL) return true;
    sfail(n, SW_ERR_ARG, "nx too large for training (nx * 96 bytes must be below 2^31)");
    return false;
}

// Forward, loss and backward: the gradient lands in n->g; the FP64 loss
// partials in the scratch (returned through *loss when asked, synchronising).
int compute_grads(sws_net *n, const float *x, const float *target, int32_t nimg, int32_t nx,
                  int32_t ny, double *loss, int ptr_kind)
{
    if (!n || !x || !target || nimg < 1 || nx < 1 || ny < 1) return SW_ERR_ARG;
    if (ptr_kind != SW_PTR_HOST && ptr_kind != SW_PTR_DEVICE)
        return sfail(n, SW_ERR_ARG, "ptr_kind must be SW_PTR_HOST or SW_PTR_DEVICE");
    if (!train_width_ok(n, nx)) return SW_ERR_ARG;
    if (!n->packed) {
        int rc = pack_all(n);
        if (rc) return rc;
    }
    const long npix = (long)nimg * nx * ny;
    const size_t xin = (size_t)npix * 5 * sizeof(float), tin = (size_t)npix * 4 * sizeof(float);
    // device inputs are read where they are; host inputs are staged in the scratch
    const bool host = ptr_kind == SW_PTR_HOST;
    const size_t need = layout(n, npix, nullptr).bytes + (host ? xin + tin : 0);
    int rc = ensure_scratch(n, need);
    if (rc) return rc;
    Scratch s = layout(n, npix, (char *)n->scratch);
    const float *xd = x, *td = target;
    if (host) {
        float *xs = (float *)((char *)n->scratch + s.bytes);
        float *ts = (float *)((char *)xs + xin);
        if ((rc = copy_in(n, xs, x, xin, ptr_kind))) return rc;
        if ((rc = copy_in(n, ts, target, tin, ptr_kind))) return rc;
        xd = xs;
        td = ts;
    }
    hipLaunchKernelGGL(k_to_nhwc, dim3(grid_for(npix)), dim3(NT), 0, n->stream, xd, 5, CIN0,
                       (long)nx * ny, nimg, s.act[0]);
    if ((rc = forward_into(n, s, nimg, nx, ny))) return rc;
    // loss and dL/dy (BF16, the stored width of the last layer's outputs)
    const int L = n->L;
    const int cs_out = MAXW;  // the other gradient buffers hold MAXW channels per pixel
    const int cs_last = stored(n->ch[L]);
    hipLaunchKernelGGL(k_mse, dim3(RED_GRID), dim3(NT), 0, n->stream, s.out, td, 4, cs_last,
                       (long)nx * ny, nimg, 1.0 / ((double)npix * 4), s.ga, s.red);
    unsigned short *gcur = s.ga, *gnext = s.gb;
    for (int l = L - 1; l >= 0; --l) {
        // weight and bias gradients of layer l from dz_l (gcur) and its input act[l]
        const int cin = n->ch[l], cout = n->ch[l + 1];
        auto dw = cout > 32 ? k_dw<3> : cout > 16 ? k_dw<2> : k_dw<1>;
        hipLaunchKernelGGL(dw, dim3(DW_GRID), dim3(DWT), 0, n->stream, s.act[l], stored(cin), cin,
                           gcur, l == L - 1 ? cs_last : cs_out, cout, nimg, nx, ny, s.dwpart);
        const int len = cout * cin * 9 + cout;
        hipLaunchKernelGGL(k_dw_sum, dim3((len + DWS_COLS - 1) / DWS_COLS), dim3(256), 0, n->stream,
                           s.dwpart, DW_GRID, len, n->g + n->woff[l]);
        if (l > 0) {  // dz_{l-1} = (W_l^T * dz_l) where act[l] > 0
            rc = conv(n, gcur, n->bwd[l], n->wpk_t[l], nullptr, 2, s.act[l], stored(n->ch[l]),
                      gnext, cs_out, nimg, nx, ny);
            if (rc) return rc;
            std::swap(gcur, gnext);
        }
    }
    if (loss) {
        std::vector<double> h(RED_GRID);
        const int rc_ = copy_out(n, h.data(), s.red, RED_GRID * sizeof(double), SW_PTR_HOST);
        if (rc_) return rc_;
        double sum = 0.0;
        for (double v : h) sum += v;
        *loss = sum / ((double)npix * 4);
    }
    return SW_OK;
}

}  // namespace

extern "C" {

int sws_grad(sws_net *n, const float *x, const float *target, int32_t nimg, int32_t nx,
             int32_t ny, float *grad, double *loss, int ptr_kind)
{
    if (!grad) return sfail(n, SW_ERR_ARG, "grad is NULL");
    int rc = compute_grads(n, x, target, nimg, nx, ny, loss, ptr_kind);
    if (rc) return rc;
    return copy_out(n, grad, n->g, n->nparam * sizeof(float), ptr_kind);
}

int sws_train_step(sws_net *n, const float *x, const float *target, int32_t nimg, int32_t nx,
                   int32_t ny, float lr, double *loss, int ptr_kind)
{
    int rc = compute_grads(n, x, target, nimg, nx, ny, loss, ptr_kind);
    if (rc) return rc;
    // Adam
    n->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)n->adam_t));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)n->adam_t));
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n->nparam)), dim3(NT), 0, n->stream, n->p, n->g, n->m,
                       n->v, n->nparam, lr, b1, b2, 1e-8f, c1, c2);
    SHIP(n, hipGetLastError());
    return pack_all(n);
}

int sws_advance(sws_net *n, sw_ctx *solver, int32_t k, double dt, double max_drift, int32_t *used)
{
    if (!n || !solver || k < 1 || !(dt > 0.0) || !(max_drift >= 0.0)) return SW_ERR_ARG;
    if (used) *used = 0;
    sws_stats st{};
    int rc = sws_advance_K(n, solver, 1, k, dt, max_drift, 0, 0.0, &st);
    if (!rc && used) *used = st.kept;
    return rc;
}

int sws_advance_K(sws_net *n, sw_ctx *solver, int32_t n_calls, int32_t k, double dt,
                  double max_drift, int32_t check_every, double max_err, sws_stats *stats)
{
    if (!n || !solver || n_calls < 0 || k < 1 || !(dt > 0.0) || !(max_drift >= 0.0) ||
        check_every < 0 || !(max_err >= 0.0))
        return SW_ERR_ARG;
    sws_stats st{};
    if (!n->packed) {
        int rc = pack_all(n);
        if (rc) return rc;
    }
    sw_grid gr;
    int rc = sw_get_grid(solver, &gr);
    if (rc) return sfail(n, rc, std::string("solver: ") + sw_last_error(solver));
    const int nx = gr.nx, ny = gr.ny;
    const long npix = (long)nx * ny;
    const size_t fbytes = (size_t)npix * 4 * sizeof(float);
    const size_t need = layout(n, npix, nullptr).bytes + 3 * fbytes;
    if ((rc = ensure_scratch(n, need))) return rc;
    Scratch s = layout(n, npix, (char *)n->scratch);
    float *f0 = (float *)((char *)n->scratch + s.bytes);   // the solver's state
    float *f1 = (float *)((char *)f0 + fbytes);            // the prediction
    float *f2 = (float *)((char *)f1 + fbytes);            // the plain steps (checks)
    const float *is = n->in_scale, *os = n->out_scale;
    for (int32_t call = 0; call < n_calls; ++call) {
        sw_sums sums;
        rc = sw_get_sums(solver, &sums);
        if (!rc) rc = sw_get_fields(solver, f0, f0 + npix, f0 + 2 * npix, f0 + 3 * npix, SW_PTR_DEVICE);
        if (!rc) rc = sw_sync(solver);
        if (rc) return sfail(n, rc, std::string("solver: ") + sw_last_error(solver));
        hipLaunchKernelGGL(k_inputs, dim3(grid_for(npix)), dim3(NT), 0, n->stream, f0, npix, is[0],
                           is[1], is[2], is[3], is[4], s.act[0]);
        if ((rc = forward_into(n, s, 1, nx, ny))) return rc;
        hipLaunchKernelGGL(k_apply, dim3(RED_GRID), dim3(NT), 0, n->stream, f0, s.out, npix, os[0],
                           os[1], os[2], os[3], f1, s.red);
        SHIP(n, hipGetLastError());
        std::vector<double> part(4 * RED_GRID);
        if ((rc = copy_out(n, part.data(), s.red, part.size() * sizeof(double), SW_PTR_HOST))) return rc;
        double v0 = 0.0, v1 = 0.0, b0 = 0.0, b1 = 0.0;
        for (int q = 0; q < RED_GRID; ++q) {  // fixed order
            v0 += part[4 * q];
            v1 += part[4 * q + 1];
            b0 += part[4 * q + 2];
            b1 += part[4 * q + 3];
        }
        // conservation: water volume, and the bed (sediment) volume, of a
        // closed domain without sources must not change
        const double drift = v0 > 0.0 ? std::fabs(v1 - v0) / v0 : (v1 > 0.0 ? INFINITY : 0.0);
        const double bdrift = std::fabs(b1 - b0) / std::max(std::fabs(b0), 1e-30);
        st.calls++;
        st.max_volume_drift = std::max(st.max_volume_drift, std::max(drift, bdrift));
        const double t1 = sums.t + k * dt;
        const int64_t step1 = sums.step + k;
        if (!(drift <= max_drift) || !(bdrift <= max_drift)) {  // NaN fails too
            st.fallbacks_volume++;
            rc = sw_advance_fixed_dt(solver, k, dt);
            if (!rc) rc = sw_sync(solver);
            if (rc) return sfail(n, rc, std::string("solver: ") + sw_last_error(solver));
            continue;
        }
        if (check_every > 0 && call % check_every == 0) {
            // the plain step judges the prediction: the same k steps from the
            // same state, compared in depth
            st.checks++;
            rc = sw_advance_fixed_dt(solver, k, dt);
            if (!rc) rc = sw_get_fields(solver, f2, nullptr, nullptr, nullptr, SW_PTR_DEVICE);
            if (rc) return sfail(n, rc, std::string("solver: ") + sw_last_error(solver));
            hipLaunchKernelGGL(k_maxdiff, dim3(RED_GRID), dim3(NT), 0, n->stream, f1, f2, npix,
                               (float *)s.red);
            SHIP(n, hipGetLastError());
            std::vector<float> mx(RED_GRID);
            if ((rc = copy_out(n, mx.data(), s.red, RED_GRID * sizeof(float), SW_PTR_HOST))) return rc;
            float e = 0.0f;
            for (float v : mx) e = std::max(e, v);
            st.max_residual = std::max(st.max_residual, (double)e);
            if (!(e <= max_err)) {  // keep the plain result the solver already holds
                st.fallbacks_residual++;
                continue;
            }
        }
        rc = sw_replace_state(solver, f1, f1 + npix, f1 + 2 * npix, f1 + 3 * npix, t1, step1);
        double bound = 0.0;
        if (!rc) rc = sw_step_bound(solver, &bound);
        if (rc && rc != SW_ERR_NONFINITE) return sfail(n, rc, std::string("solver: ") + sw_last_error(solver));
        if (rc || !(dt <= bound)) {
            // the solver could not take its step from the prediction: back
            // to the call's start, and the k plain steps
            st.fallbacks_stability++;
            rc = sw_replace_state(solver, f0, f0 + npix, f0 + 2 * npix, f0 + 3 * npix, sums.t,
                                  sums.step);
            if (!rc) rc = sw_advance_fixed_dt(solver, k, dt);
            if (!rc) rc = sw_sync(solver);
            if (rc) return sfail(n, rc, std::string("solver: ") + sw_last_error(solver));
            continue;
        }
        st.kept++;
    }
    if (stats) *stats = st;
    return SW_OK;
}

// SplitMix64 (Steele, Lea & Flood 2014): the minibatch draws of sws_train.
static uint64_t splitmix64(uint64_t &state)
{
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

int sws_train(sws_net *n, const float *x, const float *target, int32_t npairs, int32_t nx,
              int32_t ny, const sws_train_cfg *cfg, sws_train_report *report, float *losses,
              int ptr_kind)
{
    if (!n || !x || !target || !cfg || npairs < 1 || nx < 1 || ny < 1) return SW_ERR_ARG;
    if (cfg->steps < 1 || cfg->batch < 1 || cfg->batch > npairs || !(cfg->lr > 0.0f))
        return sfail(n, SW_ERR_ARG, "steps >= 1, 1 <= batch <= npairs and lr > 0 are required");
    if (!train_width_ok(n, nx)) return SW_ERR_ARG;
    const long npix = (long)nx * ny;
    const size_t xb = (size_t)npairs * 5 * npix * sizeof(float);
    const size_t tb = (size_t)npairs * 4 * npix * sizeof(float);
    const size_t bx = (size_t)cfg->batch * 5 * npix * sizeof(float);
    const size_t bt = (size_t)cfg->batch * 4 * npix * sizeof(float);
    // the whole set resides on the device; each step gathers its minibatch
    char *set = nullptr;
    int *didx = nullptr;
    SHIP(n, hipMalloc(&set, xb + tb + bx + bt));
    if (hipMalloc(&didx, cfg->batch * sizeof(int)) != hipSuccess) {
        (void)hipFree(set);
        return sfail(n, SW_ERR_HIP, "hipMalloc(minibatch indices)");
    }
    float *dx = (float *)set, *dt = (float *)(set + xb);
    float *gx = (float *)(set + xb + tb), *gt = (float *)(set + xb + tb + bx);
    auto done = [&](int rc) {
        (void)hipStreamSynchronize(n->stream);
        (void)hipFree(set);
        (void)hipFree(didx);
        return rc;
    };
    int rc = copy_in(n, dx, x, xb, ptr_kind);
    if (!rc) rc = copy_in(n, dt, target, tb, ptr_kind);
    if (rc) return done(rc);
    uint64_t state = cfg->seed;
    std::vector<int> perm(npairs), pick(cfg->batch);
    double first = 0.0, tail = 0.0;
    const int ntail = std::min(50, (int)cfg->steps);
    int *hidx = nullptr;
    if (hipHostMalloc((void **)&hidx, cfg->batch * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return done(sfail(n, SW_ERR_HIP, "hipHostMalloc(minibatch indices)"));
    for (int32_t it = 0; it < cfg->steps && !rc; ++it) {
        // batch distinct pairs: a partial Fisher-Yates shuffle
        for (int i = 0; i < npairs; ++i) perm[i] = i;
        for (int i = 0; i < cfg->batch; ++i) {
            const int j = i + (int)(splitmix64(state) % (uint64_t)(npairs - i));
            std::swap(perm[i], perm[j]);
            hidx[i] = perm[i];
        }
        if (hipMemcpyAsync(didx, hidx, cfg->batch * sizeof(int), hipMemcpyHostToDevice, n->stream) !=
            hipSuccess) {
            rc = sfail(n, SW_ERR_HIP, "index upload");
            break;
        }
        hipLaunchKernelGGL(k_gather, dim3(grid_for((long)cfg->batch * 5 * npix)), dim3(NT), 0,
                           n->stream, dx, didx, cfg->batch, 5, npix, gx);
        hipLaunchKernelGGL(k_gather, dim3(grid_for((long)cfg->batch * 4 * npix)), dim3(NT), 0,
                           n->stream, dt, didx, cfg->batch, 4, npix, gt);
        // cosine decay of the learning rate to 0 over the steps
        const float lr = (float)(cfg->lr * 0.5 * (1.0 + std::cos(M_PI * it / cfg->steps)));
        const bool want = losses || it == 0 || it >= cfg->steps - ntail;
        double loss = 0.0;
        rc = sws_train_step(n, gx, gt, cfg->batch, nx, ny, lr, want ? &loss : nullptr, SW_PTR_DEVICE);
        // the indices buffer is rewritten next step: wait for its use
        if (!rc && !want && hipStreamSynchronize(n->stream) != hipSuccess)
            rc = sfail(n, SW_ERR_HIP, "hipStreamSynchronize");
        if (rc) break;
        if (losses) losses[it] = (float)loss;
        if (it == 0) first = loss;
        if (it >= cfg->steps - ntail) tail += loss;
    }
    (void)hipStreamSynchronize(n->stream);
    (void)hipHostFree(hidx);
    if (!rc && report) {
        report->first_loss = first;
        report->final_loss = tail / ntail;
        report->steps = cfg->steps;
    }
    return done(rc);
}

const char *sws_last_error(const sws_net *n) { return n ? n->err.c_str() : "null net"; }

}  // extern "C"
