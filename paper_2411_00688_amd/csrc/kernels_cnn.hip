// Learned TV prox on gfx950: a 3x3 convolutional network 2 -> 32 -> 32 -> 32
// -> 2 that predicts a dual field qt, followed by the dual-to-primal head
// z = P_X(v + div P_lam(qt)) (the primal recovery u = b + div q of Sec. 2.1
// and the ball projection of eq. (7)).
//
// Every convolution is an implicit GEMM on the BF16 matrix cores with FP32
// accumulation (v_mfma_f32_16x16x32_bf16):
//   forward      out[co](p)     = sum_{t,ci} W[t][ci][co] x[ci](p + o_t)
//                M = output channels, N = 16 pixels of a tile row, K = (tap, ci)
//   input grad   gx[ci](p)      = sum_{t,co} W[t][ci][co] g[co](p - o_t)
//                the same kernel with the taps mirrored and W transposed
//   weight grad  dW[t][ci][co]  = sum_p x[ci](p + o_t) g[co](p)
//                M = output channels, N = (tap, ci) plus a column of ones for
//                the bias, K = pixels; per-block partial sums reduced in a
//                fixed order afterwards (deterministic).
// Activations are stored channel-last in BF16 (64 bytes per pixel for 32
// channels), so one lane's eight K values of a tap are one 16-byte load.
#include <hip/hip_runtime.h>

#include "tvs_internal.hpp"

namespace tvs {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bf16, round to nearest even: the gfx950 conversion instruction
// (v_cvt_pk_bf16_f32).  For finite inputs (denormals included) round to
// nearest even is the integer rounding of the bit pattern,
// (u + 0x7FFF + lsb) >> 16.  The parity tests compare the network against
// the float64 oracle within the bounds BF16 operands allow.
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
// two conversions in one instruction: a in the low half, b in the high half
__device__ __forceinline__ uint32_t f2bf_pk(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t){a, b}, bf16x2_t));
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ bool bf_pos(uint16_t b) { return b != 0 && !(b & 0x8000u); }

__device__ __forceinline__ bf16x8 as_bf8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float ball_scale_f(float wy, float wx, float lam) {
    float n2 = wy * wy + wx * wx;
    return (n2 > lam * lam) ? lam * __builtin_amdgcn_rsqf(fmaxf(n2, 1e-37f)) : 1.0f;
}

// ------------------------------------------------------------------ conv
// One block computes 16 x 16 output pixels of one image per tile and loops
// over tiles (the weights are staged once per block).  With SPLIT, every
// operand is carried as a pair of BF16 numbers x = hi + lo (lo = the BF16
// rounding of x - hi) and each K slice takes three MFMAs, hi*hi + hi*lo +
// lo*hi: still BF16 matrix-core work with FP32 accumulation, with a
// product error near 2^-16 instead of 2^-8.
template <int CIN, int COUTP, int IN, int OUT, bool SPLIT>
__global__ __launch_bounds__(SPLIT ? 512 : 256) void conv3x3_kernel(ConvArgs a) {
    if (a.run && *a.run == 0) return;  // the gate has already decided this call
    constexpr int NT = SPLIT ? 512 : 256;
    constexpr int NW = NT / 64;
    constexpr int RPW = CONV_TILE / NW;            // output rows per wave
    constexpr int NS = SPLIT ? 2 : 1;              // operand parts (hi, lo)
    constexpr int KP = (9 * CIN + 31) / 32 * 32;   // K padded to the MFMA depth
    constexpr int WST = KP + 8;                    // LDS row stride of the weights
    constexpr int P = CONV_TILE + 2;               // input patch edge (halo 1)
    constexpr int PST = (CIN == 32) ? 40 : 2;      // LDS pixel stride (bf16)
    constexpr int MB = COUTP / 16;
    // CIN = 32: every wave keeps all its weight fragments in registers for the
    // block's lifetime (9 taps x MB x NS x 16 bytes); only the activations
    // go through LDS.  CIN = 2: one K slice, staged once through LDS.
    constexpr int WS = (CIN == 32) ? 8 : COUTP * WST;
    // CIN = 32: two patch buffers; the next tile's patch is fetched into
    // registers while the current tile's MFMAs run (one barrier per tile)
    constexpr int NBUF = (CIN == 32) ? 2 : 1;
    constexpr int NLD = (P * P * 4 + NT - 1) / NT;  // 16-byte patch loads per thread and part
    __shared__ __attribute__((aligned(16))) uint16_t s_w[NS][WS];
    __shared__ __attribute__((aligned(16))) uint16_t s_x[NBUF][NS][P * P * PST];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nl = lane & 15, g = lane >> 4;
    const int H = a.H, W = a.W;

    bf16x8 wreg[NS][(CIN == 32) ? 9 : 1][MB];
    if constexpr (CIN == 32) {
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const uint16_t* src = sp == 0 ? a.wt : a.wt_lo;
#pragma unroll
            for (int t = 0; t < 9; ++t)
#pragma unroll
                for (int m = 0; m < MB; ++m)
                    wreg[sp][t][m] = as_bf8(*(const uint4*)&src[(size_t)(m * 16 + nl) * KP + t * 32 + g * 8]);
        }
    } else {
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const uint16_t* src = sp == 0 ? a.wt : a.wt_lo;
            for (int idx = tid; idx < COUTP * KP / 8; idx += NT) {
                int row = idx / (KP / 8), c8 = idx % (KP / 8);
                *(uint4*)&s_w[sp][row * WST + c8 * 8] = *(const uint4*)&src[(size_t)row * KP + c8 * 8];
            }
        }
        __syncthreads();
#pragma unroll
        for (int sp = 0; sp < NS; ++sp)
#pragma unroll
            for (int m = 0; m < MB; ++m)
                wreg[sp][0][m] = as_bf8(*(const uint4*)&s_w[sp][(m * 16 + nl) * WST + g * 8]);
    }

    // CIN = 32: the input patch of a tile (18 x 18 pixels x 32 channels, zero
    // outside the image) as NLD 16-byte loads per thread and part
    uint4 pre[NS][NLD];
    auto fetch = [&](int tile) {
        const int img = tile / (a.tiles_x * a.tiles_y);
        const int rem = tile % (a.tiles_x * a.tiles_y);
        const int i0 = (rem / a.tiles_x) * CONV_TILE, j0 = (rem % a.tiles_x) * CONV_TILE;
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const uint16_t* src = sp == 0 ? a.in : a.in_lo;
#pragma unroll
            for (int u = 0; u < NLD; ++u) {
                const int idx = tid + u * NT;
                const int p = idx >> 2, c = idx & 3;
                const int gi = i0 + p / P - 1, gj = j0 + p % P - 1;
                uint4 val = make_uint4(0, 0, 0, 0);
                if (idx < P * P * 4 && gi >= 0 && gi < H && gj >= 0 && gj < W)
                    val = *(const uint4*)&src[(((size_t)img * H + gi) * W + gj) * 32 + c * 8];
                pre[sp][u] = val;
            }
        }
    };
    if constexpr (CIN == 32) {
        if ((int)blockIdx.x < a.n_tiles) fetch((int)blockIdx.x);
    }
    int buf = 0;
    for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x, buf ^= (NBUF - 1)) {
        const int img = tile / (a.tiles_x * a.tiles_y);
        const int rem = tile % (a.tiles_x * a.tiles_y);
        const int i0 = (rem / a.tiles_x) * CONV_TILE, j0 = (rem % a.tiles_x) * CONV_TILE;
        if constexpr (CIN == 32) {
            // buffer buf was last read two tiles ago, before the previous barrier
#pragma unroll
            for (int sp = 0; sp < NS; ++sp)
#pragma unroll
                for (int u = 0; u < NLD; ++u) {
                    const int idx = tid + u * NT;
                    if (idx < P * P * 4)
                        *(uint4*)&s_x[buf][sp][(idx >> 2) * PST + (idx & 3) * 8] = pre[sp][u];
                }
            __syncthreads();
            if (tile + (int)gridDim.x < a.n_tiles) fetch(tile + (int)gridDim.x);
        } else {
            __syncthreads();
            for (int p = tid; p < P * P; p += NT) {
                int gi = i0 + p / P - 1, gj = j0 + p % P - 1;
                uint32_t hi = 0, lo = 0;
                if (gi >= 0 && gi < H && gj >= 0 && gj < W) {
                    size_t o = ((size_t)img * H + gi) * W + gj;
                    if (IN == IN_VLAM) {
                        const float v = a.v[o], l = a.lam[img];
                        const uint16_t vh = f2bf(v), lh = f2bf(l);
                        hi = (uint32_t)vh | ((uint32_t)lh << 16);
                        lo = (uint32_t)f2bf(v - bf2f(vh)) | ((uint32_t)f2bf(l - bf2f(lh)) << 16);
                    } else {
                        hi = *(const uint32_t*)&a.in[o * 2];
                    }
                }
                *(uint32_t*)&s_x[0][0][p * PST] = hi;
                if (SPLIT) *(uint32_t*)&s_x[0][NS - 1][p * PST] = lo;
            }
            __syncthreads();
        }

        f32x4 acc[MB][RPW];
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int r = 0; r < RPW; ++r) acc[m][r] = f32x4{0.f, 0.f, 0.f, 0.f};

        if (CIN == 32) {
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3, dx = t % 3;
#pragma unroll
                for (int rb = 0; rb < RPW; ++rb) {
                    const int pr = wave * RPW + rb + dy, pc = nl + dx;
                    bf16x8 xb[NS];
#pragma unroll
                    for (int sp = 0; sp < NS; ++sp)
                        xb[sp] = as_bf8(*(const uint4*)&s_x[buf][sp][(pr * P + pc) * PST + g * 8]);
#pragma unroll
                    for (int m = 0; m < MB; ++m) {
                        acc[m][rb] = mfma(wreg[0][t][m], xb[0], acc[m][rb]);
                        if (SPLIT) {
                            acc[m][rb] = mfma(wreg[0][t][m], xb[NS - 1], acc[m][rb]);
                            acc[m][rb] = mfma(wreg[NS - 1][t][m], xb[0], acc[m][rb]);
                        }
                    }
                }
            }
        } else {
            // K = (tap, ci) with k = 2 t + ci: lane group g holds taps 4g .. 4g+3
#pragma unroll
            for (int rb = 0; rb < RPW; ++rb) {
                bf16x8 xb[NS];
#pragma unroll
                for (int sp = 0; sp < NS; ++sp) {
                    uint32_t w4[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int t = 4 * g + j;
                        const int pr = wave * RPW + rb + t / 3, pc = nl + t % 3;
                        w4[j] = (t < 9) ? *(const uint32_t*)&s_x[0][sp][(pr * P + pc) * PST] : 0u;
                    }
                    xb[sp] = as_bf8(make_uint4(w4[0], w4[1], w4[2], w4[3]));
                }
#pragma unroll
                for (int m = 0; m < MB; ++m) {
                    acc[m][rb] = mfma(wreg[0][0][m], xb[0], acc[m][rb]);
                    if (SPLIT) {
                        acc[m][rb] = mfma(wreg[0][0][m], xb[NS - 1], acc[m][rb]);
                        acc[m][rb] = mfma(wreg[NS - 1][0][m], xb[0], acc[m][rb]);
                    }
                }
            }
        }

        // epilogue: lane holds channels 16 m + 4 g + r of pixel (row rb, column nl)
#pragma unroll
        for (int rb = 0; rb < RPW; ++rb) {
            const int i = i0 + wave * RPW + rb, j = j0 + nl;
            if (i >= H || j >= W) continue;
            const size_t pix = ((size_t)img * H + i) * W + j;
            if (OUT == OUT_F32_PLANAR) {
                if (g == 0) {
                    float qy = acc[0][rb][0] + a.bias[0];
                    float qx = acc[0][rb][1] + a.bias[1];
                    if (a.proj) {
                        float s = ball_scale_f(qy, qx, a.lam[img]);
                        qy *= s;
                        qx *= s;
                    }
                    const size_t plane = (size_t)H * W;
                    a.out_f[(size_t)img * 2 * plane + (size_t)i * W + j] = qy;
                    a.out_f[(size_t)img * 2 * plane + plane + (size_t)i * W + j] = qx;
                }
            } else {
#pragma unroll
                for (int m = 0; m < MB; ++m) {
                    const int c0 = m * 16 + 4 * g;
                    if (OUT == OUT_RELU_BF16) {
                        float val[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) val[r] = fmaxf(acc[m][rb][r] + a.bias[c0 + r], 0.f);
                        const uint32_t h01 = f2bf_pk(val[0], val[1]), h23 = f2bf_pk(val[2], val[3]);
                        *(uint2*)&a.out_bf[pix * 32 + c0] = make_uint2(h01, h23);
                        if (SPLIT) {
                            // lo = bf16(val - hi)
                            const uint32_t l01 = f2bf_pk(val[0] - __uint_as_float(h01 << 16),
                                                         val[1] - __uint_as_float(h01 & 0xFFFF0000u));
                            const uint32_t l23 = f2bf_pk(val[2] - __uint_as_float(h23 << 16),
                                                         val[3] - __uint_as_float(h23 & 0xFFFF0000u));
                            *(uint2*)&a.out_lo[pix * 32 + c0] = make_uint2(l01, l23);
                        }
                    } else {  // OUT_MASK_BF16
                        uint2 mk = *(const uint2*)&a.mask[pix * 32 + c0];
                        uint16_t mm[4] = {(uint16_t)(mk.x & 0xFFFF), (uint16_t)(mk.x >> 16),
                                          (uint16_t)(mk.y & 0xFFFF), (uint16_t)(mk.y >> 16)};
                        uint16_t o[4];
#pragma unroll
                        for (int r = 0; r < 4; ++r) o[r] = bf_pos(mm[r]) ? f2bf(acc[m][rb][r]) : (uint16_t)0;
                        *(uint2*)&a.out_bf[pix * 32 + c0] =
                            make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16),
                                       (uint32_t)o[2] | ((uint32_t)o[3] << 16));
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ weight gradient
// Tile of WG_TH x 16 pixels.  LDS holds three copies of the input patch,
// shifted by dx = -1, 0, +1 and stored channel-planar, so that the eight
// pixels a lane needs for one K slice are one aligned 16-byte read.
template <int CIN, int COUT, int XIN, int GIN>
__global__ __launch_bounds__(CONV_NT) void conv3x3_wgrad_kernel(WgradArgs a) {
    constexpr int COUTP = (COUT + 15) / 16 * 16;
    constexpr int MB = COUTP / 16;
    constexpr int NCOL = 9 * CIN + 1;              // (tap, ci) columns and the bias column
    constexpr int NB = (NCOL + 15) / 16;
    constexpr int NBW = (NB + 3) / 4;              // column blocks per wave
    constexpr int PR = WG_TH + 2;                  // patch rows
    constexpr int TPX = WG_TH * 16;                // pixels per tile
    constexpr int GST = TPX + 8;                   // LDS row stride of g
    __shared__ __attribute__((aligned(16))) uint16_t s_x[3 * CIN * PR * 16];
    __shared__ __attribute__((aligned(16))) uint16_t s_g[COUTP * GST];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nl = lane & 15, g = lane >> 4;
    const int H = a.H, W = a.W;

    f32x4 acc[MB][NBW];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int s = 0; s < NBW; ++s) acc[m][s] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const int img = tile / (a.tiles_x * a.tiles_y);
        const int rem = tile % (a.tiles_x * a.tiles_y);
        const int i0 = (rem / a.tiles_x) * WG_TH, j0 = (rem % a.tiles_x) * 16;
        __syncthreads();
        // input patch, rows i0-1 .. i0+WG_TH, columns j0-1 .. j0+16
        for (int idx = tid; idx < PR * 18; idx += CONV_NT) {
            const int pr = idx / 18, pc = idx % 18;
            const int gi = i0 + pr - 1, gj = j0 + pc - 1;
            const bool in = gi >= 0 && gi < H && gj >= 0 && gj < W;
            const size_t o = ((size_t)img * H + (in ? gi : 0)) * W + (in ? gj : 0);
            for (int ci = 0; ci < CIN; ++ci) {
                uint16_t val = 0;
                if (in) {
                    if (XIN == IN_VLAM)
                        val = ci == 0 ? f2bf(a.v[o]) : f2bf(a.lam[img]);
                    else
                        val = a.x[o * CIN + ci];
                }
                // copy dx holds column pc - dx at position pc - dx (0..15)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int c = pc - dx;
                    if (c >= 0 && c < 16) s_x[((dx * CIN + ci) * PR + pr) * 16 + c] = val;
                }
            }
        }
        // output gradient of the tile, channel-planar
        for (int idx = tid; idx < TPX; idx += CONV_NT) {
            const int i = i0 + idx / 16, j = j0 + idx % 16;
            const bool in = i < H && j < W;
            const size_t o = ((size_t)img * H + (in ? i : 0)) * W + (in ? j : 0);
            for (int co = 0; co < COUTP; ++co)
                s_g[co * GST + idx] = (in && co < COUT) ? a.g[o * GIN + co] : (uint16_t)0;
        }
        __syncthreads();

#pragma unroll
        for (int kb = 0; kb < TPX / 32; ++kb) {
            // K slice: pixels 32 kb + 8 g .. +7 = tile row 2 kb + g / 2, columns 8 (g & 1) .. +7
            const int prow = 2 * kb + (g >> 1), c0 = 8 * (g & 1);
            bf16x8 ga[MB];
#pragma unroll
            for (int m = 0; m < MB; ++m)
                ga[m] = as_bf8(*(const uint4*)&s_g[(m * 16 + nl) * GST + kb * 32 + 8 * g]);
#pragma unroll
            for (int s = 0; s < NBW; ++s) {
                const int nb = wave + 4 * s;
                if (nb >= NB) break;
                const int col = nb * 16 + nl;
                uint4 xv = make_uint4(0, 0, 0, 0);
                if (col < 9 * CIN) {
                    const int t = col / CIN, ci = col % CIN;
                    const int dy = t / 3, dx = t % 3;
                    xv = *(const uint4*)&s_x[((dx * CIN + ci) * PR + prow + dy) * 16 + c0];
                } else if (col == 9 * CIN) {
                    xv = make_uint4(0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u);
                }
                const bf16x8 xb = as_bf8(xv);
#pragma unroll
                for (int m = 0; m < MB; ++m) acc[m][s] = mfma(ga[m], xb, acc[m][s]);
            }
        }
    }

    // partial sums of this block, in the parameter order (col * COUT + co)
    float* part = a.part + (size_t)blockIdx.x * (NCOL * COUT);
#pragma unroll
    for (int s = 0; s < NBW; ++s) {
        const int nb = wave + 4 * s;
        if (nb >= NB) break;
        const int col = nb * 16 + nl;
        if (col >= NCOL) continue;
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = m * 16 + 4 * g + r;
                if (co < COUT) part[col * COUT + co] = acc[m][s][r];
            }
    }
}

// Fixed-order sum of the per-block partials into the gradient vector.  A
// block covers 32 consecutive entries; its 8 thread rows each sum every 8th
// partial (rows r, r + 8, ...), then the 8 row sums are added in row order.
constexpr int WR_COLS = 32, WR_ROWS = 8;
__global__ __launch_bounds__(WR_COLS* WR_ROWS) void wgrad_reduce_kernel(const float* part,
                                                                      int nblocks, int len,
                                                                      float* out) {
    __shared__ float s[WR_ROWS][WR_COLS];
    const int c = threadIdx.x % WR_COLS, r = threadIdx.x / WR_COLS;
    const int idx = blockIdx.x * WR_COLS + c;
    float acc = 0.f;
    if (idx < len)
        for (int b = r; b < nblocks; b += WR_ROWS) acc += part[(size_t)b * len + idx];
    s[r][c] = acc;
    __syncthreads();
    if (r == 0 && idx < len) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < WR_ROWS; ++k) t += s[k][c];
        out[idx] = t;
    }
}

// ------------------------------------------------------------------ head
// z = P_X(v + div P_lam(qt)); training mode also forms the loss terms and
// g_u = dL/du; inference mode stores P_lam(qt) and z.
__global__ void head_fwd_kernel(HeadArgs a) {
    const int H = a.H, W = a.W;
    const size_t plane = (size_t)H * W;
    const size_t tot = (size_t)a.n * plane;
    __shared__ float s_red[256];
    float sq = 0.f;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int img = (int)(idx / plane);
        const size_t p = idx % plane;
        const int i = (int)(p / W), j = (int)(p % W);
        const float lam = a.lam[img];
        const float* qy = a.qt + (size_t)img * 2 * plane;
        const float* qx = qy + plane;
        const float sc = ball_scale_f(qy[p], qx[p], lam);
        float d = 0.f;
        if (i < H - 1) d += qy[p] * sc;
        if (j < W - 1) d += qx[p] * sc;
        if (i > 0) d -= qy[p - W] * ball_scale_f(qy[p - W], qx[p - W], lam);
        if (j > 0) d -= qx[p - 1] * ball_scale_f(qy[p - 1], qx[p - 1], lam);
        const float u = a.v[idx] + d;
        const bool act = !a.nonneg || u > 0.f;
        const float z = act ? u : 0.f;
        if (a.z) a.z[idx] = z;
        if (a.z_target) {
            const float e = z - a.z_target[idx];
            sq += e * e;
            a.gu[idx] = act ? e * a.inv_npx : 0.f;
            if (a.q_target) {
                const float* tg = a.q_target + (size_t)img * 2 * plane;
                const float ry = qy[p] * sc - tg[p], rx = qx[p] * sc - tg[plane + p];
                sq += a.mu * (ry * ry + rx * rx);
            }
        }
    }
    if (!a.z_target) return;
    s_red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) s_red[threadIdx.x] += s_red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = (double)s_red[0];
}

// g_qt = J_{P_lam}(qt)^T (-D g_u + mu (q - q_target) / pixels), stored
// channel-last BF16 (2 channels)
__global__ void head_bwd_kernel(HeadArgs a) {
    const int H = a.H, W = a.W;
    const size_t plane = (size_t)H * W;
    const size_t tot = (size_t)a.n * plane;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int img = (int)(idx / plane);
        const size_t p = idx % plane;
        const int i = (int)(p / W), j = (int)(p % W);
        const float gu = a.gu[idx];
        const float gy = (i < H - 1) ? -(a.gu[idx + W] - gu) : 0.f;
        const float gx = (j < W - 1) ? -(a.gu[idx + 1] - gu) : 0.f;
        const float lam = a.lam[img];
        const float qy = a.qt[(size_t)img * 2 * plane + p];
        const float qx = a.qt[(size_t)img * 2 * plane + plane + p];
        float oy = gy, ox = gx;
        const float n2 = qy * qy + qx * qx;
        if (a.q_target) {
            const float sc = ball_scale_f(qy, qx, lam);
            const float* tg = a.q_target + (size_t)img * 2 * plane;
            oy += a.mu * (qy * sc - tg[p]) * a.inv_npx;
            ox += a.mu * (qx * sc - tg[plane + p]) * a.inv_npx;
        }
        const float by = oy, bx = ox;
        if (n2 > lam * lam) {
            const float rn = __builtin_amdgcn_rsqf(fmaxf(n2, 1e-37f));
            const float ny = qy * rn, nx = qx * rn, s = lam * rn;
            const float dot = ny * by + nx * bx;
            oy = s * (by - ny * dot);
            ox = s * (bx - nx * dot);
        }
        *(uint32_t*)&a.gq_bf[idx * 2] = (uint32_t)f2bf(oy) | ((uint32_t)f2bf(ox) << 16);
    }
}

// Fixed-order sum of n doubles by one block: thread t adds elements t,
// t + 256, ... in order, then a fixed pairwise tree over the 256 sums.
__global__ __launch_bounds__(256) void sum_doubles_kernel(const double* part, int n, double* out) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

// ------------------------------------------------------------------ optimiser
// Adam (Kingma and Ba, 2015) on the FP32 master parameters.
__global__ void adam_kernel(int n, float* p, const float* grad, float* m, float* v, float lr,
                            float b1, float b2, float c1, float c2, float eps) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 copies of one layer's weights in the two GEMM layouts:
//   forward     wf[co][t * CIN + ci]    = W[t][ci][co]   (rows padded to COUTP, K to KP)
//   input grad  wb[ci][t' * COUT + co]  = W[8 - t'][ci][co]  (mirrored taps)
__global__ void pack_weights_kernel(const float* w, int cin, int cout, int coutp, int kp,
                                    uint16_t* wf, uint16_t* wf_lo, int kpb, uint16_t* wb) {
    const int nf = coutp * kp;
    const int nb = wb ? 32 * kpb : 0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nf + nb;
         idx += gridDim.x * blockDim.x) {
        if (idx < nf) {
            const int co = idx / kp, k = idx % kp;
            float val = 0.f;
            if (co < cout && k < 9 * cin) val = w[(size_t)k * cout + co];  // k = t * cin + ci
            const uint16_t hi = f2bf(val);
            wf[idx] = hi;
            wf_lo[idx] = f2bf(val - bf2f(hi));
        } else {
            const int r = idx - nf;
            const int ci = r / kpb, k = r % kpb;
            float val = 0.f;
            if (ci < cin && k < 9 * cout) {
                const int tp = k / cout, co = k % cout;
                val = w[((size_t)(8 - tp) * cin + ci) * cout + co];
            }
            wb[r] = f2bf(val);
        }
    }
}

// ------------------------------------------------------------------ gate
// Gate of a learned prox call inside a solver run.  red[0], red[1]: gap and
// primal value at the network's dual; red[2], red[3]: the same at the
// previous call's dual.
// pregate: run = 0 when the previous dual's relative gap is at most tol
// (it is the call's result; the network is not evaluated), else 1.
// gate: with run = 0, flag = 0 and sel = 0.  Otherwise flag = 0 when the
// network's relative gap is at most tol (its dual is the result), else 1
// (FGP runs; a NaN gap falls back too); sel = 1 when the network's dual is
// the result or FGP's start: gate open, or a relative gap below the
// previous dual's.
__device__ __forceinline__ double rel_gap(const double* r) { return r[1] > 0.0 ? r[0] / r[1] : r[0]; }

__global__ void pregate_kernel(const double* red, double tol, int* run) {
    if (blockIdx.x == 0 && threadIdx.x == 0) run[0] = rel_gap(red + 2) <= tol ? 0 : 1;
}

__global__ void gate_kernel(const double* red, double tol, const int* run, int* flag, int* sel) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (run && run[0] == 0) {
            flag[0] = 0;
            sel[0] = 0;
            return;
        }
        const double rn = rel_gap(red), rp = rel_gap(red + 2);
        const int f = rn <= tol ? 0 : 1;
        flag[0] = f;
        sel[0] = (f == 0 || rn < rp) ? 1 : 0;
    }
}

// dst = src where (*flag != 0) == (when != 0)
__global__ void copy_if_kernel(size_t n, const int* flag, int when, const float* src, float* dst) {
    if ((*flag != 0) != (when != 0)) return;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ------------------------------------------------------------------ launchers
static int grid_for(const tvs_ctx* ctx, int tiles, int per_cu) {
    int g = ctx->n_cu * per_cu;
    return tiles < g ? tiles : g;
}

void launch_conv(tvs_ctx* ctx, int cin, int coutp, int in_mode, int out_mode, bool split,
                 ConvArgs a) {
    a.tiles_x = div_up(a.W, CONV_TILE);
    a.tiles_y = div_up(a.H, CONV_TILE);
    a.n_tiles = a.tiles_x * a.tiles_y * a.n;
    if (a.n_tiles == 0) return;
    TVS_REQUIRE(!split || (a.wt_lo && (in_mode == IN_VLAM || a.in_lo) &&
                           (out_mode != OUT_RELU_BF16 || a.out_lo)),
                TVS_ERR_INVALID_ARG, "conv3x3: split operands missing");
    TVS_REQUIRE(!split || out_mode != OUT_MASK_BF16, TVS_ERR_UNSUPPORTED,
                "conv3x3: the input-gradient pass is single-part");
    hipStream_t st = ctx->stream;
    // register-resident weights (32 input channels) leave room for two 4-wave
    // blocks (single part) or one 8-wave block (two parts) per CU, three for
    // the 2-channel output layer; the first layer (2 input channels, weights
    // through LDS) fits four single-part blocks or two two-part blocks
    const int per_cu = cin == 2 ? (split ? 2 : 4) : (coutp == 16 && !split ? 3 : (split ? 1 : 2));
    const dim3 grid(grid_for(ctx, a.n_tiles, per_cu)), block(split ? 512 : 256);
#define TVS_CONV(CI, CO, IM, OM, SP) conv3x3_kernel<CI, CO, IM, OM, SP><<<grid, block, 0, st>>>(a)
    if (cin == 2 && coutp == 32 && in_mode == IN_VLAM && out_mode == OUT_RELU_BF16) {
        if (split) TVS_CONV(2, 32, IN_VLAM, OUT_RELU_BF16, true);
        else TVS_CONV(2, 32, IN_VLAM, OUT_RELU_BF16, false);
    } else if (cin == 32 && coutp == 32 && in_mode == IN_BF16 && out_mode == OUT_RELU_BF16) {
        if (split) TVS_CONV(32, 32, IN_BF16, OUT_RELU_BF16, true);
        else TVS_CONV(32, 32, IN_BF16, OUT_RELU_BF16, false);
    } else if (cin == 32 && coutp == 16 && in_mode == IN_BF16 && out_mode == OUT_F32_PLANAR) {
        if (split) TVS_CONV(32, 16, IN_BF16, OUT_F32_PLANAR, true);
        else TVS_CONV(32, 16, IN_BF16, OUT_F32_PLANAR, false);
    } else if (!split && cin == 2 && coutp == 32 && in_mode == IN_BF16 && out_mode == OUT_MASK_BF16) {
        TVS_CONV(2, 32, IN_BF16, OUT_MASK_BF16, false);
    } else if (!split && cin == 32 && coutp == 32 && in_mode == IN_BF16 && out_mode == OUT_MASK_BF16) {
        TVS_CONV(32, 32, IN_BF16, OUT_MASK_BF16, false);
    } else {
        throw Error{TVS_ERR_UNSUPPORTED, "conv3x3: unsupported layer shape"};
    }
#undef TVS_CONV
    TVS_LAUNCH_CHECK();
}

int wgrad_blocks(const tvs_ctx* ctx, int n, int H, int W) {
    int tiles = div_up(W, 16) * div_up(H, WG_TH) * n;
    return grid_for(ctx, tiles, 2);
}

void launch_wgrad(tvs_ctx* ctx, int layer, WgradArgs a, float* grad_out) {
    a.tiles_x = div_up(a.W, 16);
    a.tiles_y = div_up(a.H, WG_TH);
    a.n_tiles = a.tiles_x * a.tiles_y * a.n;
    const int nblk = grid_for(ctx, a.n_tiles, 2);
    hipStream_t st = ctx->stream;
    int len = 0;
    switch (layer) {
        case 0:
            conv3x3_wgrad_kernel<2, 32, IN_VLAM, 32><<<nblk, CONV_NT, 0, st>>>(a);
            len = 19 * 32;
            break;
        case 1:
        case 2:
            conv3x3_wgrad_kernel<32, 32, IN_BF16, 32><<<nblk, CONV_NT, 0, st>>>(a);
            len = 289 * 32;
            break;
        case 3:
            conv3x3_wgrad_kernel<32, 2, IN_BF16, 2><<<nblk, CONV_NT, 0, st>>>(a);
            len = 289 * 2;
            break;
        default:
            throw Error{TVS_ERR_INVALID_ARG, "wgrad: bad layer"};
    }
    TVS_LAUNCH_CHECK();
    wgrad_reduce_kernel<<<div_up(len, WR_COLS), WR_COLS * WR_ROWS, 0, st>>>(a.part, nblk, len,
                                                                          grad_out);
    TVS_LAUNCH_CHECK();
}

int head_blocks(const tvs_ctx* ctx, size_t tot) {
    size_t b = (tot + 255) / 256;
    size_t cap = (size_t)ctx->n_cu * 8;
    return (int)(b < cap ? b : cap);
}

void launch_head_fwd(tvs_ctx* ctx, HeadArgs a, int nblk) {
    head_fwd_kernel<<<nblk, 256, 0, ctx->stream>>>(a);
    TVS_LAUNCH_CHECK();
    if (a.z_target) {
        sum_doubles_kernel<<<1, 256, 0, ctx->stream>>>(a.loss_part, nblk, a.loss_out);
        TVS_LAUNCH_CHECK();
    }
}

void launch_head_bwd(tvs_ctx* ctx, HeadArgs a, int nblk) {
    head_bwd_kernel<<<nblk, 256, 0, ctx->stream>>>(a);
    TVS_LAUNCH_CHECK();
}

void launch_adam(tvs_ctx* ctx, int n, float* p, const float* grad, float* m, float* v, float lr,
                 float b1, float b2, float c1, float c2, float eps) {
    adam_kernel<<<div_up(n, 256), 256, 0, ctx->stream>>>(n, p, grad, m, v, lr, b1, b2, c1, c2, eps);
    TVS_LAUNCH_CHECK();
}

void launch_pack(tvs_ctx* ctx, const float* w, int cin, int cout, uint16_t* wf, uint16_t* wf_lo,
                 uint16_t* wb) {
    const int coutp = (cout + 15) / 16 * 16;
    const int kp = (9 * cin + 31) / 32 * 32;
    const int kpb = (9 * cout + 31) / 32 * 32;
    const int tot = coutp * kp + (wb ? 32 * kpb : 0);
    pack_weights_kernel<<<div_up(tot, 256), 256, 0, ctx->stream>>>(w, cin, cout, coutp, kp, wf,
                                                                    wf_lo, kpb, wb);
    TVS_LAUNCH_CHECK();
}

void launch_pregate(tvs_ctx* ctx, const double* red, double tol, int* run) {
    pregate_kernel<<<1, 64, 0, ctx->stream>>>(red, tol, run);
    TVS_LAUNCH_CHECK();
}

void launch_gate(tvs_ctx* ctx, const double* red, double tol, const int* run, int* flag, int* sel) {
    gate_kernel<<<1, 64, 0, ctx->stream>>>(red, tol, run, flag, sel);
    TVS_LAUNCH_CHECK();
}

void launch_copy_if(tvs_ctx* ctx, size_t n, const int* flag, int when, const float* src,
                    float* dst) {
    size_t b = (n + 255) / 256;
    const size_t cap = (size_t)ctx->n_cu * 8;
    copy_if_kernel<<<(int)(b < cap ? b : cap), 256, 0, ctx->stream>>>(n, flag, when, src, dst);
    TVS_LAUNCH_CHECK();
}

}  // namespace cnn
}  // namespace tvs
