// Forward operators A, their adjoints, and the data-fidelity steps fused into
// their epilogues, for gfx950.
//
//  - identity: pointwise, 32 x 32 tiles.
//  - periodic blur: LDS tile with a periodic halo (radius <= 8).
//  - Joseph parallel-beam projector, ray-driven: the general kernel takes one
//    wavefront per 64 adjacent bins of one angle with the row range split over
//    8 wavefronts and summed in a fixed order; in float32, when the detector
//    spacing is 1 to 2 pixels along the interpolation axis, the paired kernel
//    lets each lane carry two adjacent rays from one 16-byte gather.
//  - its exact transpose (no atomics, fixed summation order): in general a
//    pixel-driven gather (each pixel finds, per angle, the few rays whose
//    interpolation touches it and recomputes their weights with the
//    projector's arithmetic); in float32, when every angle's rays fit the
//    staged windows, a ray-driven scatter over 52 x 52 tiles and groups of
//    angles (lane permutes move each ray's two weights to its pixels' lanes)
//    whose per-group partial images a second kernel adds in order.
//
// Data-fidelity epilogue (PrimalStep), with s = grad f(x) (ProxSkip) or
// s = A^T y (PDHGSkip-2) at a pixel:
//   w = x - step s;  xhat = w + step h
//   theta = 1: v = w + (step - step/p) h  and xhat are stored for the prox
//   theta = 0: x <- xhat; for PDHGSkip also xbar = 2 xhat - x_old (and its
//              transpose, which the projector reads for column-stepping rays).
#include "tvs_internal.hpp"

namespace tvs {

// The step with x = ps.x[g] and hh = ps.h[g] already loaded.
template <typename T>
__device__ __forceinline__ T primal_step_xh(const PrimalStep<T>& ps, size_t g, int i, int j, T s,
                                            T x, T hh) {
    const T w = x - ps.step * s;
    const T xh = w + ps.step * hh;
    if (ps.theta) {
        ps.v[g] = w + ps.coef * hh;
        ps.xhat[g] = xh;
        return T(0);
    }
    ps.x[g] = xh;
    if (ps.pdhg) {
        const T xb = ps.xcopy ? xh : T(2) * xh - x;
        ps.xbar[(size_t)i * ps.xbar_ld + j] = xb;
        return xb;
    }
    return T(0);
}

template <typename T>
__device__ __forceinline__ T primal_step(const PrimalStep<T>& ps, size_t g, int i, int j, T s) {
    return primal_step_xh(ps, g, i, j, s, ps.x[g], ps.h[g]);
}

// z += s; zbar = z + nsub s (the stochastic-angle method's dual sums).
template <typename T>
__device__ __forceinline__ void z_accumulate(const ZAcc<T>& za, size_t g, T s) {
    const T zn = za.z[g] + s;
    za.z[g] = zn;
    za.zbar[g] = zn + za.nsub * s;
}

// Splits the 32.32 fixed-point coordinate U (an integer-valued double with
// |U| < 2^51) into floor(U / 2^32) and the fraction, from the bits of
// U + 1.5 2^52, whose 52-bit mantissa is exactly U + 2^51.
__device__ __forceinline__ void fx_split(double U, int& j0, float& f) {
    const double v = U + 6755399441055744.0;
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    j0 = (int)((unsigned)(b >> 32) & 0xFFFFFu) - 524288;
    f = (float)(unsigned)b * 2.3283064365386963e-10f;
}

static int grid1d(size_t n) {
    size_t b = (n + 255) / 256;
    return (int)(b < 65536 ? (b ? b : 1) : 65536);
}

// ------------------------------------------------------------- pointwise
template <typename T>
__global__ void axpby_kernel(size_t n, T a, const T* x, T b, const T* y, T* out) {
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x)
        out[g] = a * x[g] + b * y[g];
}

template <typename T>
__global__ void copy_kernel(size_t n, const T* x, T* y) {
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x)
        y[g] = x[g];
}

template <typename T>
__global__ void fill_kernel(size_t n, T val, T* y) {
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x)
        y[g] = val;
}

template <typename T>
void launch_axpby(tvs_ctx* ctx, size_t n, T a, const T* x, T b, const T* y, T* out) {
    hipLaunchKernelGGL((axpby_kernel<T>), dim3(grid1d(n)), dim3(256), 0, ctx->stream, n, a, x, b,
                       y, out);
    TVS_LAUNCH_CHECK();
}
template <typename T>
void launch_copy(tvs_ctx* ctx, size_t n, const T* x, T* y) {
    hipLaunchKernelGGL((copy_kernel<T>), dim3(grid1d(n)), dim3(256), 0, ctx->stream, n, x, y);
    TVS_LAUNCH_CHECK();
}
template <typename T>
void launch_fill(tvs_ctx* ctx, size_t n, T val, T* y) {
    hipLaunchKernelGGL((fill_kernel<T>), dim3(grid1d(n)), dim3(256), 0, ctx->stream, n, val, y);
    TVS_LAUNCH_CHECK();
}

// 32 x 32 LDS transpose: xT[j][i] = x[i][j]
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(int H, int W, const T* x, T* xT) {
    __shared__ T t[32][33];
    const int i0 = (int)blockIdx.y * 32, j0 = (int)blockIdx.x * 32;
    for (int p = 0; p < 4; ++p) {
        const int idx = (int)threadIdx.x + p * 256;
        const int li = idx / 32, lj = idx % 32;
        if (i0 + li < H && j0 + lj < W) t[li][lj] = x[(size_t)(i0 + li) * W + j0 + lj];
    }
    __syncthreads();
    for (int p = 0; p < 4; ++p) {
        const int idx = (int)threadIdx.x + p * 256;
        const int jj = idx / 32, ii = idx % 32;
        if (i0 + ii < H && j0 + jj < W) xT[(size_t)(j0 + jj) * H + i0 + ii] = t[ii][jj];
    }
}

template <typename T>
__global__ void fista_extrap_kernel(size_t n, const T* x, const T* xprev, T beta, T* out) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        out[i] = x[i] + beta * (x[i] - xprev[i]);
}

template <typename T>
void launch_fista_extrap(tvs_ctx* ctx, size_t n, const T* x, const T* xprev, T beta, T* out) {
    hipLaunchKernelGGL((fista_extrap_kernel<T>), dim3(grid1d(n)), dim3(256), 0, ctx->stream, n, x,
                       xprev, beta, out);
    TVS_LAUNCH_CHECK();
}

// Row permutation of a rows x cols array: gather dst[r] = src[perm[r]], or
// scatter dst[perm[r]] = src[r].
template <typename T>
__global__ __launch_bounds__(256) void permute_rows_kernel(int rows, int cols, const int* perm,
                                                           const T* src, T* dst, int scatter) {
    const int r = (int)blockIdx.y;
    const int c = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (r >= rows || c >= cols) return;
    const size_t pr = (size_t)perm[r];
    if (scatter)
        dst[pr * cols + c] = src[(size_t)r * cols + c];
    else
        dst[(size_t)r * cols + c] = src[pr * cols + c];
}

template <typename T>
void launch_permute_rows(tvs_ctx* ctx, int rows, int cols, const int* perm, const T* src, T* dst,
                         bool scatter) {
    hipLaunchKernelGGL((permute_rows_kernel<T>), dim3(div_up(cols, 256), rows), dim3(256), 0,
                       ctx->stream, rows, cols, perm, src, dst, scatter ? 1 : 0);
    TVS_LAUNCH_CHECK();
}

template <typename T>
void launch_transpose(tvs_ctx* ctx, int H, int W, const T* x, T* xT) {
    hipLaunchKernelGGL((transpose_kernel<T>), dim3(div_up(W, 32), div_up(H, 32)), dim3(256), 0,
                       ctx->stream, H, W, x, xT);
    TVS_LAUNCH_CHECK();
}

// Writes the 32 x 32 tile of xbar staged in LDS to xbarT, coalesced (NT
// threads per block).
template <typename T, int NT = 256>
__device__ __forceinline__ void store_tile_transposed(T (*s_t)[33], int i0, int j0, int H, int W,
                                                      T* xT, int ldT) {
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 1024 / NT; ++p) {
        const int idx = (int)threadIdx.x + p * NT;
        const int jj = idx / 32, ii = idx % 32;
        if (i0 + ii < H && j0 + jj < W) xT[(size_t)(j0 + jj) * ldT + i0 + ii] = s_t[ii][jj];
    }
}

// ---------------------------------------------------------------- identity
// s = x - b (ProxSkip gradient, from_y = 0) or s = y (PDHGSkip A^T y, from_y = 1)
// 32 x 32 pixel tiles with one pixel per thread: at 512^2 the 256 tiles give
// every CU 16 waves
constexpr int TILE_NT = 1024;

template <typename T>
__global__ __launch_bounds__(TILE_NT) void identity_step_kernel(int H, int W, const T* src,
                                                            const T* b, PrimalStep<T> ps,
                                                            int from_y) {
    __shared__ T s_t[32][33];
    const int i0 = (int)blockIdx.y * 32, j0 = (int)blockIdx.x * 32;
#pragma unroll
    for (int p = 0; p < 1024 / TILE_NT; ++p) {
        const int idx = (int)threadIdx.x + p * TILE_NT;
        const int li = idx / 32, lj = idx % 32;
        const int i = i0 + li, j = j0 + lj;
        if (i < H && j < W) {
            const size_t g = (size_t)i * W + j;
            const T s = from_y ? src[g] : ps.x[g] - b[g];
            s_t[li][lj] = primal_step(ps, g, i, j, s);
        }
    }
    if (ps.pdhg && !ps.theta && ps.xbarT)
        store_tile_transposed<T, TILE_NT>(s_t, i0, j0, H, W, ps.xbarT, ps.xbarT_ld);
}

template <typename T>
void launch_identity_step(tvs_ctx* ctx, int H, int W, const T* b, const PrimalStep<T>& ps) {
    hipLaunchKernelGGL((identity_step_kernel<T>), dim3(div_up(W, 32), div_up(H, 32)), dim3(TILE_NT),
                       0, ctx->stream, H, W, (const T*)nullptr, b, ps, 0);
    TVS_LAUNCH_CHECK();
}

template <typename T>
void launch_identity_adj_step(tvs_ctx* ctx, int H, int W, const T* y, const PrimalStep<T>& ps) {
    hipLaunchKernelGGL((identity_step_kernel<T>), dim3(div_up(W, 32), div_up(H, 32)), dim3(TILE_NT),
                       0, ctx->stream, H, W, y, (const T*)nullptr, ps, 1);
    TVS_LAUNCH_CHECK();
}

// y = (y + tau (xbar - b)) / (1 + tau), pointwise (identity PDHGSkip dual step)
template <typename T>
__global__ void dual_prox_pointwise_kernel(size_t n, const T* xb, const T* b, T* y, T tau) {
    const T den = T(1) + tau;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x)
        y[g] = (y[g] + tau * (xb[g] - b[g])) / den;
}

template <typename T>
void launch_dual_prox_pointwise(tvs_ctx* ctx, size_t n, const T* xb, const T* b, T* y, T tau) {
    hipLaunchKernelGGL((dual_prox_pointwise_kernel<T>), dim3(grid1d(n)), dim3(256), 0,
                       ctx->stream, n, xb, b, y, tau);
    TVS_LAUNCH_CHECK();
}

// Batched ProxSkip data step for A = I over all slices' 32 x 32 tiles (block
// b -> slice by binary search of the cumulative tile counts pref_all).
__device__ __forceinline__ int find_item_ops(const int* prefix, int n, int b) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <typename T>
__global__ __launch_bounds__(256) void identity_step_batched_kernel(
    const BSlice<T>* sl, const int* pref_all, int n, const uint8_t* theta, const T* b, T* x,
    const T* h, T* xhat, T* v, T step) {
    const int blk = (int)blockIdx.x;
    const int s = find_item_ops(pref_all, n, blk);
    const BSlice<T> S = sl[s];
    const int t = blk - pref_all[s];
    const int tiles_x = div_up(S.W, 32);
    const int i0 = (t / tiles_x) * 32, j0 = (t % tiles_x) * 32;
    const int th = theta[s];
    const size_t off = (size_t)S.off;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int idx = (int)threadIdx.x + p * 256;
        const int i = i0 + idx / 32, j = j0 + idx % 32;
        if (i >= S.H || j >= S.W) continue;
        const size_t g = off + (size_t)i * S.W + j;
        const T xv = x[g], hv = h[g];
        const T w = xv - step * (xv - b[g]);
        const T xh = w + step * hv;
        if (th) {
            v[g] = w + S.coef * hv;
            xhat[g] = xh;
        } else {
            x[g] = xh;
        }
    }
}

template <typename T>
void launch_identity_step_batched(tvs_ctx* ctx, const BSlice<T>* sl, const int* pref_all, int n,
                                  int tiles, const uint8_t* theta, const T* b, T* x, const T* h,
                                  T* xhat, T* v, T step) {
    hipLaunchKernelGGL((identity_step_batched_kernel<T>), dim3(tiles), dim3(256), 0, ctx->stream,
                       sl, pref_all, n, theta, b, x, h, xhat, v, step);
    TVS_LAUNCH_CHECK();
}

// -------------------------------------------------------------------- blur
enum BlurMode { BLUR_STORE = 0, BLUR_RESIDUAL = 1, BLUR_DUAL_PROX = 2, BLUR_PRIMAL = 3 };

template <typename T>
struct BlurArgs {
    const T* x;
    const T* k;
    int kh, kw;
    int adjoint;
    const T* b;
    T* out;
    int mode;
    T tau;
    PrimalStep<T> ps;
    int H, W;
};

// (A x)_{i,j} = sum_{a,c} k[a][c] x[(i - (a - kh/2)) mod H][(j - (c - kw/2)) mod W]
// (A^T y)_{i,j} = sum_{a,c} k[a][c] y[(i + (a - kh/2)) mod H][(j + (c - kw/2)) mod W]
// one pixel of the 32 x 32 output tile per thread: at 512^2 the 256 tiles
// then give every CU 16 waves
constexpr int BLUR_NT = 1024;

// KS > 0: a KS x KS kernel known at compile time (the loops unroll and the
// weights, the same for every thread, come through scalar loads instead of
// LDS); KS = 0: any odd size up to 17, read from LDS.  Same products in the
// same order either way.
template <typename T, int KS>
__global__ __launch_bounds__(BLUR_NT) void blur_kernel(BlurArgs<T> a) {
    constexpr int TW = 32, TH = 32, RMAX = 8;
    constexpr int LW = TW + 2 * RMAX, LH = TH + 2 * RMAX;
    __shared__ T s_x[LH][LW + 1];
    __shared__ T s_k[17 * 17];
    __shared__ T s_t[32][33];
    const int H = a.H, W = a.W;
    const int kh = KS ? KS : a.kh, kw = KS ? KS : a.kw;
    const int rh = kh / 2, rw = kw / 2;
    const int i0 = (int)blockIdx.y * TH, j0 = (int)blockIdx.x * TW;
    const int tid = (int)threadIdx.x;
    if (!KS)
        for (int idx = tid; idx < kh * kw; idx += BLUR_NT) s_k[idx] = a.k[idx];
    const T* kw_src = KS ? a.k : s_k;
    const int lh = TH + 2 * rh, lw = TW + 2 * rw;
    for (int idx = tid; idx < lh * lw; idx += BLUR_NT) {
        const int li = idx / lw, lj = idx % lw;
        int gi = (i0 - rh + li) % H;
        if (gi < 0) gi += H;
        int gj = (j0 - rw + lj) % W;
        if (gj < 0) gj += W;
        s_x[li][lj] = a.x[(size_t)gi * W + gj];
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < (TW * TH) / BLUR_NT; ++p) {
        const int idx = tid + p * BLUR_NT;
        const int li = idx / TW, lj = idx % TW;
        const int i = i0 + li, j = j0 + lj;
        if (i >= H || j >= W) continue;
        T s = T(0);
        if (!a.adjoint) {
#pragma unroll
            for (int r = 0; r < kh; ++r)
#pragma unroll
                for (int c = 0; c < kw; ++c)
                    s += kw_src[r * kw + c] * s_x[li + 2 * rh - r][lj + 2 * rw - c];
        } else {
#pragma unroll
            for (int r = 0; r < kh; ++r)
#pragma unroll
                for (int c = 0; c < kw; ++c) s += kw_src[r * kw + c] * s_x[li + r][lj + c];
        }
        const size_t g = (size_t)i * W + j;
        if (a.mode == BLUR_STORE) {
            a.out[g] = s;
        } else if (a.mode == BLUR_RESIDUAL) {
            a.out[g] = s - a.b[g];
        } else if (a.mode == BLUR_DUAL_PROX) {
            a.out[g] = (a.out[g] + a.tau * (s - a.b[g])) / (T(1) + a.tau);
        } else {
            s_t[li][lj] = primal_step(a.ps, g, i, j, s);
        }
    }
    if (a.mode == BLUR_PRIMAL && a.ps.pdhg && !a.ps.theta && a.ps.xbarT)
        store_tile_transposed<T, BLUR_NT>(s_t, i0, j0, H, W, a.ps.xbarT, a.ps.xbarT_ld);
}

template <typename T>
static BlurArgs<T> blur_args(const tvs_op* op, bool adjoint) {
    BlurArgs<T> a{};
    a.k = sizeof(T) == 4 ? (const T*)op->blur.k_f : (const T*)op->blur.k_d;
    a.kh = op->blur.kh;
    a.kw = op->blur.kw;
    a.adjoint = adjoint ? 1 : 0;
    a.H = op->H;
    a.W = op->W;
    return a;
}

template <typename T>
static void launch_blur_args(tvs_ctx* ctx, const BlurArgs<T>& a) {
    const dim3 grid(div_up(a.W, 32), div_up(a.H, 32));
    if (a.kh == 9 && a.kw == 9)
        hipLaunchKernelGGL((blur_kernel<T, 9>), grid, dim3(BLUR_NT), 0, ctx->stream, a);
    else
        hipLaunchKernelGGL((blur_kernel<T, 0>), grid, dim3(BLUR_NT), 0, ctx->stream, a);
    TVS_LAUNCH_CHECK();
}

template <typename T>
void launch_blur(tvs_ctx* ctx, const tvs_op* op, bool adjoint, const T* x, const T* b, T* out) {
    BlurArgs<T> a = blur_args<T>(op, adjoint);
    a.x = x;
    a.b = b;
    a.out = out;
    a.mode = b ? BLUR_RESIDUAL : BLUR_STORE;
    launch_blur_args(ctx, a);
}

template <typename T>
void launch_blur_dual_prox(tvs_ctx* ctx, const tvs_op* op, const T* xbar, const T* b, T* y, T tau) {
    BlurArgs<T> a = blur_args<T>(op, false);
    a.x = xbar;
    a.b = b;
    a.out = y;
    a.mode = BLUR_DUAL_PROX;
    a.tau = tau;
    launch_blur_args(ctx, a);
}

template <typename T>
void launch_blur_adjoint_step(tvs_ctx* ctx, const tvs_op* op, const T* r, const PrimalStep<T>& ps) {
    BlurArgs<T> a = blur_args<T>(op, true);
    a.x = r;
    a.mode = BLUR_PRIMAL;
    a.ps = ps;
    launch_blur_args(ctx, a);
}

// ------------------------------------------------------------------ Joseph
// Byte offset 4 * (high word of V) of a float element.  The shift is written
// as one instruction on the 32-bit high word; left to itself the compiler
// forms it as a 64-bit funnel shift and a mask.
__device__ __forceinline__ unsigned fx_byte_offset(long long V) {
    const unsigned hw = (unsigned)((unsigned long long)V >> 32);
    unsigned off;
    __asm__("v_lshlrev_b32 %0, 2, %1" : "=v"(off) : "v"(hw));
    return off;
}

template <typename T>
struct JFwdArgs {
    const JAngle* ang;
    const T* x;    // element (0, 0) of the padded row-major image
    const T* xT;   // element (0, 0) of the padded transposed image
    int x_ld, xT_ld;
    const T* b;
    T* y;
    T* dy;      // FWD_DUAL_PROX_DELTA: y_new - y_old
    int H, W, n_det;
    int epi;
    int small;  // both padded copies span less than 4 GiB
    T tau;
};

template <typename T>
__device__ __forceinline__ void fwd_epilogue(int epi, size_t o, T s, const T* b, T* y, T* dy,
                                             T tau) {
    if (epi == FWD_STORE) {
        y[o] = s;
    } else if (epi == FWD_RESIDUAL) {
        y[o] = s - b[o];
    } else {
        const T yo = y[o];
        const T yn = (yo + tau * (s - b[o])) / (T(1) + tau);
        y[o] = yn;
        if (epi == FWD_DUAL_PROX_DELTA) dy[o] = yn - yo;
    }
}

// Block: 64 adjacent bins of one angle (lane = bin) x SEG wavefronts, each
// summing a contiguous part of the step range; the partial sums are added in
// a fixed order, so the result is deterministic.  Each ray visits only the
// steps whose sample can touch the image (plus at most one step of slack at
// each end, whose samples read the zero pads and add exact zeros).
template <typename T, int SEG>
__global__ __launch_bounds__(64 * SEG) void joseph_fwd_kernel(JFwdArgs<T> a) {
    __shared__ T part[SEG][64];
    const JAngle g = a.ang[blockIdx.y];
    const int lane = (int)threadIdx.x & 63;
    const int seg = (int)threadIdx.x >> 6;
    const int d = (int)blockIdx.x * 64 + lane;
    const int n_step = g.cls ? a.W : a.H;
    const int n_int = g.cls ? a.H : a.W;
    const T* img = g.cls ? a.xT : a.x;
    const int ld = g.cls ? a.xT_ld : a.x_ld;
    const int s0 = (seg * n_step) / SEG, s1 = ((seg + 1) * n_step) / SEG;
    T acc = T(0);
    if (d < a.n_det) {
        const double dd = (double)d;
        int lo = s0, hi = s1;
        // steps whose sample can touch the image: -1 <= u < n_int, u = A d + B s + C
        const double base = fma(g.A, dd, g.C);
        if (g.B != 0.0) {
            double t1 = (-1.0 - base) / g.B, t2 = ((double)n_int - base) / g.B;
            double tmin = t1 < t2 ? t1 : t2, tmax = t1 < t2 ? t2 : t1;
            // clamp both ends into [s0 - 1, s1 + 1] before converting to int
            const double cl = (double)(s0 - 1), ch = (double)(s1 + 1);
            tmin = tmin > cl ? (tmin < ch ? tmin : ch) : cl;
            tmax = tmax < ch ? (tmax > cl ? tmax : cl) : ch;
            const int a_lo = (int)floor(tmin), a_hi = (int)ceil(tmax) + 1;
            lo = a_lo > lo ? a_lo : lo;
            hi = a_hi < hi ? a_hi : hi;
        } else {
            const double u = fma(g.A, dd, fma(g.B, 0.0, g.C));
            if (!(u >= -1.0 && u < (double)n_int)) hi = lo;
        }
        const T* row = img + (size_t)(lo > 0 ? lo : 0) * ld;
        if constexpr (sizeof(T) == 4) {
            // 32.32 fixed point: U = Aq d + Bq s + Cq exactly, floor(u) is the
            // high word and the fraction the low word.  V adds the element
            // offset of row s in the padded buffer (pads included) to the high
            // word, so one 64-bit add per step advances both the sample and
            // the row, and the high word indexes the left neighbour directly.
            // (1 - f) v0 + f v1 is summed as v0 + f (v1 - v0), the two parts in
            // separate accumulators, f (v1 - v0) scaled by 2^32.
            const int s_lo = lo > 0 ? lo : 0;
            long long V = g.Aqi * (long long)d + g.Cqi + g.Bqi * (long long)s_lo +
                          (((long long)s_lo * ld + JPAD) << 32);
            const long long dV = g.Bqi + ((long long)ld << 32);
            const float* base = img - JPAD;
            float acc0 = 0.0f, acc1 = 0.0f;
            if (a.small) {
                // byte offsets of the padded buffer fit 32 bits: the load takes
                // the base in scalar registers and a 32-bit offset, formed
                // from the high word by one shift.  Eight loads are issued
                // before their sums.
                int s = s_lo;
                for (; s + 8 <= hi; s += 8) {
                    float2 v[8];
                    unsigned fr[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        __builtin_memcpy(&v[k], (const char*)base + fx_byte_offset(V), sizeof(float2));
                        fr[k] = (unsigned)V;
                        V += dV;
                        // one induction variable: keeps the compiler from
                        // splitting V into separate high- and low-word chains
                        __asm__("" : "+v"(V));
                    }
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        acc0 += v[k].x;
                        acc1 = fmaf((float)fr[k], v[k].y - v[k].x, acc1);
                    }
                }
                for (; s < hi; ++s) {
                    float2 v;
                    __builtin_memcpy(&v, (const char*)base + fx_byte_offset(V), sizeof(v));
                    acc0 += v.x;
                    acc1 = fmaf((float)(unsigned)V, v.y - v.x, acc1);
                    V += dV;
                }
            } else {
#pragma unroll 8
                for (int s = s_lo; s < hi; ++s) {
                    // both neighbours in one 8-byte load (4-byte aligned, inside
                    // the padded row)
                    float2 v;
                    __builtin_memcpy(&v, base + (size_t)(unsigned)(V >> 32), sizeof(v));
                    acc0 += v.x;
                    acc1 = fmaf((float)(unsigned)V, v.y - v.x, acc1);
                    V += dV;
                }
            }
            acc = acc0 + acc1 * 2.3283064365386963e-10f;
        } else {
#pragma unroll 4
            for (int s = lo; s < hi; ++s) {
                const double u = fma(g.A, dd, fma(g.B, (double)s, g.C));
                const double fl = floor(u);
                const T f = (T)(u - fl);
                const int j0 = (int)fl;
                const T v0 = row[j0], v1 = row[j0 + 1];
                acc += (T(1) - f) * v0;
                acc += f * v1;
                row += ld;
            }
        }
    }
    part[seg][lane] = acc;
    __syncthreads();
    if (seg == 0 && d < a.n_det) {
        T s = part[0][lane];
#pragma unroll
        for (int k = 1; k < SEG; ++k) s += part[k][lane];
        s *= (T)g.wgt;
        const size_t o = (size_t)blockIdx.y * a.n_det + d;
        fwd_epilogue<T>(a.epi, o, s, a.b, a.y, a.dy, a.tau);
    }
}

// Paired-ray projector (float32, padded copies within 4 GiB, 1 <= |A| < 2).
// Lane l of a block takes the adjacent bins d = 2 l and d + 1 of one angle:
// their samples are 1 to 2 pixels apart along the interpolation axis, so one
// 16-byte gather of four consecutive pixels from the floor of the smaller
// sample position holds both rays' neighbour pairs.
// Half as many vector-memory instructions as one ray per lane (the texture
// unit handles a quarter-wave per clock whatever the width), the same
// arithmetic per ray in the same order, so the sums equal
// joseph_fwd_kernel's bit for bit.  The gather start is clamped into the
// padded row [-JPAD, n_int], so every load stays inside the copy.
// med3(x, lo, hi) in one instruction (lo <= hi is the caller's to ensure;
// the compiler emits a min and a max when it cannot prove it)
__device__ __forceinline__ int clamp_med3(int x, int lo, int hi) {
    int r;
    __asm__("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "s"(hi));
    return r;
}

// base + 4 x in one instruction (left to itself the compiler refactors the
// sum around the row base and spends two)
__device__ __forceinline__ unsigned byte_off4(int x, unsigned base) {
    unsigned r;
    __asm__("v_lshl_add_u32 %0, %1, 2, %2" : "=v"(r) : "v"(x), "v"(base));
    return r;
}

// The steps of one pair of rays, tracked by the left one: UL its 32.32
// position, the right ray at UL + D (D = |bin step| in [2^32, 2^33)), so the
// right ray's fraction is the low word of UL plus that of D, and its pixel
// pair starts 1 pixel further, or 2 when that addition carries.  Both
// advance by dB per step.  rb: the lane's first row in bytes from img0 (pads
// included); row k of the walk is rb + k ld4 bytes, k ld4 the same for every
// lane.
__device__ __forceinline__ void pair_walk(const char* img0, long long UL, unsigned Dlo,
                                          long long dB, int rb, int ld4, int n_int, int n,
                                          float& accL0, float& accL1, float& accR0,
                                          float& accR1) {
    int k = 0;
    // four gathers in flight before their sums
    for (; k + 4 <= n; k += 4) {
        float4 p[4];
        unsigned fl[4], fr[4];
        bool two[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            // gather start clamped into the padded row [-JPAD, n_int]
            const int h = (int)(UL >> 32);
            const int cc = clamp_med3(h, -JPAD, n_int);  // n_int >= 1 > -JPAD
            const char* row = img0 + (size_t)(k + u) * ld4;
            __builtin_memcpy(&p[u], row + byte_off4(cc, (unsigned)rb), sizeof(float4));
            fl[u] = (unsigned)UL;
            fr[u] = fl[u] + Dlo;
            two[u] = fr[u] < fl[u];  // the carry: right pair 2 pixels further
            UL += dB;
            // one induction variable (the compiler would otherwise keep a copy
            // of the position per unrolled step)
            __asm__("" : "+v"(UL));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float q0 = two[u] ? p[u].z : p[u].y, q1 = two[u] ? p[u].w : p[u].z;
            accL0 += p[u].x;
            accL1 = fmaf((float)fl[u], p[u].y - p[u].x, accL1);
            accR0 += q0;
            accR1 = fmaf((float)fr[u], q1 - q0, accR1);
        }
    }
    for (; k < n; ++k) {
        const int h = (int)(UL >> 32);
        const int cc = clamp_med3(h, -JPAD, n_int);  // n_int >= 1 > -JPAD
        const char* row = img0 + (size_t)k * ld4;
        float4 p;
        __builtin_memcpy(&p, row + byte_off4(cc, (unsigned)rb), sizeof(float4));
        const unsigned fl = (unsigned)UL, fr = fl + Dlo;
        const bool two = fr < fl;
        const float q0 = two ? p.z : p.y, q1 = two ? p.w : p.z;
        accL0 += p.x;
        accL1 = fmaf((float)fl, p.y - p.x, accL1);
        accR0 += q0;
        accR1 = fmaf((float)fr, q1 - q0, accR1);
        UL += dB;
    }
}

template <int SEG>
__global__ __launch_bounds__(64 * SEG) void joseph_fwd_pair_kernel(JFwdArgs<float> a) {
    __shared__ float part[SEG][128];
    const JAngle g = a.ang[blockIdx.y];
    const int lane = (int)threadIdx.x & 63;
    const int seg = (int)threadIdx.x >> 6;
    const int d0 = (int)blockIdx.x * 128 + 2 * lane;
    const int n_step = g.cls ? a.W : a.H;
    const int n_int = g.cls ? a.H : a.W;
    const float* img = g.cls ? a.xT : a.x;
    const int ld = g.cls ? a.xT_ld : a.x_ld;
    const int s0 = (seg * n_step) / SEG, s1 = ((seg + 1) * n_step) / SEG;
    const bool neg = g.A < 0.0;  // wave-uniform: which ray of the pair lies left
    float acc0a = 0.0f, acc1a = 0.0f, acc0b = 0.0f, acc1b = 0.0f;
    int lo = s1, hi = s0;  // no steps for lanes past the detector
    if (d0 < a.n_det) {
        // steps where either ray's sample can touch the image: with
        // u_a = A d0 + B s + C and u_b = u_a + A, the union of -1 <= u < n_int
        // over both is -1 - max(A, 0) <= u_a < n_int - min(A, 0)
        const double base = fma(g.A, (double)d0, g.C);
        const double ulo = -1.0 - (g.A > 0.0 ? g.A : 0.0), uhi = (double)n_int - (g.A < 0.0 ? g.A : 0.0);
        lo = s0;
        hi = s1;
        if (g.B != 0.0) {
            double t1 = (ulo - base) / g.B, t2 = (uhi - base) / g.B;
            double tmin = t1 < t2 ? t1 : t2, tmax = t1 < t2 ? t2 : t1;
            const double cl = (double)(s0 - 1), ch = (double)(s1 + 1);
            tmin = tmin > cl ? (tmin < ch ? tmin : ch) : cl;
            tmax = tmax < ch ? (tmax > cl ? tmax : cl) : ch;
            const int a_lo = (int)floor(tmin), a_hi = (int)ceil(tmax) + 1;
            lo = a_lo > lo ? a_lo : lo;
            hi = a_hi < hi ? a_hi : hi;
        } else if (!(base >= ulo && base < uhi)) {
            hi = lo;
        }
    }
    // The wavefront walks the union of its lanes' step ranges, every lane on
    // the same row at each step (its 64 gathers then share a few cache
    // lines).  Outside a lane's own range both of its samples lie outside
    // [-1, n_int), so the gathered pixels are pads and add exact zeros.
    int lo_w = lo, hi_w = hi;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        lo_w = min(lo_w, __shfl_xor(lo_w, o));
        hi_w = max(hi_w, __shfl_xor(hi_w, o));
    }
    lo_w = __builtin_amdgcn_readfirstlane(lo_w);
    hi_w = __builtin_amdgcn_readfirstlane(hi_w);
    if (hi_w > lo_w) {
        const int s_lo = lo_w;  // >= s0 >= 0
        // 32.32 positions of both rays relative to their row; the row's
        // byte offset in the padded copy (pads included) is the same for
        // every lane, and a gather's offset is formed from it and the
        // clamped start in one instruction
        const long long Ua0 = g.Aqi * (long long)d0 + g.Cqi + g.Bqi * (long long)s_lo;
        const char* img0 = (const char*)(img - JPAD);
        const int rb = (s_lo * ld + JPAD) * 4;
        // the left ray: a (A > 0) or b (A < 0)
        const long long UL = neg ? Ua0 + g.Aqi : Ua0;
        const unsigned Dlo = (unsigned)(neg ? -g.Aqi : g.Aqi);
        if (neg)
            pair_walk(img0, UL, Dlo, g.Bqi, rb, ld * 4, n_int, hi_w - s_lo, acc0b, acc1b, acc0a, acc1a);
        else
            pair_walk(img0, UL, Dlo, g.Bqi, rb, ld * 4, n_int, hi_w - s_lo, acc0a, acc1a, acc0b, acc1b);
    }
    part[seg][2 * lane] = acc0a + acc1a * 2.3283064365386963e-10f;
    part[seg][2 * lane + 1] = acc0b + acc1b * 2.3283064365386963e-10f;
    __syncthreads();
    // the block's 128 bins, one per thread of the first two wavefronts
    const int t = (int)threadIdx.x;
    const int d = (int)blockIdx.x * 128 + t;
    if (t < 128 && d < a.n_det) {
        float sum = part[0][t];
#pragma unroll
        for (int k = 1; k < SEG; ++k) sum += part[k][t];
        sum *= (float)g.wgt;
        fwd_epilogue<float>(a.epi, (size_t)blockIdx.y * a.n_det + d, sum, a.b, a.y, a.dy, a.tau);
    }
}

template <typename T>
void launch_joseph_fwd(tvs_ctx* ctx, const tvs_op* op, const T* x, const T* xT, const T* b, T* y,
                       int epi, T tau, T* dy) {
    JFwdArgs<T> a;
    a.ang = op->joseph.ang;
    a.x = x;
    a.xT = xT;
    a.x_ld = op->W + 2 * JPAD;
    a.xT_ld = op->H + 2 * JPAD;
    a.b = b;
    a.y = y;
    a.dy = dy;
    a.H = op->H;
    a.W = op->W;
    a.n_det = op->joseph.n_det;
    a.epi = epi;
    a.tau = tau;
    a.small = (size_t)op->H * a.x_ld * sizeof(T) < (1ull << 32) &&
              (size_t)op->W * a.xT_ld * sizeof(T) < (1ull << 32);
    if constexpr (sizeof(T) == 4) {
        if (a.small && op->joseph.pair_ok) {
            hipLaunchKernelGGL((joseph_fwd_pair_kernel<8>), dim3(div_up(a.n_det, 128), op->joseph.n_ang),
                               dim3(512), 0, ctx->stream, a);
            TVS_LAUNCH_CHECK();
            return;
        }
    }
    dim3 grid(div_up(a.n_det, 64), op->joseph.n_ang);
    hipLaunchKernelGGL((joseph_fwd_kernel<T, 8>), grid, dim3(512), 0, ctx->stream, a);
    TVS_LAUNCH_CHECK();
}

// Both zero-padded copies of x (row-major and transposed), pads included.
// 32 x 32 tiles through LDS; the pad columns are written by the edge tiles.
template <typename T>
__global__ __launch_bounds__(TILE_NT) void pad_copy_kernel(int H, int W, const T* x, T* xp, T* xTp) {
    __shared__ T t[32][33];
    const int i0 = (int)blockIdx.y * 32, j0 = (int)blockIdx.x * 32;
    const int ld = W + 2 * JPAD, ldT = H + 2 * JPAD;
    for (int p = 0; p < 1024 / TILE_NT; ++p) {
        const int idx = (int)threadIdx.x + p * TILE_NT;
        const int li = idx / 32, lj = idx % 32;
        const int i = i0 + li, j = j0 + lj;
        if (i < H && j < W) {
            const T v = x[(size_t)i * W + j];
            t[li][lj] = v;
            xp[(size_t)i * ld + j] = v;
        }
    }
    // pads of the row-major copy: columns -JPAD..-1 and W..W+JPAD-1 of rows i
    if (blockIdx.x == 0) {
        for (int idx = (int)threadIdx.x; idx < 32 * 2 * JPAD; idx += TILE_NT) {
            const int li = idx / (2 * JPAD), k = idx % (2 * JPAD);
            const int i = i0 + li;
            if (i < H) {
                const int col = k < JPAD ? k - JPAD : W + (k - JPAD);
                xp[(size_t)i * ld + col] = T(0);
            }
        }
    }
    __syncthreads();
    for (int p = 0; p < 1024 / TILE_NT; ++p) {
        const int idx = (int)threadIdx.x + p * TILE_NT;
        const int jj = idx / 32, ii = idx % 32;
        if (i0 + ii < H && j0 + jj < W) xTp[(size_t)(j0 + jj) * ldT + i0 + ii] = t[ii][jj];
    }
    // pads of the transposed copy: columns -JPAD..-1 and H..H+JPAD-1 of rows j
    if (blockIdx.y == 0) {
        for (int idx = (int)threadIdx.x; idx < 32 * 2 * JPAD; idx += TILE_NT) {
            const int lj = idx / (2 * JPAD), k = idx % (2 * JPAD);
            const int j = j0 + lj;
            if (j < W) {
                const int col = k < JPAD ? k - JPAD : H + (k - JPAD);
                xTp[(size_t)j * ldT + col] = T(0);
            }
        }
    }
}

template <typename T>
void launch_pad_copy(tvs_ctx* ctx, int H, int W, const T* x, T* xp, T* xTp) {
    hipLaunchKernelGGL((pad_copy_kernel<T>), dim3(div_up(W, 32), div_up(H, 32)), dim3(TILE_NT), 0,
                       ctx->stream, H, W, x, xp, xTp);
    TVS_LAUNCH_CHECK();
}

template <typename T>
struct JAdjArgs {
    const JAngle* ang;
    int n_ang;
    const T* y;
    int H, W, n_det;
    T* x_out;
    PrimalStep<T> ps;
    int has_ps;
    ZAcc<T> za;
    int has_za;
};

// One angle of the backprojector for the thread's 4 pixels, with NC
// candidate rays each: the 4 * NC gathers are issued before any weight is
// formed (clamped indices, masked weights, no branches around loads).
template <typename T, int NC>
__device__ __forceinline__ void bp_angle(const JAngle& g, const T* __restrict__ yrow, int n_det,
                                         int i_base, int j, T (&acc)[4]) {
    int d1[4], t[4];
    double K[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i_base + 8 * r;
        const int s_idx = g.cls ? j : i;
        t[r] = g.cls ? i : j;
        if constexpr (sizeof(T) == 4) {
            K[r] = fma(g.Bq, (double)s_idx, g.Cq);
            const float Kf = (float)K[r] * 2.3283064365386963e-10f;
            d1[r] = (int)floorf(((float)t[r] - Kf) * g.inv_Af - g.half_spanf);
        } else {
            K[r] = fma(g.B, (double)s_idx, g.C);
            d1[r] = (int)floor(((double)t[r] - K[r]) * g.inv_A - g.half_span);
        }
    }
    T yv[4][NC];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int d = d1[r] + c;
            yv[r][c] = yrow[d < 0 ? 0 : (d >= n_det ? n_det - 1 : d)];
        }
    const T wgt = (T)g.wgt;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        T sum = T(0);
        double U = 0.0;
        if constexpr (sizeof(T) == 4) U = fma(g.Aq, (double)d1[r], K[r]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int d = d1[r] + c;
            int jj;
            T f;
            if constexpr (sizeof(T) == 4) {
                float ff;
                fx_split(U, jj, ff);
                f = ff;
                U += g.Aq;
            } else {
                const double u = fma(g.A, (double)d, K[r]);
                const double fl = floor(u);
                f = (T)(u - fl);
                jj = (int)fl;
            }
            T wt = (jj == t[r]) ? (T(1) - f) : ((jj == t[r] - 1) ? f : T(0));
            wt = (d >= 0 && d < n_det) ? wt : T(0);
            sum += wt * yv[r][c];
        }
        acc[r] += wgt * sum;
    }
}

// Pixel-driven transpose of joseph_fwd.  Block: a 32 x 32 pixel tile, 256
// threads, 4 pixels each (rows li, li + 8, li + 16, li + 24).  For every angle
// (uniform across the block) each pixel enumerates the n_cand rays around
// the one whose sample lands on it and accumulates
//   (1 - f) y[a][d]  if the ray's sample at this step has floor(u) == t
//   f y[a][d]        if floor(u) == t - 1
// where t is the pixel's interpolation index and u is recomputed exactly as
// the projector computes it.
template <typename T>
__global__ __launch_bounds__(256) void joseph_adj_kernel(JAdjArgs<T> a) {
    __shared__ T s_t[32][33];
    const int i0 = (int)blockIdx.y * 32, j0 = (int)blockIdx.x * 32;
    const int lj = (int)threadIdx.x & 31, lr = (int)threadIdx.x >> 5;  // lr in [0, 8)
    const int j = j0 + lj;
    T acc[4] = {T(0), T(0), T(0), T(0)};
    const int n_det = a.n_det;
    for (int an = 0; an < a.n_ang; ++an) {
        const JAngle g = a.ang[an];
        const T* yrow = a.y + (size_t)an * n_det;
        switch (g.n_cand) {
            case 2: bp_angle<T, 2>(g, yrow, n_det, i0 + lr, j, acc); break;
            case 3: bp_angle<T, 3>(g, yrow, n_det, i0 + lr, j, acc); break;
            case 4: bp_angle<T, 4>(g, yrow, n_det, i0 + lr, j, acc); break;
            default: {
                const T wgt = (T)g.wgt;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + lr + 8 * r;
                    const int s_idx = g.cls ? j : i;
                    const int t_idx = g.cls ? i : j;
                    T sum = T(0);
                    if constexpr (sizeof(T) == 4) {
                        const double K = fma(g.Bq, (double)s_idx, g.Cq);
                        const float Kf = (float)K * 2.3283064365386963e-10f;
                        const int d1 = (int)floorf(((float)t_idx - Kf) * g.inv_Af - g.half_spanf);
                        double U = fma(g.Aq, (double)d1, K);
                        for (int c = 0; c < g.n_cand; ++c, U += g.Aq) {
                            const int d = d1 + c;
                            if (d >= 0 && d < n_det) {
                                int jj;
                                float f;
                                fx_split(U, jj, f);
                                const T wt = (jj == t_idx) ? (T(1) - f) : ((jj == t_idx - 1) ? f : T(0));
                                sum += wt * yrow[d];
                            }
                        }
                    } else {
                        const double K = fma(g.B, (double)s_idx, g.C);
                        const int d1 = (int)floor(((double)t_idx - K) * g.inv_A - g.half_span);
                        for (int c = 0; c < g.n_cand; ++c) {
                            const int d = d1 + c;
                            if (d >= 0 && d < n_det) {
                                const double u = fma(g.A, (double)d, K);
                                const double fl = floor(u);
                                const T f = (T)(u - fl);
                                const int jj = (int)fl;
                                const T wt = (jj == t_idx) ? (T(1) - f) : ((jj == t_idx - 1) ? f : T(0));
                                sum += wt * yrow[d];
                            }
                        }
                    }
                    acc[r] += wgt * sum;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int li = lr + 8 * r;
        const int i = i0 + li;
        if (i < a.H && j < a.W) {
            const size_t gidx = (size_t)i * a.W + j;
            if (a.has_ps)
                s_t[li][lj] = primal_step(a.ps, gidx, i, j, acc[r]);
            else if (a.has_za)
                z_accumulate(a.za, gidx, acc[r]);
            else
                a.x_out[gidx] = acc[r];
        }
    }
    if (a.has_ps && a.ps.pdhg && !a.ps.theta && a.ps.xbarT) {
        __syncthreads();
        for (int p = 0; p < 4; ++p) {
            const int idx = (int)threadIdx.x + p * 256;
            const int jj = idx / 32, ii = idx % 32;
            if (i0 + ii < a.H && j0 + jj < a.W)
                a.ps.xbarT[(size_t)(j0 + jj) * a.ps.xbarT_ld + i0 + ii] = s_t[ii][jj];
        }
    }
}

// ---------------------------------------------------------------------------
// Ray-driven backprojector for float32 data and detector spacing >= pixel
// (|Aq| >= 2^32: at one step two rays never floor to the same pixel).
//
// Block: a 52 x 52 pixel tile and one group of angles (g, g + G, ...),
// RD_H sets of four wavefronts, set h taking the group's angles h, h + RD_H,
// ...  For a row-stepping angle wavefront w owns tile rows
// 13 w .. 13 w + 12, for a column-stepping angle the same columns.  Per
// (wavefront, angle) the 64 lanes take 64 consecutive rays that include every
// ray reaching the wavefront's strip; a lane keeps its ray, its sinogram value
// and its exact 32.32 position (one 64-bit add per step) for all 13 steps.
// Per step the ray lanes hand their two weights to the pixel lanes of the
// strip's 52 pixels with forward permutes (distinct rays never share a
// destination lane; no LDS memory is involved) and the pixel lanes add them
// into registers.  Row-stepping sums are held per (row, lane = column),
// column-stepping ones per (column, lane = row) and meet through an LDS
// transpose, so every pixel's sum has one fixed order.  Each block writes its
// group's partial image; joseph_adj_sum adds the G partials in order and
// applies the epilogue, so the result is deterministic.
static constexpr int RD_P = 52;     // tile side
static constexpr int RD_L = 13;     // steps (rows or columns) per wavefront
static constexpr int RD_NB = 128;   // staged bins per angle
static constexpr int RD_MAXA = 36;  // at most this many angles per group
static constexpr int RD_H = 2;      // wavefront sets per tile, set h taking angles h, h + RD_H, ...
static constexpr int RD_T = 64 * 4 * RD_H;  // threads per block
static_assert(4 * RD_L == RD_P, "four wavefronts cover the tile");
static_assert(RD_P + 1 < 62, "the lanes past the strip (RD_P, RD_P + 1, 62, 63) are no pixel lanes");

// The ray-driven path applies to an angle when rays are at least a pixel
// apart along the interpolation axis, the rays of a tile fit the staged
// window (span + the margins of rd_window) and the rays of a wavefront's
// strip fit 64 lanes (span + the margins of rd_entry).
bool joseph_rd_angle_ok(const JAngle& e) {
    if (std::fabs(e.Aq) < 4294967296.0) return false;
    const double t = (RD_P + 1) * e.half_span, b = std::fabs(e.B) * e.half_span;
    return t + (RD_P - 1) * b + 6.0 <= RD_NB && t + (RD_L - 1) * b + 4.0 <= 64.0;
}

template <typename T>
struct JAdjRdArgs {
    const JAngle* ang;
    int n_ang, groups;
    const T* y;
    int H, W, n_det;
    T* part;  // [groups][H][W]
};

// real-valued index of the ray whose sample is at u = v at step s
__device__ __forceinline__ double rd_ray_at(const JAngle& g, double v, double s) {
    return (v - fma(g.B, s, g.C)) * g.inv_A;
}

// First staged bin of angle g for the tile: three rays before every ray whose
// sample reaches u in [t0 - 1, t0 + RD_P) at one of the tile's steps.
__device__ __forceinline__ int rd_window(const JAngle& g, int i0, int j0) {
    const int s0 = g.cls ? j0 : i0, t0 = g.cls ? i0 : j0;
    const double lo = (double)(t0 - 1), hi = (double)(t0 + RD_P);
    const double e1 = rd_ray_at(g, lo, s0), e2 = rd_ray_at(g, hi, s0);
    const double e3 = rd_ray_at(g, lo, s0 + RD_P - 1), e4 = rd_ray_at(g, hi, s0 + RD_P - 1);
    return (int)floor(fmin(fmin(e1, e2), fmin(e3, e4))) - 3;
}

// Lane window of wavefront w for angle g: its first ray d0 (one before every
// ray that reaches the strip) and the 32.32 position of ray d0 at the strip's
// first step, relative to pixel t0 - 1 of the interpolation axis.
__device__ __forceinline__ void rd_entry(const JAngle& g, int i0, int j0, int w, int& d0,
                                         long long& K) {
    const int s_first = (g.cls ? j0 : i0) + RD_L * w, t0 = g.cls ? i0 : j0;
    const double lo = (double)(t0 - 1), hi = (double)(t0 + RD_P);
    const double e1 = rd_ray_at(g, lo, s_first), e2 = rd_ray_at(g, hi, s_first);
    const double e3 = rd_ray_at(g, lo, s_first + RD_L - 1), e4 = rd_ray_at(g, hi, s_first + RD_L - 1);
    d0 = (int)floor(fmin(fmin(e1, e2), fmin(e3, e4))) - 1;
    K = g.Aqi * (long long)d0 + g.Bqi * (long long)s_first + g.Cqi - ((long long)(t0 - 1) << 32);
}

// A value every lane of the wavefront holds, moved to scalar registers.
__device__ __forceinline__ long long wave_uniform64(long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Permute byte addresses of one step: (1 - f) val goes to pixel lane h - 1,
// f val to pixel lane h, with h the high word of U (h - 1 = -1 wraps to lane
// 63: the permute takes the lane modulo 64).  h is clamped into [-1, RD_P + 1]
// first: a ray outside the strip then pushes to lanes 62 and 63 or RD_P and
// RD_P + 1, none of which is a pixel of the strip, so no range test is needed.
// Returns the address for lane h - 1; lane h's is that + 4, which the
// permute instruction takes as its immediate offset.
__device__ __forceinline__ int rd_dest(long long U) {
    int h = (int)(U >> 32);
    h = h < -1 ? -1 : (h > RD_P + 1 ? RD_P + 1 : h);
    int da = 4 * h - 4;
    // opaque to the optimiser (no instruction), which would otherwise fold
    // da + 4 back into 4 h and compute both addresses
    __asm__("" : "+v"(da));
    return da;
}

// The steps of one angle for one wavefront.  U: the lane's ray position
// relative to pixel t0 - 1 (high word h = pixel index + 1 in the strip, valid
// in [0, RD_P]); val: the ray's weighted sinogram value.  Each step moves the
// ray lanes' two weights to the pixel lanes with forward permutes (lanes no
// ray pushes to receive 0; distinct rays never share a destination) and adds
// them to that step's accumulator.
template <bool FULL>
__device__ __forceinline__ void rd_angle(int lane, int n_s, long long U, long long dU, float val,
                                         float (&acc)[RD_L]) {
    const float vs = val * 2.3283064365386963e-10f;  // val 2^-32, exact
#pragma unroll
    for (int k = 0; k < RD_L; ++k) {
        if (FULL || k < n_s) {
            // the projector's weights, rounded as the projector rounds them,
            // so the two operators are transposes bit for bit
            // (1 - f = fl(1 - fr 2^-32), f val = fl(fr (val 2^-32)), fr the
            // float fraction word: the same roundings in fewer operations)
            const float fr = (float)(unsigned)U;
            const int da = rd_dest(U);
            const float wa = fmaf(fr, -2.3283064365386963e-10f, 1.0f) * val, wb = fr * vs;
            const float ra = __int_as_float(__builtin_amdgcn_ds_permute(da, __float_as_int(wa)));
            const float rb = __int_as_float(__builtin_amdgcn_ds_permute(da + 4, __float_as_int(wb)));
            acc[k] += ra + rb;
            U += dU;
        }
    }
}

// One angle of the block's group as the wavefronts read it: the lane-0 ray
// position of each wavefront's strip (rd_entry) and its first ray's offset
// in the staged window, the bin and step increments, and the angle's row of
// the staged sinogram.  The records of a wavefront set are listed per class
// in the order of the group's angles.
struct RdRec {
    long long K[4];
    long long A, B;  // 32.32 increments per bin and per step
    int bo[4];       // first ray of wavefront w minus the window start
    int m;           // row of yS
    int pad;
};

// All angles of one class of the wavefront set for wavefront w (FULL: the
// strip has all RD_L steps, decided once for the loop so that the
// accumulators stay in place from one angle to the next).  The next angle's
// record and sinogram value are read while the current angle's steps run.
template <bool FULL>
__device__ __forceinline__ void rd_class(const RdRec* rec, int cnt, const float (*yS)[RD_NB],
                                         int w, int lane, int n_s, float (&acc)[RD_L]) {
    if (n_s <= 0 || cnt <= 0) return;
    auto fetch = [&](int k, long long& K, long long& A, long long& B, float& val) {
        const RdRec& r = rec[k];
        K = r.K[w];
        A = r.A;
        B = r.B;
        int bi = r.bo[w] + lane;
        bi = bi < 0 ? 0 : (bi > RD_NB - 1 ? RD_NB - 1 : bi);
        val = yS[r.m][bi];
    };
    long long K, A, B;
    float val;
    fetch(0, K, A, B, val);
    for (int k = 0; k < cnt; ++k) {
        long long Kn = K, An = A, Bn = B;
        float valn = val;
        if (k + 1 < cnt) fetch(k + 1, Kn, An, Bn, valn);
        rd_angle<FULL>(lane, n_s, K + A * (long long)lane, B, val, acc);
        K = Kn;
        A = An;
        B = Bn;
        val = valn;
    }
}

__global__ __launch_bounds__(RD_T) void joseph_adj_rd_kernel(JAdjRdArgs<float> a) {
    // the staged sinogram windows and, once every angle is done, the two
    // transposition tiles share one buffer
    __shared__ union {
        float yS[RD_MAXA][RD_NB];
        struct {
            float tileT[RD_P][RD_P + 1];
            float rowS[RD_P][RD_P + 1];
        } t;
    } sm;
    float (*yS)[RD_NB] = sm.yS;
    float (*tileT)[RD_P + 1] = sm.t.tileT;
    float (*rowS)[RD_P + 1] = sm.t.rowS;
    __shared__ int wst[RD_MAXA];
    __shared__ float wgtS[RD_MAXA];
    __shared__ int lpos[RD_MAXA];        // an angle's place in its (set, class) list
    __shared__ int lcnt[RD_H][2];        // list lengths
    constexpr int RD_PER = (RD_MAXA + RD_H - 1) / RD_H;  // angles per set
    __shared__ RdRec rec[RD_H][2][RD_PER];
    // block -> (angle group, tile), each XCD taking a contiguous range so that
    // the blocks sharing a group's sinogram rows share one L2
    const int tiles_x = div_up(a.W, RD_P), tiles = tiles_x * div_up(a.H, RD_P);
    const int L = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int G = a.groups, g = L / tiles, tl = L - (L / tiles) * tiles;
    const int i0 = (tl / tiles_x) * RD_P, j0 = (tl % tiles_x) * RD_P;
    const int tid = (int)threadIdx.x, lane = tid & 63;
    // wavefront -> (angle set hf, band of RD_L rows / columns w)
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int w = wv & 3, hf = wv >> 2;
    const int na_g = (a.n_ang - g + G - 1) / G;
    if (tid < 64) {
        // wavefront 0, lane m = the group's angle m: window start, weight and
        // the angle's place among the same set's angles of its class
        const bool on = tid < na_g;
        int cls = 0;
        if (on) {
            const JAngle& gg = a.ang[g + tid * G];
            wst[tid] = rd_window(gg, i0, j0);
            wgtS[tid] = (float)gg.wgt;
            cls = gg.cls;
        }
        const unsigned long long below = (1ull << tid) - 1ull;
#pragma unroll
        for (int h = 0; h < RD_H; ++h)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const unsigned long long mk = __ballot(on && tid % RD_H == h && cls == c);
                if (on && tid % RD_H == h && cls == c) lpos[tid] = __popcll(mk & below);
                if (tid == 0) lcnt[h][c] = __popcll(mk);
            }
    }
    __syncthreads();
    if (tid < 4 * na_g) {
        const int m = tid >> 2, ww = tid & 3;
        const JAngle& gg = a.ang[g + m * G];
        RdRec& r = rec[m % RD_H][gg.cls][lpos[m]];
        int d0;
        long long K;
        rd_entry(gg, i0, j0, ww, d0, K);
        r.K[ww] = K;
        r.bo[ww] = d0 - wst[m];
        if (ww == 0) {
            r.A = gg.Aqi;
            r.B = gg.Bqi;
            r.m = m;
        }
    }
    __syncthreads();
    // the group's sinogram windows, RD_MAXA * RD_NB / RD_T loads per thread
    // issued together (a loop over the runtime count would wait for each)
    {
        constexpr int NL = (RD_MAXA * RD_NB + RD_T - 1) / RD_T;
        float v[NL];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int idx = tid + RD_T * r;
            const int m = idx / RD_NB, bb = idx - m * RD_NB;
            const int d = m < na_g ? wst[m] + bb : -1;
            v[r] = (d >= 0 && d < a.n_det) ? a.y[(size_t)(g + m * G) * a.n_det + d] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int idx = tid + RD_T * r;
            const int m = idx / RD_NB, bb = idx - m * RD_NB;
            if (m < na_g) yS[m][bb] = wgtS[m] * v[r];
        }
    }
    __syncthreads();
    float accR[RD_L], accC[RD_L];
#pragma unroll
    for (int r = 0; r < RD_L; ++r) accR[r] = accC[r] = 0.0f;
    const int nR = __builtin_amdgcn_readfirstlane(a.H - (i0 + RD_L * w));
    const int nC = __builtin_amdgcn_readfirstlane(a.W - (j0 + RD_L * w));
    const int cR = __builtin_amdgcn_readfirstlane(lcnt[hf][0]);
    const int cC = __builtin_amdgcn_readfirstlane(lcnt[hf][1]);
    if (nR >= RD_L)
        rd_class<true>(rec[hf][0], cR, yS, w, lane, nR, accR);
    else
        rd_class<false>(rec[hf][0], cR, yS, w, lane, nR, accR);
    if (nC >= RD_L)
        rd_class<true>(rec[hf][1], cC, yS, w, lane, nC, accC);
    else
        rd_class<false>(rec[hf][1], cC, yS, w, lane, nC, accC);
    __syncthreads();  // every wavefront is done with yS, which tileT and rowS overlay
    // Column-stepping sums are held per (column = 13 w + k, row = lane) and
    // are transposed through tileT.  The last set stores both its sums, the
    // sets before it add theirs in place in descending order, and set 0 adds
    // its column sums and writes the tile: a fixed order per pixel.
    if (hf == RD_H - 1 && lane < RD_P) {
#pragma unroll
        for (int k = 0; k < RD_L; ++k) {
            tileT[lane][RD_L * w + k] = accC[k];
            rowS[RD_L * w + k][lane] = accR[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int hs = RD_H - 2; hs >= 1; --hs) {
        if (hf == hs && lane < RD_P) {
#pragma unroll
            for (int k = 0; k < RD_L; ++k) {
                tileT[lane][RD_L * w + k] += accC[k];
                rowS[RD_L * w + k][lane] += accR[k];
            }
        }
        __syncthreads();
    }
    if (hf == 0 && lane < RD_P) {
#pragma unroll
        for (int k = 0; k < RD_L; ++k) tileT[lane][RD_L * w + k] += accC[k];
    }
    __syncthreads();
    if (hf != 0) return;
    const size_t plane = (size_t)a.H * a.W;
#pragma unroll
    for (int k = 0; k < RD_L; ++k) {
        const int i = i0 + RD_L * w + k, j = j0 + lane;
        if (lane < RD_P && i < a.H && j < a.W)
            a.part[(size_t)g * plane + (size_t)i * a.W + j] =
                accR[k] + rowS[RD_L * w + k][lane] + tileT[RD_L * w + k][lane];
    }
}

// Sums the G partial images in order and applies the backprojector epilogue
// (store, or the data step with the transposed xbar copy).  32 x 32 tiles.
template <typename T>
__global__ __launch_bounds__(1024) void joseph_adj_sum_kernel(const T* part, int G, int H, int W,
                                                              T* x_out, PrimalStep<T> ps, int has_ps,
                                                              ZAcc<T> za, int has_za) {
    // one thread per pixel of a 32 x 32 tile: 16 waves per block keep the
    // G independent partial loads of many pixels in flight
    __shared__ T s_t[32][33];
    const int i0 = (int)blockIdx.y * 32, j0 = (int)blockIdx.x * 32;
    const size_t plane = (size_t)H * W;
    const int li = (int)threadIdx.x / 32, lj = (int)threadIdx.x % 32;
    const int i = i0 + li, j = j0 + lj;
    if (i < H && j < W) {
        const size_t gi = (size_t)i * W + j;
        // the data step's own operands are loaded with the partials, so that
        // all of them are in flight together
        T xo = T(0), ho = T(0);
        if (has_ps) {
            xo = ps.x[gi];
            ho = ps.h[gi];
        }
        T s = part[gi];
        // partials 1 .. G-1 in order, eight loads in flight at a time (a
        // plain loop over the runtime G waits for each load before the
        // next); indices clamped to the last partial, so no branch guards a
        // load, and only the partials below G are added
        for (int k = 1; k < G; k += 8) {
            T v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = part[(size_t)(k + u < G ? k + u : G - 1) * plane + gi];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k + u < G) s += v[u];
        }
        if (has_ps)
            s_t[li][lj] = primal_step_xh(ps, gi, i, j, s, xo, ho);
        else if (has_za)
            z_accumulate(za, gi, s);
        else
            x_out[gi] = s;
    }
    if (has_ps && ps.pdhg && !ps.theta && ps.xbarT)
        store_tile_transposed<T, 1024>(s_t, i0, j0, H, W, ps.xbarT, ps.xbarT_ld);
}

int joseph_rd_max_angles() { return RD_MAXA; }

// Angle groups of the ray-driven backprojector (one block per tile and
// group), chosen once per operator unless set by tvs_op_joseph_set_groups.
int joseph_rd_groups(const tvs_ctx* ctx, const tvs_op* op) {
    const JosephGeom& jg = op->joseph;
    if (jg.rd_groups > 0) return jg.rd_groups;
    // All blocks are resident at once, so the slowest compute unit sets the
    // time: it runs ceil(tiles G / n_cu) blocks of ceil(n_ang / G) angles.
    // Take the G with the least such load (the smallest on ties: fewer
    // partial images to sum), with at most RD_MAXA angles per group.
    const long long tiles = (long long)div_up(op->W, RD_P) * div_up(op->H, RD_P);
    const long long ncu = ctx->n_cu > 0 ? ctx->n_cu : 256;
    const int na = jg.n_ang;
    int best_g = na;
    long long best = -1;
    for (int G = div_up(na, RD_MAXA); G <= na; ++G) {
        const long long load = ((tiles * G + ncu - 1) / ncu) * div_up(na, G);
        if (best < 0 || load < best) {
            best = load;
            best_g = G;
        }
        if ((tiles * G + ncu - 1) / ncu > 4 * ((tiles * div_up(na, RD_MAXA) + ncu - 1) / ncu) + 8)
            break;  // far past the point where more groups can help
    }
    jg.rd_groups = best_g;
    return best_g;
}

template <typename T>
void launch_joseph_adj(tvs_ctx* ctx, const tvs_op* op, const T* y, T* x_out,
                       const PrimalStep<T>* ps, const ZAcc<T>* za) {
    JAdjArgs<T> a{};
    a.ang = op->joseph.ang;
    a.n_ang = op->joseph.n_ang;
    a.y = y;
    a.H = op->H;
    a.W = op->W;
    a.n_det = op->joseph.n_det;
    a.x_out = x_out;
    if (ps) {
        a.ps = *ps;
        a.has_ps = 1;
    } else if (za) {
        a.za = *za;
        a.has_za = 1;
    }
    if constexpr (sizeof(T) == 4) {
        if (op->joseph.rd_ok) {
            const int tiles = div_up(a.W, RD_P) * div_up(a.H, RD_P);
            const int G = joseph_rd_groups(ctx, op);
            const size_t plane = (size_t)a.H * a.W;
            T* part = (T*)scratch(ctx, S_PARTIMG, (size_t)G * plane * sizeof(T));
            JAdjRdArgs<float> r;
            r.ang = a.ang;
            r.n_ang = a.n_ang;
            r.groups = G;
            r.y = y;
            r.H = a.H;
            r.W = a.W;
            r.n_det = a.n_det;
            r.part = part;
            hipLaunchKernelGGL(joseph_adj_rd_kernel, dim3(tiles * G), dim3(RD_T), 0, ctx->stream, r);
            TVS_LAUNCH_CHECK();
            hipLaunchKernelGGL((joseph_adj_sum_kernel<T>), dim3(div_up(a.W, 32), div_up(a.H, 32)),
                               dim3(1024), 0, ctx->stream, (const T*)part, G, a.H, a.W, x_out, a.ps,
                               a.has_ps, a.za, a.has_za);
            TVS_LAUNCH_CHECK();
            return;
        }
    }
    dim3 grid(div_up(a.W, 32), div_up(a.H, 32));
    hipLaunchKernelGGL((joseph_adj_kernel<T>), grid, dim3(256), 0, ctx->stream, a);
    TVS_LAUNCH_CHECK();
}

#define TVS_INST(T)                                                                              \
    template void launch_axpby<T>(tvs_ctx*, size_t, T, const T*, T, const T*, T*);               \
    template void launch_copy<T>(tvs_ctx*, size_t, const T*, T*);                                \
    template void launch_fill<T>(tvs_ctx*, size_t, T, T*);                                       \
    template void launch_transpose<T>(tvs_ctx*, int, int, const T*, T*);                         \
    template void launch_permute_rows<T>(tvs_ctx*, int, int, const int*, const T*, T*, bool);    \
    template void launch_fista_extrap<T>(tvs_ctx*, size_t, const T*, const T*, T, T*);          \
    template void launch_identity_step<T>(tvs_ctx*, int, int, const T*, const PrimalStep<T>&);   \
    template void launch_identity_adj_step<T>(tvs_ctx*, int, int, const T*, const PrimalStep<T>&); \
    template void launch_dual_prox_pointwise<T>(tvs_ctx*, size_t, const T*, const T*, T*, T);    \
    template void launch_blur<T>(tvs_ctx*, const tvs_op*, bool, const T*, const T*, T*);         \
    template void launch_blur_dual_prox<T>(tvs_ctx*, const tvs_op*, const T*, const T*, T*, T);  \
    template void launch_blur_adjoint_step<T>(tvs_ctx*, const tvs_op*, const T*, const PrimalStep<T>&); \
    template void launch_joseph_fwd<T>(tvs_ctx*, const tvs_op*, const T*, const T*, const T*, T*, int, T, T*); \
    template void launch_pad_copy<T>(tvs_ctx*, int, int, const T*, T*, T*);                      \
    template void launch_identity_step_batched<T>(tvs_ctx*, const BSlice<T>*, const int*, int, int, \
                                                  const uint8_t*, const T*, T*, const T*, T*, T*, T); \
    template void launch_joseph_adj<T>(tvs_ctx*, const tvs_op*, const T*, T*, const PrimalStep<T>*, \
                                       const ZAcc<T>*);
TVS_INST(float)
TVS_INST(double)
#undef TVS_INST

}  // namespace tvs
