// Deterministic reductions for objectives and duality gaps (gfx950).
//
// Stage 1: block b owns the fixed index range [b*2048, (b+1)*2048); each of
// its 256 threads accumulates 8 strided terms in float64, the wavefront sums
// with a fixed butterfly of lane shuffles, and the four wavefront sums are
// added in order.  Stage 2: one block adds the per-block partials the same
// way.  The grid depends only on the size, so repeated runs give bitwise
// identical results.
#include "tvs_internal.hpp"

namespace tvs {

static constexpr int RB = 256;
static constexpr int RITEMS = 8;
static constexpr int RCHUNK = RB * RITEMS;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* s_w) {
    v = wave_sum(v);
    const int lane = (int)threadIdx.x & 63, wid = (int)threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_w[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < RB / 64; ++w) t += s_w[w];
    return t;
}

static int nblocks(size_t n) { return (int)((n + RCHUNK - 1) / RCHUNK); }

void reserve_reduce_scratch(tvs_ctx* ctx, size_t n) {
    scratch(ctx, S_PART, (size_t)3 * nblocks(n) * sizeof(double));
    scratch(ctx, S_RED, 8 * sizeof(double));
}

// sum (a - b)^2, or sum a^2 if b is null
template <typename T>
__global__ __launch_bounds__(RB) void sqdiff_stage1(size_t n, const T* a, const T* b, double* part) {
    __shared__ double s_w[RB / 64];
    const size_t base = (size_t)blockIdx.x * RCHUNK + threadIdx.x;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RITEMS; ++k) {
        const size_t g = base + (size_t)k * RB;
        if (g < n) {
            const double d = b ? (double)a[g] - (double)b[g] : (double)a[g];
            acc += d * d;
        }
    }
    const double t = block_sum(acc, s_w);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

template <typename T>
__global__ __launch_bounds__(RB) void dot_stage1(size_t n, const T* a, const T* b, double* part) {
    __shared__ double s_w[RB / 64];
    const size_t base = (size_t)blockIdx.x * RCHUNK + threadIdx.x;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RITEMS; ++k) {
        const size_t g = base + (size_t)k * RB;
        if (g < n) acc += (double)a[g] * (double)b[g];
    }
    const double t = block_sum(acc, s_w);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// isotropic TV(u) = sum |(D_y u, D_x u)|
template <typename T>
__global__ __launch_bounds__(RB) void tv_stage1(int H, int W, const T* u, double* part) {
    __shared__ double s_w[RB / 64];
    const size_t n = (size_t)H * W;
    const size_t base = (size_t)blockIdx.x * RCHUNK + threadIdx.x;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < RITEMS; ++k) {
        const size_t g = base + (size_t)k * RB;
        if (g < n) {
            const int i = (int)(g / W), j = (int)(g % W);
            const double uc = (double)u[g];
            const double dy = (i < H - 1) ? (double)u[g + W] - uc : 0.0;
            const double dx = (j < W - 1) ? (double)u[g + 1] - uc : 0.0;
            acc += sqrt(dy * dy + dx * dx);
        }
    }
    const double t = block_sum(acc, s_w);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// TV-prox duality gap at q with z = P_X(v + div q) given:
//   gap = sum lam |D z| - <D z, q>,  tv = sum |D z|,  fid = sum (z - v)^2
template <typename T>
__global__ __launch_bounds__(RB) void gap_stage1(int H, int W, const T* v, const T* z, const T* q,
                                                 double lam, double* part, int nb) {
    __shared__ double s_w[RB / 64];
    const size_t n = (size_t)H * W;
    const size_t base = (size_t)blockIdx.x * RCHUNK + threadIdx.x;
    double a_gap = 0.0, a_tv = 0.0, a_fid = 0.0;
#pragma unroll
    for (int k = 0; k < RITEMS; ++k) {
        const size_t g = base + (size_t)k * RB;
        if (g < n) {
            const int i = (int)(g / W), j = (int)(g % W);
            const double zc = (double)z[g];
            const double gy = (i < H - 1) ? (double)z[g + W] - zc : 0.0;
            const double gx = (j < W - 1) ? (double)z[g + 1] - zc : 0.0;
            const double nrm = sqrt(gy * gy + gx * gx);
            a_gap += lam * nrm - (gy * (double)q[g] + gx * (double)q[n + g]);
            a_tv += nrm;
            const double dz = zc - (double)v[g];
            a_fid += dz * dz;
        }
    }
    double t = block_sum(a_gap, s_w);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
    t = block_sum(a_tv, s_w);
    if (threadIdx.x == 0) part[nb + blockIdx.x] = t;
    t = block_sum(a_fid, s_w);
    if (threadIdx.x == 0) part[2 * nb + blockIdx.x] = t;
}

// out[blockIdx.x] = sum of part[blockIdx.x * nb ... + nb)
__global__ __launch_bounds__(RB) void sum_stage2(int nb, const double* part, double* out) {
    __shared__ double s_w[RB / 64];
    const double* p = part + (size_t)blockIdx.x * nb;
    double acc = 0.0;
    for (int k = (int)threadIdx.x; k < nb; k += RB) acc += p[k];
    const double t = block_sum(acc, s_w);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

__global__ void combine_kernel(const double* x, double a, const double* y, double b, double* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = a * x[0] + b * y[0];
}

template <typename T>
double* reduce_sq_diff(tvs_ctx* ctx, size_t n, const T* a, const T* b, double* out_dev) {
    const int nb = nblocks(n);
    double* part = (double*)scratch(ctx, S_PART, (size_t)nb * sizeof(double));
    hipLaunchKernelGGL((sqdiff_stage1<T>), dim3(nb), dim3(RB), 0, ctx->stream, n, a, b, part);
    TVS_LAUNCH_CHECK();
    hipLaunchKernelGGL(sum_stage2, dim3(1), dim3(RB), 0, ctx->stream, nb, part, out_dev);
    TVS_LAUNCH_CHECK();
    return out_dev;
}

template <typename T>
double* reduce_dot(tvs_ctx* ctx, size_t n, const T* a, const T* b, double* out_dev) {
    const int nb = nblocks(n);
    double* part = (double*)scratch(ctx, S_PART, (size_t)nb * sizeof(double));
    hipLaunchKernelGGL((dot_stage1<T>), dim3(nb), dim3(RB), 0, ctx->stream, n, a, b, part);
    TVS_LAUNCH_CHECK();
    hipLaunchKernelGGL(sum_stage2, dim3(1), dim3(RB), 0, ctx->stream, nb, part, out_dev);
    TVS_LAUNCH_CHECK();
    return out_dev;
}

template <typename T>
double* reduce_tv(tvs_ctx* ctx, int H, int W, const T* u, double* out_dev) {
    const int nb = nblocks((size_t)H * W);
    double* part = (double*)scratch(ctx, S_PART, (size_t)nb * sizeof(double));
    hipLaunchKernelGGL((tv_stage1<T>), dim3(nb), dim3(RB), 0, ctx->stream, H, W, u, part);
    TVS_LAUNCH_CHECK();
    hipLaunchKernelGGL(sum_stage2, dim3(1), dim3(RB), 0, ctx->stream, nb, part, out_dev);
    TVS_LAUNCH_CHECK();
    return out_dev;
}

// gap_dev[0] = gap, primal_dev[0] = 1/2 fid + lam tv  (primal_dev may equal gap_dev + 1)
template <typename T>
void reduce_gap(tvs_ctx* ctx, int H, int W, const T* v, const T* z, const T* q, double lam,
                double* gap_dev, double* primal_dev) {
    const int nb = nblocks((size_t)H * W);
    double* part = (double*)scratch(ctx, S_PART, (size_t)3 * nb * sizeof(double));
    double* sums = (double*)scratch(ctx, S_RED, 8 * sizeof(double));
    hipLaunchKernelGGL((gap_stage1<T>), dim3(nb), dim3(RB), 0, ctx->stream, H, W, v, z, q, lam,
                       part, nb);
    TVS_LAUNCH_CHECK();
    hipLaunchKernelGGL(sum_stage2, dim3(3), dim3(RB), 0, ctx->stream, nb, part, sums + 4);
    TVS_LAUNCH_CHECK();
    // sums[4] = gap, sums[5] = tv, sums[6] = fid
    hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(1), 0, ctx->stream, sums + 4, 1.0, sums + 4,
                       0.0, gap_dev);
    TVS_LAUNCH_CHECK();
    hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(1), 0, ctx->stream, sums + 6, 0.5, sums + 5,
                       lam, primal_dev);
    TVS_LAUNCH_CHECK();
}

void launch_combine(tvs_ctx* ctx, const double* x, double a, const double* y, double b,
                    double* out) {
    hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(1), 0, ctx->stream, x, a, y, b, out);
    TVS_LAUNCH_CHECK();
}

#define TVS_INST(T)                                                                       \
    template double* reduce_sq_diff<T>(tvs_ctx*, size_t, const T*, const T*, double*);    \
    template double* reduce_dot<T>(tvs_ctx*, size_t, const T*, const T*, double*);        \
    template double* reduce_tv<T>(tvs_ctx*, int, int, const T*, double*);                 \
    template void reduce_gap<T>(tvs_ctx*, int, int, const T*, const T*, const T*, double, \
                                double*, double*);
TVS_INST(float)
TVS_INST(double)
#undef TVS_INST

}  // namespace tvs
