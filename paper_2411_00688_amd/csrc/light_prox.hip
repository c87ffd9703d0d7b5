// ProxSkip on the light-prox problems of Sec. 2.1-2.2: the dual of TV
// denoising (Dual-ROF) and, with eps > 0, the Dual-Huber-ROF of Sec. 2.2,
//
//   min_{|q_i| <= alpha}  F(q) = 1/2 |div q + b|^2 + eps / (2 alpha) |q|^2,
//
// grad F(q) = -D(div q + b) + mu q with mu = eps / alpha, and the prox of the
// indicator of the alpha-ball set is the projection of eq. (7).  One
// ProxSkip step (Alg. "ProxSkip"): w = q - gamma grad F(q), qhat = w + gamma h;
// with probability p: q+ = P(w + (gamma - gamma / p) h), h += (p / gamma)(q+ -
// qhat); else q+ = qhat.
//
// With the constraint z >= 0 (the TV prox of a non-negative image) the dual
// is the constrained one of Beck and Teboulle 2009: grad F(q) = -D P_+(b +
// div q), with eps = 0; the kernel clips z before its differences.
//
// The kernel fuses TS steps per launch on a tile with a TS-pixel halo (each
// step widens the dependency cone by one pixel), the state (q, h) of every
// pixel of the tile region in registers and q and z = div q + b exchanged
// through LDS.  The coin of the fused steps comes in as a bit mask (bit s =
// theta of the launch's step s), known on the host before anything runs.
#include <cmath>
#include <type_traits>
#include <vector>

#include "tvs_internal.hpp"

namespace tvs {

template <typename T>
__device__ __forceinline__ T lp_ball_scale(T wy, T wx, T lam);
template <>
__device__ __forceinline__ float lp_ball_scale<float>(float wy, float wx, float lam) {
    float n2 = wy * wy + wx * wx;
    return (n2 > lam * lam) ? lam * __builtin_amdgcn_rsqf(fmaxf(n2, 1e-37f)) : 1.0f;
}
template <>
__device__ __forceinline__ double lp_ball_scale<double>(double wy, double wx, double lam) {
    double nrm = sqrt(wy * wy + wx * wx);
    return (nrm > lam) ? lam / nrm : 1.0;
}

template <typename T>
struct LpArgs {
    const T* b;
    const T* q;   // in  [2][H][W]
    const T* h;
    T* qo;        // out
    T* ho;
    int H, W;
    size_t plane;
    int nsteps;
    unsigned theta;  // bit s: prox at step s of this launch
    int nonneg;      // z = max(b + div q, 0) (eps = 0 only)
    T alpha, gamma, mu, coef, rate;
};

enum : int { LF_IN = 1, LF_DY = 2, LF_UP = 4, LF_DX = 8, LF_LEFT = 16, LF_DOWN = 32,
             LF_RIGHT = 64, LF_OUT = 128 };

template <typename T, int BW, int BH, int TS, int NT>
__global__ __launch_bounds__(NT) void dual_rof_tb_kernel(LpArgs<T> a) {
    constexpr int RW = BW + 2 * TS, RH = BH + 2 * TS, R = RW * RH;
    constexpr int PPT = (R + NT - 1) / NT;
    // one guard row before and after each array (read by the flag-free steps)
    __shared__ T s_qy_g[R + 2 * RW];
    __shared__ T s_qx_g[R + 2 * RW];
    __shared__ T s_z_g[R + 2 * RW];
    T* const s_qy = s_qy_g + RW;
    T* const s_qx = s_qx_g + RW;
    T* const s_z = s_z_g + RW;

    const int H = a.H, W = a.W;
    const int gx = div_up(W, BW);
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int i0 = (t / gx) * BH - TS, j0 = (t % gx) * BW - TS;
    const int tid = (int)threadIdx.x;
    // A region that holds neither the image's last row nor its last column
    // steps without flags: away from its edge every pixel has all four
    // neighbours, and its edge pixels (wrong either way) reach only the TS-wide
    // halo within TS steps.
    const bool interior = i0 >= 0 && j0 >= 0 && i0 + RH < H && j0 + RW < W;

    T qy[PPT], qx[PPT], hy[PPT], hx[PPT], bb[PPT], zz[PPT];
    int fl[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int idx = tid + p * NT;
        const int li = idx / RW, lj = idx - (idx / RW) * RW;
        const int i = i0 + li, j = j0 + lj;
        const bool in = idx < R && i >= 0 && i < H && j >= 0 && j < W;
        int f = 0;
        if (in) {
            f |= LF_IN;
            if (i < H - 1) f |= LF_DY;
            if (i > 0 && li > 0) f |= LF_UP;
            if (j < W - 1) f |= LF_DX;
            if (j > 0 && lj > 0) f |= LF_LEFT;
            if (i < H - 1 && li < RH - 1) f |= LF_DOWN;
            if (j < W - 1 && lj < RW - 1) f |= LF_RIGHT;
            if (li >= TS && li < TS + BH && lj >= TS && lj < TS + BW) f |= LF_OUT;
        }
        fl[p] = f;
        const size_t g = in ? (size_t)i * W + j : 0;
        qy[p] = in ? a.q[g] : T(0);
        qx[p] = in ? a.q[a.plane + g] : T(0);
        hy[p] = in ? a.h[g] : T(0);
        hx[p] = in ? a.h[a.plane + g] : T(0);
        bb[p] = in ? a.b[g] : T(0);
    }

    auto steps = [&](auto fast) {
    constexpr bool FAST = decltype(fast)::value;
    for (int s = 0; s < a.nsteps; ++s) {
        const bool prox = (a.theta >> s) & 1u;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int idx = tid + p * NT;
            if (idx < R) {
                s_qy[idx] = qy[p];
                s_qx[idx] = qx[p];
            }
        }
        __syncthreads();
        // z = b + div q  (u = b + div q, Sec. 2.1), the terms in the same
        // order either way
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int idx = tid + p * NT;
            T d;
            if (FAST) {
                // slots past the region (last p only) read in-bounds guard
                // values and store nothing
                d = qy[p];
                d -= s_qy[idx < R ? idx - RW : 0];
                d += qx[p];
                d -= s_qx[idx < R ? idx - 1 : 0];
            } else {
                const int f = fl[p];
                d = T(0);
                if (f & LF_DY) d += qy[p];
                if (f & LF_UP) d -= s_qy[idx - RW];
                if (f & LF_DX) d += qx[p];
                if (f & LF_LEFT) d -= s_qx[idx - 1];
            }
            zz[p] = bb[p] + d;
            if (a.nonneg) zz[p] = zz[p] > T(0) ? zz[p] : T(0);
            if (idx < R) s_z[idx] = zz[p];
        }
        __syncthreads();
        // grad F = -D z + mu q; the ProxSkip step
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int idx = tid + p * NT;
            const int f = fl[p];
            T dy, dx;
            if (FAST) {
                dy = s_z[idx < R ? idx + RW : 0] - zz[p];
                dx = s_z[idx < R ? idx + 1 : 0] - zz[p];
            } else {
                dy = (f & LF_DOWN) ? s_z[idx + RW] - zz[p] : T(0);
                dx = (f & LF_RIGHT) ? s_z[idx + 1] - zz[p] : T(0);
            }
            const T gyv = -dy + a.mu * qy[p];
            const T gxv = -dx + a.mu * qx[p];
            const T wy = qy[p] - a.gamma * gyv, wx = qx[p] - a.gamma * gxv;
            const T hy_ = wy + a.gamma * hy[p], hx_ = wx + a.gamma * hx[p];
            if (prox) {
                const T vy = wy + a.coef * hy[p], vx = wx + a.coef * hx[p];
                const T sc = lp_ball_scale<T>(vy, vx, a.alpha);
                const T ny = vy * sc, nx = vx * sc;
                hy[p] = hy[p] + a.rate * (ny - hy_);
                hx[p] = hx[p] + a.rate * (nx - hx_);
                qy[p] = ny;
                qx[p] = nx;
            } else {
                qy[p] = hy_;
                qx[p] = hx_;
            }
            if (!FAST && !(f & LF_IN)) qy[p] = qx[p] = hy[p] = hx[p] = T(0);
        }
        // No barrier here: the next step writes s_qy / s_qx (last read before
        // this step's second barrier) and writes s_z only after its own first
        // barrier.
    }
    };
    if (interior)
        steps(std::true_type{});
    else
        steps(std::false_type{});

#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        if (fl[p] & LF_OUT) {
            const int idx = tid + p * NT;
            const int li = idx / RW, lj = idx - (idx / RW) * RW;
            const size_t g = (size_t)(i0 + li) * W + (j0 + lj);
            a.qo[g] = qy[p];
            a.qo[a.plane + g] = qx[p];
            a.ho[g] = hy[p];
            a.ho[a.plane + g] = hx[p];
        }
    }
}

template <typename T, int BW, int BH, int TS, int NT>
static void launch_lp(const LpArgs<T>& a, hipStream_t st) {
    const int tiles = div_up(a.W, BW) * div_up(a.H, BH);
    hipLaunchKernelGGL((dual_rof_tb_kernel<T, BW, BH, TS, NT>), dim3(tiles), dim3(NT), 0, st, a);
}

}  // namespace tvs

using namespace tvs;

namespace {

// Large images (at least two 32 x 32 tiles per CU) use 32 x 32 tiles with 6
// steps per launch (40 x 40 regions instead of 48 x 48: the halo
// recomputation, which bounds the kernel, shrinks faster than the extra
// launches' traffic grows); images with one such tile per CU 32 x 32 tiles
// with 8 steps; both with 1024-thread workgroups, so that a CU runs 16 waves
// of one tile.  Smaller images use 16 x 16 tiles with 8 steps and 256
// threads so that the launch still fills the GPU.
constexpr int LP_TS_SMALL = 8, LP_TS_BIG = 6;

// Runs K steps (coins theta[0 .. K)) from (q, h), each launch reading one
// pair of buffers and writing the other; returns true when the result sits
// in (q2, h2).
template <typename T>
bool lp_steps(tvs_ctx* ctx, LpArgs<T> a, int64_t K, const uint8_t* theta, T* q, T* h, T* q2,
              T* h2) {
    const long long t32 = (long long)div_up(a.W, 32) * div_up(a.H, 32);
    const bool big = t32 >= 2LL * ctx->n_cu;
    const bool mid = !big && t32 >= ctx->n_cu;
    const T* qi = q;
    const T* hi = h;
    bool in_caller = true;
    const int ts = big ? LP_TS_BIG : LP_TS_SMALL;
    for (int64_t k = 0; k < K; k += ts) {
        const int ns = (int)std::min<int64_t>(ts, K - k);
        unsigned mask = 0;
        for (int s = 0; s < ns; ++s) mask |= (unsigned)theta[(size_t)(k + s)] << s;
        a.q = qi;
        a.h = hi;
        a.qo = in_caller ? q2 : q;
        a.ho = in_caller ? h2 : h;
        a.nsteps = ns;
        a.theta = mask;
        if (big)
            launch_lp<T, 32, 32, LP_TS_BIG, 1024>(a, ctx->stream);
        else if (mid)
            launch_lp<T, 32, 32, LP_TS_SMALL, 1024>(a, ctx->stream);
        else
            launch_lp<T, 16, 16, LP_TS_SMALL, 256>(a, ctx->stream);
        TVS_LAUNCH_CHECK();
        qi = a.qo;
        hi = a.ho;
        in_caller = !in_caller;
    }
    return !in_caller;
}

template <typename T>
void run_dual_rof(tvs_ctx* ctx, int H, int W, const T* b, T* q, T* h,
                  const tvs_dual_rof_params* P, const std::vector<uint8_t>& theta) {
    const size_t n = (size_t)H * W;
    T* q2 = (T*)scratch(ctx, S_Q1, 2 * n * sizeof(T));
    T* h2 = (T*)scratch(ctx, S_Q2, 2 * n * sizeof(T));
    LpArgs<T> a{};
    a.b = b;
    a.H = H;
    a.W = W;
    a.plane = n;
    a.nonneg = 0;
    a.alpha = (T)P->alpha;
    a.gamma = (T)P->step;
    a.mu = (T)(P->alpha > 0 ? P->eps / P->alpha : 0.0);
    a.coef = (T)(P->step - P->step / P->p);
    a.rate = (T)(P->p / P->step);
    if (lp_steps<T>(ctx, a, P->outer_iters, theta.data(), q, h, q2, h2)) {
        launch_copy<T>(ctx, 2 * n, q2, q);
        launch_copy<T>(ctx, 2 * n, h2, h);
    }
}

template <typename F>
tvs_status guarded_lp(F&& f) {
    try {
        f();
        return TVS_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return TVS_ERR_OOM;
    } catch (...) {
        set_error("unexpected C++ exception");
        return TVS_ERR_DEVICE;
    }
}

}  // namespace

namespace tvs {

template <typename T>
T* run_tv_prox_skip(tvs_ctx* ctx, int H, int W, const T* v, double lam, int nonneg, int iters,
                    double p_in, const uint8_t* theta, T* q, T* h) {
    const size_t n = (size_t)H * W;
    T* q2 = (T*)scratch(ctx, S_Q1, 2 * n * sizeof(T));
    T* h2 = (T*)scratch(ctx, S_Q2, 2 * n * sizeof(T));
    const double gamma = 0.125;
    LpArgs<T> a{};
    a.b = v;
    a.H = H;
    a.W = W;
    a.plane = n;
    a.nonneg = nonneg ? 1 : 0;
    a.alpha = (T)lam;
    a.gamma = (T)gamma;
    a.mu = T(0);
    a.coef = (T)(gamma - gamma / p_in);
    a.rate = (T)(p_in / gamma);
    if (!lp_steps<T>(ctx, a, iters, theta, q, h, q2, h2)) return q;
    launch_copy<T>(ctx, 2 * n, h2, h);
    return q2;
}

template float* run_tv_prox_skip<float>(tvs_ctx*, int, int, const float*, double, int, int,
                                        double, const uint8_t*, float*, float*);
template double* run_tv_prox_skip<double>(tvs_ctx*, int, int, const double*, double, int, int,
                                          double, const uint8_t*, double*, double*);

}  // namespace tvs

extern "C" tvs_status tvs_dual_rof_proxskip(tvs_ctx* ctx, tvs_dtype dtype, int H, int W,
                                            const void* b, void* q, void* h,
                                            const tvs_dual_rof_params* P, uint8_t* theta_trace,
                                            int64_t* n_prox_out) {
    return guarded_lp([&] {
        TVS_REQUIRE(ctx && b && q && h && P, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(dtype == TVS_F32 || dtype == TVS_F64, TVS_ERR_INVALID_ARG, "bad dtype");
        TVS_REQUIRE(H >= 1 && W >= 1 && (long long)H * W <= (1LL << 31), TVS_ERR_SHAPE,
                    "image size out of range");
        TVS_REQUIRE(std::isfinite(P->alpha) && P->alpha >= 0, TVS_ERR_INVALID_ARG,
                    "alpha >= 0 required");
        TVS_REQUIRE(std::isfinite(P->eps) && P->eps >= 0, TVS_ERR_INVALID_ARG, "eps >= 0 required");
        TVS_REQUIRE(std::isfinite(P->step) && P->step > 0, TVS_ERR_INVALID_ARG,
                    "step > 0 required");
        TVS_REQUIRE(P->p > 0 && P->p <= 1, TVS_ERR_INVALID_ARG, "p must be in (0, 1]");
        TVS_REQUIRE(P->outer_iters >= 0 && P->k0 >= 0, TVS_ERR_INVALID_ARG,
                    "outer_iters >= 0 and k0 >= 0 required");
        TVS_HIP(hipSetDevice(ctx->device));
        const int64_t K = P->outer_iters;
        std::vector<uint8_t> theta((size_t)K);
        int64_t nprox = 0;
        for (int64_t kk = 0; kk < K; ++kk) {
            theta[kk] = (uint8_t)coin(P->seed, P->stream_id, P->k0 + kk, P->p);
            nprox += theta[kk];
        }
        const size_t n = (size_t)H * W;
        const size_t bytes = dtype == TVS_F32 ? 4 : 8;
        scratch(ctx, S_Q1, 2 * n * bytes);
        scratch(ctx, S_Q2, 2 * n * bytes);
        auto enqueue = [&] {
            if (dtype == TVS_F32)
                run_dual_rof<float>(ctx, H, W, (const float*)b, (float*)q, (float*)h, P, theta);
            else
                run_dual_rof<double>(ctx, H, W, (const double*)b, (double*)q, (double*)h, P, theta);
        };
        if ((P->flags & TVS_FLAG_GRAPH) && K > 0) {
            uint64_t ab, eb, sb, pb;
            std::memcpy(&ab, &P->alpha, 8);
            std::memcpy(&eb, &P->eps, 8);
            std::memcpy(&sb, &P->step, 8);
            std::memcpy(&pb, &P->p, 8);
            graph_run_key(ctx, {0xD0A1ULL, (uint64_t)dtype, (uint64_t)H, (uint64_t)W,
                                (uint64_t)(uintptr_t)b, (uint64_t)(uintptr_t)q,
                                (uint64_t)(uintptr_t)h, ab, eb, sb, pb, (uint64_t)K, P->seed,
                                P->stream_id, (uint64_t)P->k0},
                          enqueue);
        } else {
            enqueue();
        }
        if (theta_trace && K > 0) std::memcpy(theta_trace, theta.data(), (size_t)K);
        if (n_prox_out) *n_prox_out = nprox;
    });
}
