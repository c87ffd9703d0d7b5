// C ABI of the gfx950 TV-skip library: contexts, operators, the TV prox and
// the ProxSkip / PDHGSkip-2 outer loops.  The loops run on the host and
// enqueue kernels on the context's stream; the coin schedule is a pure
// function of (seed, stream, k), so the host knows it before launching and
// simply does not enqueue the prox on skipped iterations.
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "tvs_internal.hpp"

namespace tvs {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

template <typename F>
static tvs_status guarded(F&& f) {
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

void* scratch(tvs_ctx* ctx, Slot s, size_t bytes) {
    Scratch& sc = ctx->slots[s];
    if (bytes <= sc.bytes && sc.ptr) return sc.ptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TVS_HIP(hipStreamIsCapturing(ctx->stream, &cs));
    TVS_REQUIRE(cs == hipStreamCaptureStatusNone, TVS_ERR_DEVICE,
                "scratch memory would have to grow during graph capture");
    if (sc.ptr) {
        TVS_HIP(hipDeviceSynchronize());
        graph_cache_clear(ctx);  // cached graphs hold the old address
        TVS_HIP(hipFree(sc.ptr));
        sc.ptr = nullptr;
        sc.bytes = 0;
    }
    size_t want = bytes < 256 ? 256 : bytes;
    want = (want + 255) & ~(size_t)255;
    TVS_HIP(hipMalloc(&sc.ptr, want));
    // new scratch starts zeroed (the padded projector inputs rely on zero
    // pads that no kernel writes)
    TVS_HIP(hipMemset(sc.ptr, 0, want));
    TVS_HIP(hipDeviceSynchronize());
    sc.bytes = want;
    return sc.ptr;
}

// ---------------------------------------------------------------- coin
// SplitMix64 (Steele, Lea and Flood 2014) with Stafford's "variant 13" mix.
static constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ULL;

uint64_t splitmix_mix(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

int coin(uint64_t seed, uint64_t stream, int64_t k, double p) {
    if (!(p > 0.0 && p <= 1.0) || k < 0) return -1;
    const uint64_t key = splitmix_mix(seed ^ splitmix_mix(stream + kGolden));
    const uint64_t r = splitmix_mix(key + (uint64_t)(k + 1) * kGolden);
    const uint64_t thresh = (uint64_t)std::floor(std::ldexp(p, 53));
    return (r >> 11) < thresh ? 1 : 0;
}

// Angle subset of the stochastic-angle method at iteration k: the coin's
// generator on stream `stream` xor 2^63, floor((r >> 11) n / 2^53), in
// 64-bit integer arithmetic (exact: r >> 11 < 2^53 and n < 2^10).
int subset_draw(uint64_t seed, uint64_t stream, int64_t k, int n) {
    if (n < 1 || n > 1024 || k < 0) return -1;
    const uint64_t key = splitmix_mix(seed ^ splitmix_mix((stream ^ (1ULL << 63)) + kGolden));
    const uint64_t r = splitmix_mix(key + (uint64_t)(k + 1) * kGolden);
    return (int)(((r >> 11) * (uint64_t)n) >> 53);
}

// ---------------------------------------------------- FGP momentum table
// beta[0] = 0 and beta[k] = (t_{k-1} - 1) / t_k, t_0 = 1,
// t_k = (1 + sqrt(1 + 4 t_{k-1}^2)) / 2, computed once in float64.
const double* beta_table_host(int n) {
    static std::vector<double> tab;
    if ((int)tab.size() < n) {
        tab.assign(n, 0.0);
        double t = 1.0;
        for (int k = 1; k < n; ++k) {
            const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
            tab[k] = (t - 1.0) / tn;
            t = tn;
        }
    }
    return tab.data();
}

template <typename T>
const T* beta_table_dev(tvs_ctx* ctx, int n) {
    const int want = n < 1024 ? 1024 : n;
    Slot s = sizeof(T) == 4 ? S_BETAF : S_BETA;
    if (ctx->beta_len < want || !ctx->slots[S_BETA].ptr || !ctx->slots[S_BETAF].ptr) {
        const double* h = beta_table_host(want);
        std::vector<float> hf(h, h + want);
        void* pd = scratch(ctx, S_BETA, (size_t)want * sizeof(double));
        void* pf = scratch(ctx, S_BETAF, (size_t)want * sizeof(float));
        TVS_HIP(hipMemcpy(pd, h, (size_t)want * sizeof(double), hipMemcpyHostToDevice));
        TVS_HIP(hipMemcpy(pf, hf.data(), (size_t)want * sizeof(float), hipMemcpyHostToDevice));
        ctx->beta_len = want;
    }
    return (const T*)ctx->slots[s].ptr;
}

FgpConfig fgp_config(tvs_ctx* ctx, int H, int W, int dtype_bytes) {
    auto it = ctx->fgp_tuned.find(tune_key(TK_IMAGE, H, W, dtype_bytes));
    if (it != ctx->fgp_tuned.end()) return it->second.cfg;
    it = ctx->fgp_tuned.find(tune_key(TK_CLASS, size_class(H), size_class(W), dtype_bytes));
    if (it != ctx->fgp_tuned.end()) return it->second.cfg;
    FgpConfig c;
    c.tile_w = 32;
    c.tile_h = 32;
    c.steps = 4;
    return c;
}

FgpConfig fgp_config_batched(tvs_ctx* ctx, int n_slices, int dtype_bytes) {
    auto it = ctx->fgp_tuned.find(tune_key(TK_BATCH, n_slices, 0, dtype_bytes));
    if (it != ctx->fgp_tuned.end()) return it->second.cfg;
    // large total sizes favour wide tiles
    FgpConfig c;
    c.tile_w = 64;
    c.tile_h = 16;
    c.steps = 4;
    return c;
}

// ------------------------------------------------------------- validation
static void check_ctx(tvs_ctx* ctx) { TVS_REQUIRE(ctx, TVS_ERR_INVALID_ARG, "null context"); }
static void check_dtype(tvs_dtype d) {
    TVS_REQUIRE(d == TVS_F32 || d == TVS_F64, TVS_ERR_INVALID_ARG, "dtype must be TVS_F32 or TVS_F64");
}
static void check_hw(int H, int W) {
    TVS_REQUIRE(H >= 1 && W >= 1 && (long long)H * W <= (1LL << 31), TVS_ERR_SHAPE,
                "image size out of range");
}
static void use_device(tvs_ctx* ctx) { TVS_HIP(hipSetDevice(ctx->device)); }

}  // namespace tvs

using namespace tvs;

// ================================================================ context
extern "C" tvs_status tvs_ctx_create(int device, void* hip_stream, tvs_ctx** out) {
    return guarded([&] {
        TVS_REQUIRE(out, TVS_ERR_INVALID_ARG, "null output pointer");
        int n = 0;
        TVS_HIP(hipGetDeviceCount(&n));
        TVS_REQUIRE(device >= 0 && device < n, TVS_ERR_INVALID_ARG, "device index out of range");
        TVS_HIP(hipSetDevice(device));
        auto* c = new tvs_ctx();
        c->device = device;
        c->stream = (hipStream_t)hip_stream;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
        try {
            noalloc_setup(device);  // device address of the no-allocation scratch
        } catch (...) {
            delete c;
            throw;
        }
        *out = c;
    });
}

extern "C" void tvs_ctx_destroy(tvs_ctx* ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    graph_cache_clear(ctx);
    for (auto& s : ctx->slots)
        if (s.ptr) hipFree(s.ptr);
    delete ctx;
}

extern "C" tvs_status tvs_ctx_set_stream(tvs_ctx* ctx, void* hip_stream) {
    return guarded([&] {
        check_ctx(ctx);
        ctx->stream = (hipStream_t)hip_stream;
    });
}

extern "C" const char* tvs_last_error(void) { return g_last_error.c_str(); }

extern "C" tvs_status tvs_sync(tvs_ctx* ctx) {
    return guarded([&] {
        check_ctx(ctx);
        use_device(ctx);
        TVS_HIP(hipStreamSynchronize(ctx->stream));
    });
}

// ============================================================== operators
extern "C" tvs_status tvs_op_identity(tvs_ctx* ctx, int H, int W, tvs_op** out) {
    return guarded([&] {
        check_ctx(ctx);
        check_hw(H, W);
        TVS_REQUIRE(out, TVS_ERR_INVALID_ARG, "null output pointer");
        auto* op = new tvs_op();
        op->ctx = ctx;
        op->kind = OP_IDENTITY;
        op->H = H;
        op->W = W;
        *out = op;
    });
}

extern "C" tvs_status tvs_op_blur_periodic(tvs_ctx* ctx, int H, int W, const double* kernel_host,
                                           int kh, int kw, tvs_op** out) {
    return guarded([&] {
        check_ctx(ctx);
        check_hw(H, W);
        TVS_REQUIRE(out && kernel_host, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(kh >= 1 && kw >= 1 && kh % 2 == 1 && kw % 2 == 1 && kh <= 17 && kw <= 17 &&
                        kh <= H && kw <= W,
                    TVS_ERR_SHAPE, "blur kernel must be odd-sized, <= 17 and <= the image");
        use_device(ctx);
        auto op = std::make_unique<tvs_op>();
        op->ctx = ctx;
        op->kind = OP_BLUR;
        op->H = H;
        op->W = W;
        op->blur.kh = kh;
        op->blur.kw = kw;
        const size_t n = (size_t)kh * kw;
        std::vector<float> kf(kernel_host, kernel_host + n);
        TVS_HIP(hipMalloc(&op->blur.k_f, n * sizeof(float)));
        TVS_HIP(hipMalloc(&op->blur.k_d, n * sizeof(double)));
        TVS_HIP(hipMemcpy(op->blur.k_f, kf.data(), n * sizeof(float), hipMemcpyHostToDevice));
        TVS_HIP(hipMemcpy(op->blur.k_d, kernel_host, n * sizeof(double), hipMemcpyHostToDevice));
        *out = op.release();
    });
}

extern "C" tvs_status tvs_op_ct_joseph(tvs_ctx* ctx, int H, int W, int n_ang,
                                       const double* angles_host, int n_det, double pixel,
                                       double det_spacing, tvs_op** out) {
    return guarded([&] {
        check_ctx(ctx);
        check_hw(H, W);
        TVS_REQUIRE(out && angles_host, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(n_ang >= 1 && n_det >= 1 && n_ang <= 65535, TVS_ERR_SHAPE,
                    "n_ang in [1, 65535] and n_det >= 1 required");
        TVS_REQUIRE(pixel > 0 && det_spacing >= pixel / 4 && det_spacing <= 4 * pixel,
                    TVS_ERR_INVALID_ARG, "pixel > 0 and pixel / 4 <= det_spacing <= 4 pixel required");
        TVS_REQUIRE(n_det <= 32768 && H <= 32768 && W <= 32768, TVS_ERR_SHAPE,
                    "n_det, H and W must be <= 32768");
        use_device(ctx);
        auto op = std::make_unique<tvs_op>();
        op->ctx = ctx;
        op->kind = OP_JOSEPH;
        op->H = H;
        op->W = W;
        JosephGeom& g = op->joseph;
        g.n_ang = n_ang;
        g.n_det = n_det;
        g.pixel = pixel;
        g.det_spacing = det_spacing;
        g.host.resize(n_ang);
        for (int a = 0; a < n_ang; ++a) {
            const double c = std::cos(angles_host[a]), s = std::sin(angles_host[a]);
            JAngle e;
            int n_step, n_int;
            if (std::fabs(c) >= std::fabs(s)) {
                // steps over rows i; interpolation coordinate = column
                e.cls = 0;
                e.A = det_spacing / (pixel * c);
                e.B = s / c;
                e.wgt = pixel / std::fabs(c);
                n_step = H;
                n_int = W;
            } else {
                // steps over columns j; interpolation coordinate = row
                e.cls = 1;
                e.A = -det_spacing / (pixel * s);
                e.B = c / s;
                e.wgt = pixel / std::fabs(s);
                n_step = W;
                n_int = H;
            }
            e.C = (n_int - 1) / 2.0 - (n_det - 1) / 2.0 * e.A - (n_step - 1) / 2.0 * e.B;
            e.inv_A = 1.0 / e.A;
            e.half_span = 1.0 / std::fabs(e.A);
            // candidates per pixel: rays whose u lies in [t - 1, t + 1), an
            // interval of 2 / |A| rays, plus one for the rounding of its start
            e.n_cand = (int)std::floor(2.0 / std::fabs(e.A) + 1e-3) + 2;
            e.Aq = std::nearbyint(std::ldexp(e.A, 32));
            e.Bq = std::nearbyint(std::ldexp(e.B, 32));
            e.Cq = std::nearbyint(std::ldexp(e.C, 32));
            e.Aqi = (long long)e.Aq;
            e.Bqi = (long long)e.Bq;
            e.Cqi = (long long)e.Cq;
            e.inv_Af = (float)e.inv_A;
            e.half_spanf = (float)e.half_span;
            g.host[a] = e;
        }
        joseph_upload(op.get());
        *out = op.release();
    });
}

namespace tvs {

// Device tables of a Joseph operator from its host angle table: the angle
// table, and whether the ray-driven float32 backprojector applies (every
// angle must qualify).
void joseph_upload(tvs_op* op) {
    JosephGeom& g = op->joseph;
    g.rd_ok = true;
    for (const JAngle& e : g.host) g.rd_ok = g.rd_ok && joseph_rd_angle_ok(e);
    g.pair_ok = true;
    for (const JAngle& e : g.host)
        g.pair_ok = g.pair_ok && std::fabs(e.Aq) >= 4294967296.0 && std::fabs(e.Aq) < 8589934592.0;
    TVS_HIP(hipMalloc(&g.ang, g.n_ang * sizeof(JAngle)));
    TVS_HIP(hipMemcpy(g.ang, g.host.data(), g.n_ang * sizeof(JAngle), hipMemcpyHostToDevice));
}

// The operators of the n angle subsets of a Joseph operator (subset j: the
// angles j, j + n, ..., with the parent's geometry entries, so every row is
// the parent's row bit for bit), built once per n and kept by the parent;
// the row permutation that puts each subset's rows together (subset 0's
// first) on the device.
void joseph_make_subsets(tvs_op* op, int n) {
    JosephGeom& g = op->joseph;
    if (g.sub_n == n) return;
    joseph_free_subsets(op);
    std::vector<int> perm;
    for (int j = 0; j < n; ++j) {
        auto s = std::make_unique<tvs_op>();
        s->ctx = op->ctx;
        s->kind = OP_JOSEPH;
        s->H = op->H;
        s->W = op->W;
        JosephGeom& sg = s->joseph;
        sg.n_det = g.n_det;
        sg.pixel = g.pixel;
        sg.det_spacing = g.det_spacing;
        g.sub_off.push_back((int)perm.size());
        for (int a = j; a < g.n_ang; a += n) {
            sg.host.push_back(g.host[a]);
            perm.push_back(a);
        }
        sg.n_ang = (int)sg.host.size();
        joseph_upload(s.get());
        g.subsets.push_back(s.release());
    }
    g.sub_off.push_back((int)perm.size());
    TVS_HIP(hipMalloc(&g.sub_perm, perm.size() * sizeof(int)));
    TVS_HIP(hipMemcpy(g.sub_perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice));
    g.sub_n = n;
}

void joseph_free_subsets(tvs_op* op) {
    JosephGeom& g = op->joseph;
    for (tvs_op* s : g.subsets) {
        if (s->joseph.ang) hipFree(s->joseph.ang);
        delete s;
    }
    g.subsets.clear();
    g.sub_off.clear();
    if (g.sub_perm) hipFree(g.sub_perm);
    g.sub_perm = nullptr;
    g.sub_n = 0;
}

}  // namespace tvs

extern "C" tvs_status tvs_op_joseph_set_groups(tvs_op* op, int groups) {
    return guarded([&] {
        TVS_REQUIRE(op && op->kind == OP_JOSEPH, TVS_ERR_INVALID_ARG, "not a Joseph operator");
        const int na = op->joseph.n_ang;
        const int gmin = (na + joseph_rd_max_angles() - 1) / joseph_rd_max_angles();
        TVS_REQUIRE(groups == 0 || (groups >= gmin && groups <= na), TVS_ERR_INVALID_ARG,
                    "groups must be 0 (automatic) or in [ceil(n_ang / max angles per group), n_ang]");
        use_device(op->ctx);
        TVS_HIP(hipDeviceSynchronize());
        graph_cache_clear(op->ctx);
        op->joseph.rd_groups = groups;
    });
}

extern "C" int tvs_op_joseph_groups(const tvs_op* op) {
    if (!op || op->kind != OP_JOSEPH) return -1;
    return joseph_rd_groups(op->ctx, op);
}

extern "C" void tvs_op_destroy(tvs_op* op) {
    if (!op) return;
    hipSetDevice(op->ctx->device);
    hipDeviceSynchronize();
    graph_cache_clear(op->ctx);
    if (op->blur.k_f) hipFree(op->blur.k_f);
    if (op->blur.k_d) hipFree(op->blur.k_d);
    if (op->joseph.ang) hipFree(op->joseph.ang);
    joseph_free_subsets(op);
    delete op;
}

extern "C" size_t tvs_op_out_size(const tvs_op* op) { return op ? op->out_size() : 0; }

namespace tvs {

template <typename T>
static void op_apply(tvs_op* op, const T* x, T* y, const T* b /* nullable: y = Ax - b */) {
    tvs_ctx* ctx = op->ctx;
    const size_t n = (size_t)op->H * op->W;
    if (op->kind == OP_IDENTITY) {
        if (b)
            launch_axpby<T>(ctx, n, T(1), x, T(-1), b, y);
        else
            launch_copy<T>(ctx, n, x, y);
    } else if (op->kind == OP_BLUR) {
        launch_blur<T>(ctx, op, false, x, b, y);
    } else {
        T* xp = (T*)scratch(ctx, S_PADX, (size_t)op->H * (op->W + 2 * JPAD) * sizeof(T)) + JPAD;
        T* xTp = (T*)scratch(ctx, S_TR_IMG, (size_t)op->W * (op->H + 2 * JPAD) * sizeof(T)) + JPAD;
        launch_pad_copy<T>(ctx, op->H, op->W, x, xp, xTp);
        launch_joseph_fwd<T>(ctx, op, xp, xTp, b, y, b ? FWD_RESIDUAL : FWD_STORE, T(0));
    }
}

template <typename T>
static void op_adjoint(tvs_op* op, const T* y, T* x) {
    tvs_ctx* ctx = op->ctx;
    const size_t n = (size_t)op->H * op->W;
    if (op->kind == OP_IDENTITY)
        launch_copy<T>(ctx, n, y, x);
    else if (op->kind == OP_BLUR)
        launch_blur<T>(ctx, op, true, y, (const T*)nullptr, x);
    else
        launch_joseph_adj<T>(ctx, op, y, x, nullptr);
}

// Phi(x) = 1/2 |A x - b|^2 + alpha TV(x) into out_dev[0] (device, no sync)
template <typename T>
static void objective_dev(tvs_op* op, const T* b, const T* x, double alpha, double* out_dev) {
    tvs_ctx* ctx = op->ctx;
    const size_t m = op->out_size();
    double* red = (double*)scratch(ctx, S_RED, 8 * sizeof(double));
    if (op->kind == OP_IDENTITY) {
        reduce_sq_diff<T>(ctx, m, x, b, red + 0);
    } else {
        T* res = (T*)scratch(ctx, S_RES, m * sizeof(T));
        op_apply<T>(op, x, res, b);
        reduce_sq_diff<T>(ctx, m, res, (const T*)nullptr, red + 0);
    }
    reduce_tv<T>(ctx, op->H, op->W, x, red + 1);
    launch_combine(ctx, red + 0, 0.5, red + 1, alpha, out_dev);
}

}  // namespace tvs

extern "C" tvs_status tvs_op_apply(tvs_op* op, tvs_dtype dtype, const void* x, void* y) {
    return guarded([&] {
        TVS_REQUIRE(op && x && y, TVS_ERR_INVALID_ARG, "null pointer");
        check_dtype(dtype);
        use_device(op->ctx);
        if (dtype == TVS_F32)
            op_apply<float>(op, (const float*)x, (float*)y, nullptr);
        else
            op_apply<double>(op, (const double*)x, (double*)y, nullptr);
    });
}

extern "C" tvs_status tvs_op_adjoint(tvs_op* op, tvs_dtype dtype, const void* y, void* x) {
    return guarded([&] {
        TVS_REQUIRE(op && x && y, TVS_ERR_INVALID_ARG, "null pointer");
        check_dtype(dtype);
        use_device(op->ctx);
        if (dtype == TVS_F32)
            op_adjoint<float>(op, (const float*)y, (float*)x);
        else
            op_adjoint<double>(op, (const double*)y, (double*)x);
    });
}

extern "C" tvs_status tvs_op_norm(tvs_op* op, int iters, uint64_t seed, double* norm_out) {
    return guarded([&] {
        TVS_REQUIRE(op && norm_out, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(iters >= 1, TVS_ERR_INVALID_ARG, "iters >= 1 required");
        tvs_ctx* ctx = op->ctx;
        use_device(ctx);
        const size_t n = (size_t)op->H * op->W, m = op->out_size();
        std::vector<double> h(n);
        for (size_t i = 0; i < n; ++i)
            h[i] = (double)(splitmix_mix(seed + (uint64_t)(i + 1) * kGolden) >> 11) *
                       (1.0 / 9007199254740992.0) - 0.5;
        double nrm = 0;
        for (double v : h) nrm += v * v;
        nrm = std::sqrt(nrm);
        for (double& v : h) v /= nrm;
        double* x = (double*)scratch(ctx, S_NORMV, n * sizeof(double));
        double* ax = (double*)scratch(ctx, S_RES, m * sizeof(double));
        double* y = (double*)scratch(ctx, S_Z, n * sizeof(double));
        double* red = (double*)scratch(ctx, S_RED, 8 * sizeof(double));
        TVS_HIP(hipMemcpyAsync(x, h.data(), n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        double est = 0.0;
        for (int it = 0; it < iters; ++it) {
            op_apply<double>(op, x, ax, nullptr);
            op_adjoint<double>(op, ax, y);
            reduce_sq_diff<double>(ctx, n, y, (const double*)nullptr, red);
            double s2 = 0;
            TVS_HIP(hipMemcpyAsync(&s2, red, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
            TVS_HIP(hipStreamSynchronize(ctx->stream));
            const double s = std::sqrt(s2);
            TVS_REQUIRE(std::isfinite(s) && s > 0, TVS_ERR_NONFINITE, "power iteration broke down");
            est = s;
            launch_axpby<double>(ctx, n, 1.0 / s, y, 0.0, y, x);
        }
        *norm_out = std::sqrt(est);
    });
}

// ========================================================= TV building blocks
extern "C" tvs_status tvs_grad(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, const void* u, void* q) {
    return guarded([&] {
        check_ctx(ctx);
        check_dtype(dtype);
        check_hw(H, W);
        TVS_REQUIRE(u && q, TVS_ERR_INVALID_ARG, "null pointer");
        use_device(ctx);
        if (dtype == TVS_F32)
            launch_grad<float>(ctx, H, W, (const float*)u, (float*)q);
        else
            launch_grad<double>(ctx, H, W, (const double*)u, (double*)q);
    });
}

extern "C" tvs_status tvs_div(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, const void* q, void* u) {
    return guarded([&] {
        check_ctx(ctx);
        check_dtype(dtype);
        check_hw(H, W);
        TVS_REQUIRE(u && q, TVS_ERR_INVALID_ARG, "null pointer");
        use_device(ctx);
        if (dtype == TVS_F32)
            launch_div<float>(ctx, H, W, (const float*)q, (float*)u);
        else
            launch_div<double>(ctx, H, W, (const double*)q, (double*)u);
    });
}

namespace tvs {

template <typename T>
void gap_host(tvs_ctx* ctx, int H, int W, const T* v, double lam, int nonneg, const T* q,
                     double* gap, double* primal) {
    const size_t n = (size_t)H * W;
    T* z = (T*)scratch(ctx, S_Z, n * sizeof(T));
    Finalize<T> f{};
    f.v = v;
    f.q = q;
    f.q_out = const_cast<T*>(q);
    f.z = z;
    f.nonneg = nonneg;
    f.mode = 0;
    launch_finalize<T>(ctx, H, W, f);
    double* red = (double*)scratch(ctx, S_RED, 8 * sizeof(double));
    reduce_gap<T>(ctx, H, W, v, z, q, lam, red + 0, red + 1);
    double hv[2];
    TVS_HIP(hipMemcpyAsync(hv, red, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    TVS_HIP(hipStreamSynchronize(ctx->stream));
    if (gap) *gap = hv[0];
    if (primal) *primal = hv[1];
}

template <typename T>
void tv_prox_impl(tvs_ctx* ctx, int H, int W, const T* v, double lambda, int iters,
                         int nonneg, T* q, T* z, double* rel_gap) {
    const FgpConfig cfg = fgp_config(ctx, H, W, (int)sizeof(T));
    T* qf = run_fgp<T>(ctx, H, W, v, lambda, iters, nonneg, q, cfg);
    Finalize<T> f{};
    f.v = v;
    f.q = qf;
    f.q_out = q;
    f.z = z;
    f.nonneg = nonneg;
    f.mode = 0;
    launch_finalize<T>(ctx, H, W, f);
    if (rel_gap) {
        double g = 0, pr = 0;
        gap_host<T>(ctx, H, W, v, lambda, nonneg, q, &g, &pr);
        *rel_gap = pr > 0 ? g / pr : g;
    }
}

template void gap_host<float>(tvs_ctx*, int, int, const float*, double, int, const float*,
                              double*, double*);
template void tv_prox_impl<float>(tvs_ctx*, int, int, const float*, double, int, int, float*,
                                  float*, double*);

}  // namespace tvs

extern "C" tvs_status tvs_tv_prox(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, const void* v,
                                  double lambda, int inner_iters, int nonneg, void* q_inout,
                                  void* z_out, double* rel_gap_out) {
    return guarded([&] {
        check_ctx(ctx);
        check_dtype(dtype);
        check_hw(H, W);
        TVS_REQUIRE(v && q_inout && z_out, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(lambda >= 0 && std::isfinite(lambda), TVS_ERR_INVALID_ARG, "lambda >= 0 required");
        TVS_REQUIRE(inner_iters >= 0, TVS_ERR_INVALID_ARG, "inner_iters >= 0 required");
        use_device(ctx);
        if (dtype == TVS_F32)
            tv_prox_impl<float>(ctx, H, W, (const float*)v, lambda, inner_iters, nonneg ? 1 : 0,
                                (float*)q_inout, (float*)z_out, rel_gap_out);
        else
            tv_prox_impl<double>(ctx, H, W, (const double*)v, lambda, inner_iters, nonneg ? 1 : 0,
                                 (double*)q_inout, (double*)z_out, rel_gap_out);
    });
}

extern "C" tvs_status tvs_tv_gap(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, const void* v,
                                 double lambda, int nonneg, const void* q, double* gap_out,
                                 double* primal_out) {
    return guarded([&] {
        check_ctx(ctx);
        check_dtype(dtype);
        check_hw(H, W);
        TVS_REQUIRE(v && q, TVS_ERR_INVALID_ARG, "null pointer");
        use_device(ctx);
        if (dtype == TVS_F32)
            gap_host<float>(ctx, H, W, (const float*)v, lambda, nonneg ? 1 : 0, (const float*)q,
                            gap_out, primal_out);
        else
            gap_host<double>(ctx, H, W, (const double*)v, lambda, nonneg ? 1 : 0, (const double*)q,
                             gap_out, primal_out);
    });
}

extern "C" tvs_status tvs_objective(tvs_op* op, tvs_dtype dtype, const void* b, const void* x,
                                    double alpha, double* out) {
    return guarded([&] {
        TVS_REQUIRE(op && b && x && out, TVS_ERR_INVALID_ARG, "null pointer");
        check_dtype(dtype);
        tvs_ctx* ctx = op->ctx;
        use_device(ctx);
        double* red = (double*)scratch(ctx, S_RED, 8 * sizeof(double));
        if (dtype == TVS_F32)
            objective_dev<float>(op, (const float*)b, (const float*)x, alpha, red + 2);
        else
            objective_dev<double>(op, (const double*)b, (const double*)x, alpha, red + 2);
        TVS_HIP(hipMemcpyAsync(out, red + 2, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        TVS_HIP(hipStreamSynchronize(ctx->stream));
        TVS_REQUIRE(std::isfinite(*out), TVS_ERR_NONFINITE, "objective is not finite");
    });
}

extern "C" int tvs_coin(uint64_t seed, uint64_t stream_id, int64_t k, double p) {
    return tvs::coin(seed, stream_id, k, p);
}

extern "C" int tvs_subset(uint64_t seed, uint64_t stream_id, int64_t k, int n) {
    return tvs::subset_draw(seed, stream_id, k, n);
}

// ================================================================ solvers
namespace tvs {

static void check_params(const tvs_params* P, bool pdhg) {
    TVS_REQUIRE(P, TVS_ERR_INVALID_ARG, "null params");
    TVS_REQUIRE(P->p > 0.0 && P->p <= 1.0, TVS_ERR_INVALID_ARG, "p must be in (0, 1]");
    TVS_REQUIRE(P->step > 0.0 && std::isfinite(P->step), TVS_ERR_INVALID_ARG, "step > 0 required");
    TVS_REQUIRE(P->alpha >= 0.0 && std::isfinite(P->alpha), TVS_ERR_INVALID_ARG, "alpha >= 0 required");
    TVS_REQUIRE(P->outer_iters >= 0, TVS_ERR_INVALID_ARG, "outer_iters >= 0 required");
    TVS_REQUIRE(P->inner_iters >= 1, TVS_ERR_INVALID_ARG, "inner_iters >= 1 required");
    TVS_REQUIRE(P->k0 >= 0, TVS_ERR_INVALID_ARG, "k0 >= 0 required");
    if (pdhg)
        TVS_REQUIRE(P->dual_step > 0.0 && std::isfinite(P->dual_step), TVS_ERR_INVALID_ARG,
                    "dual_step > 0 required");
}

// Enqueues the whole run (no host synchronisation).  obj_dev (nullable):
// device array receiving Phi(x_{k+1}).
template <typename T>
static void run_solver(tvs_op* op, bool pdhg, const T* b, const tvs_state* st,
                       const tvs_params* P, const std::vector<uint8_t>& theta, double* obj_dev,
                       const SolveExt& ext) {
    tvs_ctx* ctx = op->ctx;
    const int H = op->H, W = op->W;
    const size_t n = (size_t)H * W, m = op->out_size();
    T* x = (T*)st->x;
    T* h = (T*)st->h;
    T* q = (T*)st->q;
    T* y = (T*)st->y;
    T* xhat = (T*)scratch(ctx, S_XHAT, n * sizeof(T));
    T* v = (T*)scratch(ctx, S_V, n * sizeof(T));
    // xbar: the projector reads it through zero-padded copies (row stride
    // W + 2 JPAD and a transposed copy with row stride H + 2 JPAD)
    const bool jos = op->kind == OP_JOSEPH;
    const int xbar_ld = jos ? W + 2 * JPAD : W, xbarT_ld = H + 2 * JPAD;
    T* xbar = nullptr;
    T* xbarT = nullptr;
    if (pdhg && jos) {
        xbar = (T*)scratch(ctx, S_XBARP, (size_t)H * xbar_ld * sizeof(T)) + JPAD;
        xbarT = (T*)scratch(ctx, S_XBARTP, (size_t)W * xbarT_ld * sizeof(T)) + JPAD;
        // zero pads (a fill kernel, so the run stays capturable)
        launch_fill<T>(ctx, (size_t)H * xbar_ld, T(0), xbar - JPAD);
        launch_fill<T>(ctx, (size_t)W * xbarT_ld, T(0), xbarT - JPAD);
    } else if (pdhg) {
        xbar = (T*)scratch(ctx, S_XBAR, n * sizeof(T));
    }
    T* res = (T*)scratch(ctx, S_RES, m * sizeof(T));
    T* xp = nullptr;
    T* xTp = nullptr;
    if (!pdhg && jos) {
        xp = (T*)scratch(ctx, S_PADX, (size_t)H * (W + 2 * JPAD) * sizeof(T)) + JPAD;
        xTp = (T*)scratch(ctx, S_TR_IMG, (size_t)W * (H + 2 * JPAD) * sizeof(T)) + JPAD;
    }
    const double step = P->step, p = P->p;
    const double lam = P->alpha * step / p;
    const FgpConfig cfg = fgp_config(ctx, H, W, (int)sizeof(T));
    PrimalStep<T> ps{};
    ps.x = x;
    ps.h = h;
    ps.xhat = xhat;
    ps.v = v;
    ps.xbar = xbar;
    ps.xbarT = xbarT;
    ps.xbar_ld = xbar_ld;
    ps.xbarT_ld = xbarT_ld;
    ps.step = (T)step;
    ps.coef = (T)(step - step / p);
    ps.pdhg = pdhg ? 1 : 0;
    int64_t call = 0;
    for (int64_t kk = 0; kk < P->outer_iters; ++kk) {
        ps.theta = theta[kk];
        // data-fidelity step, fused with the control-variate bookkeeping
        if (!pdhg) {
            if (op->kind == OP_IDENTITY) {
                launch_identity_step<T>(ctx, H, W, b, ps);
            } else if (op->kind == OP_BLUR) {
                launch_blur<T>(ctx, op, false, x, b, res);
                launch_blur_adjoint_step<T>(ctx, op, res, ps);
            } else {
                launch_pad_copy<T>(ctx, H, W, x, xp, xTp);
                launch_joseph_fwd<T>(ctx, op, xp, xTp, b, res, FWD_RESIDUAL, T(0));
                launch_joseph_adj<T>(ctx, op, res, nullptr, &ps);
            }
        } else {
            if (op->kind == OP_IDENTITY)
                launch_identity_adj_step<T>(ctx, H, W, y, ps);
            else if (op->kind == OP_BLUR)
                launch_blur_adjoint_step<T>(ctx, op, y, ps);
            else
                launch_joseph_adj<T>(ctx, op, y, nullptr, &ps);
        }
        // the prox, only when the coin says so
        if (ps.theta) {
            if (ext.v_record && call < ext.max_record)
                launch_copy<T>(ctx, n, v, (T*)ext.v_record + (size_t)call * n);
            T* qf;
            if (ext.cnn) {
                qf = (T*)cnn::enqueue_solver_prox(ext.cnn, H, W, (const float*)v, lam, P->nonneg,
                                                  ext.gap_tol, P->inner_iters, (float*)q, cfg,
                                                  ext.gate + call);
            } else if (ext.inner_p > 0) {
                qf = run_tv_prox_skip<T>(ctx, H, W, v, lam, P->nonneg, P->inner_iters,
                                         ext.inner_p,
                                         ext.inner_theta + (size_t)call * P->inner_iters, q,
                                         (T*)ext.inner_h);
            } else {
                qf = run_fgp<T>(ctx, H, W, v, lam, P->inner_iters, P->nonneg, q, cfg);
            }
            ++call;
            Finalize<T> f{};
            f.v = v;
            f.q = qf;
            f.q_out = q;
            f.x = x;
            f.h = h;
            f.xhat = xhat;
            f.xbar = xbar;
            f.xbarT = xbarT;
            f.xbar_ld = xbar_ld;
            f.xbarT_ld = xbarT_ld;
            f.rate = (T)(p / step);
            f.nonneg = P->nonneg;
            f.mode = pdhg ? 2 : 1;
            launch_finalize<T>(ctx, H, W, f);
        }
        // dual step of PDHGSkip-2: y = prox_{tau f*}(y + tau A xbar)
        if (pdhg) {
            const T tau = (T)P->dual_step;
            if (op->kind == OP_IDENTITY)
                launch_dual_prox_pointwise<T>(ctx, n, xbar, b, y, tau);
            else if (op->kind == OP_BLUR)
                launch_blur_dual_prox<T>(ctx, op, xbar, b, y, tau);
            else
                launch_joseph_fwd<T>(ctx, op, xbar, xbarT, b, y, FWD_DUAL_PROX, tau);
        }
        if (obj_dev) objective_dev<T>(op, b, x, P->alpha, obj_dev + kk);
    }
}

// Allocates every scratch buffer and table run_solver uses, so that the
// launch sequence can be captured into a graph.
template <typename T>
static void prepare_solver(tvs_op* op, bool pdhg, const tvs_params* P) {
    tvs_ctx* ctx = op->ctx;
    const size_t n = (size_t)op->H * op->W, m = op->out_size();
    scratch(ctx, S_XHAT, n * sizeof(T));
    scratch(ctx, S_V, n * sizeof(T));
    if (op->kind == OP_JOSEPH) {
        const size_t rows = (size_t)op->H * (op->W + 2 * JPAD), cols = (size_t)op->W * (op->H + 2 * JPAD);
        scratch(ctx, pdhg ? S_XBARP : S_PADX, rows * sizeof(T));
        scratch(ctx, pdhg ? S_XBARTP : S_TR_IMG, cols * sizeof(T));
        if (sizeof(T) == 4 && op->joseph.rd_ok)
            scratch(ctx, S_PARTIMG, (size_t)joseph_rd_groups(ctx, op) * n * sizeof(T));
    }
    if (pdhg && op->kind != OP_JOSEPH) scratch(ctx, S_XBAR, n * sizeof(T));
    scratch(ctx, S_RES, m * sizeof(T));
    scratch(ctx, S_Q1, 2 * n * sizeof(T));
    scratch(ctx, S_Q2, 2 * n * sizeof(T));
    scratch(ctx, S_Q3, 2 * n * sizeof(T));
    beta_table_dev<T>(ctx, P->inner_iters + 1);
}

static tvs_status solve(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* st,
                        const tvs_params* P, double* obj_trace, uint8_t* theta_trace,
                        tvs_report* report, bool pdhg, tvs_solve_ext* ext_io) {
    return guarded([&] {
        TVS_REQUIRE(op && b && st, TVS_ERR_INVALID_ARG, "null pointer");
        check_dtype(dtype);
        check_params(P, pdhg);
        TVS_REQUIRE(st->x && st->h && st->q, TVS_ERR_INVALID_ARG, "state x, h, q required");
        TVS_REQUIRE(!pdhg || st->y, TVS_ERR_INVALID_ARG, "state y required for PDHGSkip");
        tvs_ctx* ctx = op->ctx;
        use_device(ctx);
        const int64_t K = P->outer_iters;
        std::vector<uint8_t> theta((size_t)K);
        int64_t nprox = 0;
        for (int64_t kk = 0; kk < K; ++kk) {
            theta[kk] = (uint8_t)coin(P->seed, P->stream_id, P->k0 + kk, P->p);
            nprox += theta[kk];
        }
        double* obj_dev = nullptr;
        if (obj_trace && K > 0) obj_dev = (double*)scratch(ctx, S_OBJ, (size_t)K * sizeof(double));
        const bool use_graph = (P->flags & TVS_FLAG_GRAPH) && !obj_dev && K > 0;
        SolveExt ext;
        std::vector<uint8_t> inner_theta;
        int64_t n_inner_proj = 0;
        if (ext_io) {
            TVS_REQUIRE(ext_io->max_record >= 0 && (ext_io->v_record || ext_io->max_record == 0),
                        TVS_ERR_INVALID_ARG, "v_record required when max_record > 0");
            ext.v_record = ext_io->v_record;
            ext.max_record = ext_io->max_record;
            if (ext_io->inner_p != 0.0) {
                TVS_REQUIRE(ext_io->inner_p > 0 && ext_io->inner_p <= 1, TVS_ERR_INVALID_ARG,
                            "inner_p must be in (0, 1]");
                TVS_REQUIRE(ext_io->inner_h, TVS_ERR_INVALID_ARG,
                            "inner_h required when inner_p > 0");
                TVS_REQUIRE(!ext_io->cnn, TVS_ERR_INVALID_ARG,
                            "the learned prox and the skipping inner solver exclude each other");
                ext.inner_p = ext_io->inner_p;
                ext.inner_h = ext_io->inner_h;
                // inner coins: stream stream_id xor 2^62, index k inner_iters + i
                const int Kin = P->inner_iters;
                inner_theta.resize((size_t)nprox * Kin);
                size_t c = 0;
                for (int64_t kk = 0; kk < K; ++kk) {
                    if (!theta[kk]) continue;
                    const int64_t k = P->k0 + kk;
                    for (int i = 0; i < Kin; ++i, ++c) {
                        inner_theta[c] = (uint8_t)coin(P->seed, P->stream_id ^ INNER_STREAM,
                                                       k * Kin + i, ext.inner_p);
                        n_inner_proj += inner_theta[c];
                    }
                }
                ext.inner_theta = inner_theta.data();
            }
            if (ext_io->cnn) {
                TVS_REQUIRE(dtype == TVS_F32, TVS_ERR_UNSUPPORTED,
                            "the learned prox runs on float32 only");
                TVS_REQUIRE(!std::isnan(ext_io->gap_tol), TVS_ERR_INVALID_ARG,
                            "gap_tol must be a number");
                ext.cnn = ext_io->cnn;
                ext.gap_tol = ext_io->gap_tol;
                ext.gate = (int*)scratch(ctx, S_GATE, (size_t)(nprox > 0 ? nprox : 1) * sizeof(int));
                cnn::prepare_solver_prox(ext.cnn, op->H, op->W, P->alpha * P->step / P->p);
            }
        }
        if (dtype == TVS_F32)
            prepare_solver<float>(op, pdhg, P);
        else
            prepare_solver<double>(op, pdhg, P);
        auto enqueue = [&] {
            if (dtype == TVS_F32)
                run_solver<float>(op, pdhg, (const float*)b, st, P, theta, obj_dev, ext);
            else
                run_solver<double>(op, pdhg, (const double*)b, st, P, theta, obj_dev, ext);
        };
        if (use_graph) {
            std::vector<uint64_t> key = graph_key(op, pdhg, (int)dtype, b, st, P);
            uint64_t tol_bits;
            std::memcpy(&tol_bits, &ext.gap_tol, sizeof(tol_bits));
            key.insert(key.end(), {(uint64_t)(uintptr_t)ext.cnn, tol_bits,
                                   (uint64_t)(uintptr_t)ext.v_record, (uint64_t)ext.max_record,
                                   (uint64_t)(uintptr_t)ext.gate,
                                   ext.cnn ? (uint64_t)cnn::fast_forward(ext.cnn) : 0});
            uint64_t pin_bits;
            std::memcpy(&pin_bits, &ext.inner_p, sizeof(pin_bits));
            key.insert(key.end(), {pin_bits, (uint64_t)(uintptr_t)ext.inner_h});
            graph_run_key(ctx, key, enqueue);
        } else {
            enqueue();
        }
        if (ext_io) {
            ext_io->n_recorded = nprox < ext.max_record ? nprox : ext.max_record;
            ext_io->n_fallback = 0;
            ext_io->n_inner_proj = n_inner_proj;
            if (ext.cnn && nprox > 0) {
                std::vector<int> g((size_t)nprox);
                TVS_HIP(hipMemcpyAsync(g.data(), ext.gate, (size_t)nprox * sizeof(int),
                                       hipMemcpyDeviceToHost, ctx->stream));
                TVS_HIP(hipStreamSynchronize(ctx->stream));
                for (int v : g) ext_io->n_fallback += v;
            }
        }
        if (theta_trace && K > 0) std::memcpy(theta_trace, theta.data(), (size_t)K);
        if (obj_dev) {
            TVS_HIP(hipMemcpyAsync(obj_trace, obj_dev, (size_t)K * sizeof(double),
                                   hipMemcpyDeviceToHost, ctx->stream));
            TVS_HIP(hipStreamSynchronize(ctx->stream));
        }
        if (report) {
            report->n_prox = nprox;
            report->iters = K;
        }
    });
}

// ------------------------------------------------------- comparison methods
// Alg. "FISTA" with the FGP prox (Beck-Teboulle momentum, restarted at every
// call): ybar = x_k + beta_k (x_k - x_{k-1}), x_{k+1} = prox_{gamma g}(ybar -
// gamma grad f(ybar)).  The data step at ybar is the ProxSkip data step with
// a zero control variate and theta = 1 (v = ybar - gamma grad f(ybar)); the
// iterates rotate through the caller's x and two scratch images.
template <typename T>
static void run_fista(tvs_op* op, const T* b, const tvs_state* st, const tvs_params* P,
                      const std::vector<double>& beta, double* obj_dev) {
    tvs_ctx* ctx = op->ctx;
    const int H = op->H, W = op->W;
    const size_t n = (size_t)H * W, m = op->out_size();
    T* xs[3] = {(T*)st->x, (T*)scratch(ctx, S_FX1, n * sizeof(T)),
                (T*)scratch(ctx, S_FX2, n * sizeof(T))};
    T* q = (T*)st->q;
    T* ybar = (T*)scratch(ctx, S_XBAR, n * sizeof(T));
    T* hz = (T*)scratch(ctx, S_HZERO, n * sizeof(T));
    T* xhat = (T*)scratch(ctx, S_XHAT, n * sizeof(T));
    T* v = (T*)scratch(ctx, S_V, n * sizeof(T));
    T* res = (T*)scratch(ctx, S_RES, m * sizeof(T));
    T* xp = nullptr;
    T* xTp = nullptr;
    if (op->kind == OP_JOSEPH) {
        xp = (T*)scratch(ctx, S_PADX, (size_t)H * (W + 2 * JPAD) * sizeof(T)) + JPAD;
        xTp = (T*)scratch(ctx, S_TR_IMG, (size_t)W * (H + 2 * JPAD) * sizeof(T)) + JPAD;
    }
    launch_fill<T>(ctx, n, T(0), hz);
    const double gamma = P->step;
    const FgpConfig cfg = fgp_config(ctx, H, W, (int)sizeof(T));
    PrimalStep<T> ps{};
    ps.x = ybar;
    ps.h = hz;
    ps.xhat = xhat;
    ps.v = v;
    ps.step = (T)gamma;
    ps.coef = T(0);
    ps.theta = 1;
    int cur = 0, prev = 0;  // x_{k-1} = x_k at the start of a call
    for (int64_t k = 0; k < P->outer_iters; ++k) {
        launch_fista_extrap<T>(ctx, n, xs[cur], xs[prev], (T)beta[k], ybar);
        if (op->kind == OP_IDENTITY) {
            launch_identity_step<T>(ctx, H, W, b, ps);
        } else if (op->kind == OP_BLUR) {
            launch_blur<T>(ctx, op, false, ybar, b, res);
            launch_blur_adjoint_step<T>(ctx, op, res, ps);
        } else {
            launch_pad_copy<T>(ctx, H, W, ybar, xp, xTp);
            launch_joseph_fwd<T>(ctx, op, xp, xTp, b, res, FWD_RESIDUAL, T(0));
            launch_joseph_adj<T>(ctx, op, res, nullptr, &ps);
        }
        const int nxt = (cur != 0 && prev != 0) ? 0 : ((cur != 1 && prev != 1) ? 1 : 2);
        T* qf = run_fgp<T>(ctx, H, W, v, P->alpha * gamma, P->inner_iters, P->nonneg, q, cfg);
        Finalize<T> f{};
        f.v = v;
        f.q = qf;
        f.q_out = q;
        f.z = xs[nxt];
        f.nonneg = P->nonneg;
        f.mode = 0;
        launch_finalize<T>(ctx, H, W, f);
        prev = cur;
        cur = nxt;
        if (obj_dev) objective_dev<T>(op, b, xs[cur], P->alpha, obj_dev + k);
    }
    if (cur != 0) launch_copy<T>(ctx, n, xs[cur], xs[0]);
}

// Alg. "PDHGSkip-1" (omega + 1 = 1/p): theta_k = 1: x+ = prox_{sigma g}(x_k -
// sigma K^T y_k) (the adjoint's primal-step epilogue with a zero control
// variate gives x_k - sigma K^T y_k), e = (1 + 1/p) x+ - x_k / p (finalize
// mode 4); theta_k = 0: x and e = x_k unchanged, neither K^T y nor the prox
// is run.  Then y = (y + tau (K e - b)) / (1 + tau).
template <typename T>
static void run_pdhgskip1(tvs_op* op, const T* b, const tvs_state* st, const tvs_params* P,
                          const std::vector<uint8_t>& theta, double* obj_dev) {
    tvs_ctx* ctx = op->ctx;
    const int H = op->H, W = op->W;
    const size_t n = (size_t)H * W;
    T* x = (T*)st->x;
    T* q = (T*)st->q;
    T* y = (T*)st->y;
    T* hz = (T*)scratch(ctx, S_HZERO, n * sizeof(T));
    T* xhat = (T*)scratch(ctx, S_XHAT, n * sizeof(T));
    T* v = (T*)scratch(ctx, S_V, n * sizeof(T));
    const bool jos = op->kind == OP_JOSEPH;
    const int e_ld = jos ? W + 2 * JPAD : W, eT_ld = H + 2 * JPAD;
    T* e = nullptr;
    T* eT = nullptr;
    if (jos) {
        e = (T*)scratch(ctx, S_XBARP, (size_t)H * e_ld * sizeof(T)) + JPAD;
        eT = (T*)scratch(ctx, S_XBARTP, (size_t)W * eT_ld * sizeof(T)) + JPAD;
        launch_fill<T>(ctx, (size_t)H * e_ld, T(0), e - JPAD);
        launch_fill<T>(ctx, (size_t)W * eT_ld, T(0), eT - JPAD);
    } else {
        e = (T*)scratch(ctx, S_XBAR, n * sizeof(T));
    }
    launch_fill<T>(ctx, n, T(0), hz);
    const double sigma = P->step, p = P->p;
    const T tau = (T)P->dual_step;
    const FgpConfig cfg = fgp_config(ctx, H, W, (int)sizeof(T));
    PrimalStep<T> ps{};
    ps.x = x;
    ps.h = hz;
    ps.xhat = xhat;
    ps.v = v;
    ps.step = (T)sigma;
    ps.coef = T(0);
    ps.theta = 1;
    for (int64_t kk = 0; kk < P->outer_iters; ++kk) {
        const T* ep;
        if (theta[kk]) {
            if (op->kind == OP_IDENTITY)
                launch_identity_adj_step<T>(ctx, H, W, y, ps);
            else if (op->kind == OP_BLUR)
                launch_blur_adjoint_step<T>(ctx, op, y, ps);
            else
                launch_joseph_adj<T>(ctx, op, y, nullptr, &ps);
            T* qf = run_fgp<T>(ctx, H, W, v, P->alpha * sigma, P->inner_iters, P->nonneg, q, cfg);
            Finalize<T> f{};
            f.v = v;
            f.q = qf;
            f.q_out = q;
            f.x = x;
            f.xbar = e;
            f.xbarT = jos ? eT : nullptr;
            f.xbar_ld = e_ld;
            f.xbarT_ld = eT_ld;
            f.c1 = (T)(1.0 + 1.0 / p);
            f.c2 = (T)(1.0 / p);
            f.nonneg = P->nonneg;
            f.mode = 4;
            launch_finalize<T>(ctx, H, W, f);
            ep = e;
        } else if (jos) {
            launch_pad_copy<T>(ctx, H, W, x, e, eT);
            ep = e;
        } else {
            ep = x;
        }
        if (op->kind == OP_IDENTITY)
            launch_dual_prox_pointwise<T>(ctx, n, ep, b, y, tau);
        else if (op->kind == OP_BLUR)
            launch_blur_dual_prox<T>(ctx, op, ep, b, y, tau);
        else
            launch_joseph_fwd<T>(ctx, op, ep, eT, b, y, FWD_DUAL_PROX, tau);
        if (obj_dev) objective_dev<T>(op, b, x, P->alpha, obj_dev + kk);
    }
}

// ------------------------------------------- stochastic angle subsets
// SPDHG over the n angle subsets with the prox skipped as in PDHGSkip-2
// (the paper's "Discussion and Future work"):
//   w = x - sigma zbar;  xhat = w + sigma h;  theta: x+ = prox(w + coef h),
//   h += (p/sigma)(x+ - xhat); else x+ = xhat;
//   j = j_k:  y_j <- (y_j + tau (A_j x+ - b_j)) / (1 + tau);  dy = change;
//   z += A_j^T dy;  zbar = z + n A_j^T dy;   z = zbar = A^T y at the start.
// The sinogram is worked on in a row order that puts each subset's rows
// together (b and y are permuted in and y back out), so that subset j is the
// parent's rows [off_j, off_{j+1}) and its own operator's whole output.
template <typename T>
static void run_spdhg(tvs_op* op, int nsub, const T* b, const tvs_state* st, const tvs_params* P,
                      const std::vector<uint8_t>& theta, const std::vector<int>& sub,
                      double* obj_dev) {
    tvs_ctx* ctx = op->ctx;
    JosephGeom& g = op->joseph;
    const int H = op->H, W = op->W, nd = g.n_det;
    const size_t n = (size_t)H * W, m = op->out_size();
    T* x = (T*)st->x;
    T* h = (T*)st->h;
    T* q = (T*)st->q;
    T* y = (T*)st->y;
    T* xhat = (T*)scratch(ctx, S_XHAT, n * sizeof(T));
    T* v = (T*)scratch(ctx, S_V, n * sizeof(T));
    const int xp_ld = W + 2 * JPAD, xTp_ld = H + 2 * JPAD;
    T* xp = (T*)scratch(ctx, S_XBARP, (size_t)H * xp_ld * sizeof(T)) + JPAD;
    T* xTp = (T*)scratch(ctx, S_XBARTP, (size_t)W * xTp_ld * sizeof(T)) + JPAD;
    T* bp = (T*)scratch(ctx, S_SB, m * sizeof(T));
    T* yp = (T*)scratch(ctx, S_SY, m * sizeof(T));
    T* dy = (T*)scratch(ctx, S_SDY, m * sizeof(T));
    T* z = (T*)scratch(ctx, S_SZ, n * sizeof(T));
    T* zbar = (T*)scratch(ctx, S_SZB, n * sizeof(T));
    launch_fill<T>(ctx, (size_t)H * xp_ld, T(0), xp - JPAD);
    launch_fill<T>(ctx, (size_t)W * xTp_ld, T(0), xTp - JPAD);
    launch_permute_rows<T>(ctx, g.n_ang, nd, g.sub_perm, b, bp, false);
    launch_permute_rows<T>(ctx, g.n_ang, nd, g.sub_perm, y, yp, false);
    launch_joseph_adj<T>(ctx, op, y, z, nullptr);
    launch_copy<T>(ctx, n, z, zbar);
    const double sigma = P->step, p = P->p;
    const double lam = P->alpha * sigma / p;
    const FgpConfig cfg = fgp_config(ctx, H, W, (int)sizeof(T));
    PrimalStep<T> ps{};
    ps.x = x;
    ps.h = h;
    ps.xhat = xhat;
    ps.v = v;
    ps.xbar = xp;
    ps.xbarT = xTp;
    ps.xbar_ld = xp_ld;
    ps.xbarT_ld = xTp_ld;
    ps.step = (T)sigma;
    ps.coef = (T)(sigma - sigma / p);
    ps.pdhg = 1;
    ps.xcopy = 1;
    ZAcc<T> za{z, zbar, (T)nsub};
    const T tau = (T)P->dual_step;
    for (int64_t kk = 0; kk < P->outer_iters; ++kk) {
        ps.theta = theta[kk];
        launch_identity_adj_step<T>(ctx, H, W, zbar, ps);
        if (ps.theta) {
            T* qf = run_fgp<T>(ctx, H, W, v, lam, P->inner_iters, P->nonneg, q, cfg);
            Finalize<T> f{};
            f.v = v;
            f.q = qf;
            f.q_out = q;
            f.x = x;
            f.h = h;
            f.xhat = xhat;
            f.xbar = xp;
            f.xbarT = xTp;
            f.xbar_ld = xp_ld;
            f.xbarT_ld = xTp_ld;
            f.rate = (T)(p / sigma);
            f.nonneg = P->nonneg;
            f.mode = 3;
            launch_finalize<T>(ctx, H, W, f);
        }
        const int j = sub[kk];
        const tvs_op* sj = g.subsets[j];
        const size_t off = (size_t)g.sub_off[j] * nd;
        launch_joseph_fwd<T>(ctx, sj, xp, xTp, bp + off, yp + off, FWD_DUAL_PROX_DELTA, tau, dy);
        launch_joseph_adj<T>(ctx, sj, dy, nullptr, nullptr, &za);
        if (obj_dev) objective_dev<T>(op, b, x, P->alpha, obj_dev + kk);
    }
    launch_permute_rows<T>(ctx, g.n_ang, nd, g.sub_perm, yp, y, true);
}

template <typename T>
static void prepare_spdhg(tvs_op* op, const tvs_params* P) {
    tvs_ctx* ctx = op->ctx;
    const JosephGeom& g = op->joseph;
    const size_t n = (size_t)op->H * op->W, m = op->out_size();
    scratch(ctx, S_XHAT, n * sizeof(T));
    scratch(ctx, S_V, n * sizeof(T));
    scratch(ctx, S_XBARP, (size_t)op->H * (op->W + 2 * JPAD) * sizeof(T));
    scratch(ctx, S_XBARTP, (size_t)op->W * (op->H + 2 * JPAD) * sizeof(T));
    for (Slot s : {S_SB, S_SY, S_SDY}) scratch(ctx, s, m * sizeof(T));
    scratch(ctx, S_SZ, n * sizeof(T));
    scratch(ctx, S_SZB, n * sizeof(T));
    scratch(ctx, S_RES, m * sizeof(T));
    scratch(ctx, S_Q1, 2 * n * sizeof(T));
    scratch(ctx, S_Q2, 2 * n * sizeof(T));
    scratch(ctx, S_Q3, 2 * n * sizeof(T));
    beta_table_dev<T>(ctx, P->inner_iters + 1);
    if (sizeof(T) == 4) {
        size_t part = 0;
        std::vector<const tvs_op*> ops(g.subsets.begin(), g.subsets.end());
        ops.push_back(op);
        for (const tvs_op* o : ops)
            if (o->joseph.rd_ok) part = std::max(part, (size_t)joseph_rd_groups(ctx, o) * n * sizeof(T));
        if (part) scratch(ctx, S_PARTIMG, part);
    }
}

static tvs_status spdhg_solve(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* st,
                              const tvs_params* P, int nsub, double* obj_trace,
                              uint8_t* theta_trace, int32_t* subset_trace, tvs_report* report) {
    return guarded([&] {
        TVS_REQUIRE(op && b && st, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(op->kind == OP_JOSEPH, TVS_ERR_UNSUPPORTED,
                    "angle subsets need a Joseph (CT) operator");
        check_dtype(dtype);
        check_params(P, true);
        TVS_REQUIRE(st->x && st->h && st->q && st->y, TVS_ERR_INVALID_ARG,
                    "state x, h, q, y required");
        TVS_REQUIRE(nsub >= 1 && nsub <= op->joseph.n_ang && nsub <= 1024, TVS_ERR_INVALID_ARG,
                    "n_subsets must be in [1, min(n_ang, 1024)]");
        tvs_ctx* ctx = op->ctx;
        use_device(ctx);
        const int64_t K = P->outer_iters;
        std::vector<uint8_t> theta((size_t)K);
        std::vector<int> sub((size_t)K);
        int64_t nprox = 0;
        for (int64_t kk = 0; kk < K; ++kk) {
            theta[kk] = (uint8_t)coin(P->seed, P->stream_id, P->k0 + kk, P->p);
            sub[kk] = subset_draw(P->seed, P->stream_id, P->k0 + kk, nsub);
            nprox += theta[kk];
        }
        if (op->joseph.sub_n != nsub) {
            TVS_HIP(hipDeviceSynchronize());
            graph_cache_clear(ctx);
            joseph_make_subsets(op, nsub);
        }
        double* obj_dev = nullptr;
        if (obj_trace && K > 0) obj_dev = (double*)scratch(ctx, S_OBJ, (size_t)K * sizeof(double));
        const bool use_graph = (P->flags & TVS_FLAG_GRAPH) && !obj_dev && K > 0;
        if (dtype == TVS_F32)
            prepare_spdhg<float>(op, P);
        else
            prepare_spdhg<double>(op, P);
        auto enqueue = [&] {
            if (dtype == TVS_F32)
                run_spdhg<float>(op, nsub, (const float*)b, st, P, theta, sub, obj_dev);
            else
                run_spdhg<double>(op, nsub, (const double*)b, st, P, theta, sub, obj_dev);
        };
        if (use_graph) {
            std::vector<uint64_t> key = graph_key(op, true, (int)dtype, b, st, P);
            key.insert(key.end(), {0x5BD61ULL, (uint64_t)nsub});
            graph_run_key(ctx, key, enqueue);
        } else {
            enqueue();
        }
        if (theta_trace && K > 0) std::memcpy(theta_trace, theta.data(), (size_t)K);
        if (subset_trace)
            for (int64_t kk = 0; kk < K; ++kk) subset_trace[kk] = sub[kk];
        if (obj_dev) {
            TVS_HIP(hipMemcpyAsync(obj_trace, obj_dev, (size_t)K * sizeof(double),
                                   hipMemcpyDeviceToHost, ctx->stream));
            TVS_HIP(hipStreamSynchronize(ctx->stream));
        }
        if (report) {
            report->n_prox = nprox;
            report->iters = K;
        }
    });
}

template <typename T>
static void prepare_cmp(tvs_op* op, bool skip1, const tvs_params* P) {
    tvs_ctx* ctx = op->ctx;
    const size_t n = (size_t)op->H * op->W, m = op->out_size();
    for (Slot s : {S_XHAT, S_V, S_HZERO}) scratch(ctx, s, n * sizeof(T));
    if (!skip1)
        for (Slot s : {S_FX1, S_FX2, S_XBAR}) scratch(ctx, s, n * sizeof(T));
    scratch(ctx, S_RES, m * sizeof(T));
    if (op->kind == OP_JOSEPH) {
        const size_t rows = (size_t)op->H * (op->W + 2 * JPAD), cols = (size_t)op->W * (op->H + 2 * JPAD);
        scratch(ctx, skip1 ? S_XBARP : S_PADX, rows * sizeof(T));
        scratch(ctx, skip1 ? S_XBARTP : S_TR_IMG, cols * sizeof(T));
        if (sizeof(T) == 4 && op->joseph.rd_ok)
            scratch(ctx, S_PARTIMG, (size_t)joseph_rd_groups(ctx, op) * n * sizeof(T));
    } else if (skip1) {
        scratch(ctx, S_XBAR, n * sizeof(T));
    }
    scratch(ctx, S_Q1, 2 * n * sizeof(T));
    scratch(ctx, S_Q2, 2 * n * sizeof(T));
    scratch(ctx, S_Q3, 2 * n * sizeof(T));
    beta_table_dev<T>(ctx, P->inner_iters + 1);
}

// FISTA (skip1 = false) and PDHGSkip-1 (skip1 = true): host-side schedule
// (momentum coefficients / coin), optional graph capture, traces.
static tvs_status cmp_solve(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* st,
                            const tvs_params* P, double* obj_trace, uint8_t* theta_trace,
                            tvs_report* report, bool skip1) {
    return guarded([&] {
        TVS_REQUIRE(op && b && st, TVS_ERR_INVALID_ARG, "null pointer");
        check_dtype(dtype);
        check_params(P, skip1);
        TVS_REQUIRE(st->x && st->q, TVS_ERR_INVALID_ARG, "state x, q required");
        TVS_REQUIRE(!skip1 || st->y, TVS_ERR_INVALID_ARG, "state y required for PDHGSkip-1");
        tvs_ctx* ctx = op->ctx;
        use_device(ctx);
        const int64_t K = P->outer_iters;
        std::vector<uint8_t> theta((size_t)K, 1);
        std::vector<double> beta((size_t)K, 0.0);
        int64_t nprox = K;
        if (skip1) {
            nprox = 0;
            for (int64_t kk = 0; kk < K; ++kk) {
                theta[kk] = (uint8_t)coin(P->seed, P->stream_id, P->k0 + kk, P->p);
                nprox += theta[kk];
            }
        } else {
            double t = 1.0;
            for (int64_t kk = 0; kk < K; ++kk) {
                const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
                beta[kk] = (t - 1.0) / tn;
                t = tn;
            }
        }
        double* obj_dev = nullptr;
        if (obj_trace && K > 0) obj_dev = (double*)scratch(ctx, S_OBJ, (size_t)K * sizeof(double));
        const bool use_graph = (P->flags & TVS_FLAG_GRAPH) && !obj_dev && K > 0;
        if (dtype == TVS_F32)
            prepare_cmp<float>(op, skip1, P);
        else
            prepare_cmp<double>(op, skip1, P);
        auto enqueue = [&] {
            if (dtype == TVS_F32) {
                if (skip1)
                    run_pdhgskip1<float>(op, (const float*)b, st, P, theta, obj_dev);
                else
                    run_fista<float>(op, (const float*)b, st, P, beta, obj_dev);
            } else {
                if (skip1)
                    run_pdhgskip1<double>(op, (const double*)b, st, P, theta, obj_dev);
                else
                    run_fista<double>(op, (const double*)b, st, P, beta, obj_dev);
            }
        };
        if (use_graph) {
            std::vector<uint64_t> key = graph_key(op, skip1, (int)dtype, b, st, P);
            key.insert(key.end(), {skip1 ? 0x5C1ULL : 0xF157AULL});
            graph_run_key(ctx, key, enqueue);
        } else {
            enqueue();
        }
        if (theta_trace && K > 0) std::memcpy(theta_trace, theta.data(), (size_t)K);
        if (obj_dev) {
            TVS_HIP(hipMemcpyAsync(obj_trace, obj_dev, (size_t)K * sizeof(double),
                                   hipMemcpyDeviceToHost, ctx->stream));
            TVS_HIP(hipStreamSynchronize(ctx->stream));
        }
        if (report) {
            report->n_prox = nprox;
            report->iters = K;
        }
    });
}

}  // namespace tvs

extern "C" tvs_status tvs_fista(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                                const tvs_params* params, double* obj_trace, tvs_report* report) {
    return cmp_solve(op, dtype, b, state, params, obj_trace, nullptr, report, false);
}

extern "C" tvs_status tvs_pdhgskip1(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                                    const tvs_params* params, double* obj_trace,
                                    uint8_t* theta_trace, tvs_report* report) {
    return cmp_solve(op, dtype, b, state, params, obj_trace, theta_trace, report, true);
}

extern "C" tvs_status tvs_spdhgskip(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                                    const tvs_params* params, int n_subsets, double* obj_trace,
                                    uint8_t* theta_trace, int32_t* subset_trace,
                                    tvs_report* report) {
    return spdhg_solve(op, dtype, b, state, params, n_subsets, obj_trace, theta_trace,
                       subset_trace, report);
}

extern "C" tvs_status tvs_proxskip(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                                   const tvs_params* params, double* obj_trace,
                                   uint8_t* theta_trace, tvs_report* report) {
    return solve(op, dtype, b, state, params, obj_trace, theta_trace, report, false, nullptr);
}

extern "C" tvs_status tvs_pdhgskip(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                                   const tvs_params* params, double* obj_trace,
                                   uint8_t* theta_trace, tvs_report* report) {
    return solve(op, dtype, b, state, params, obj_trace, theta_trace, report, true, nullptr);
}

extern "C" tvs_status tvs_proxskip_ex(tvs_op* op, tvs_dtype dtype, const void* b,
                                      tvs_state* state, const tvs_params* params,
                                      tvs_solve_ext* ext, double* obj_trace,
                                      uint8_t* theta_trace, tvs_report* report) {
    return solve(op, dtype, b, state, params, obj_trace, theta_trace, report, false, ext);
}

extern "C" tvs_status tvs_pdhgskip_ex(tvs_op* op, tvs_dtype dtype, const void* b,
                                      tvs_state* state, const tvs_params* params,
                                      tvs_solve_ext* ext, double* obj_trace,
                                      uint8_t* theta_trace, tvs_report* report) {
    return solve(op, dtype, b, state, params, obj_trace, theta_trace, report, true, ext);
}
