// C ABI of the learned TV prox: parameters, forward / backward passes,
// Adam, the gap-gated prox and save / load.  The kernels live in
// kernels_cnn.hip; this file sequences them on the context's stream.
#include <cmath>
#include <cstdio>
#include <vector>

#include "tvs_internal.hpp"

namespace tvs {
namespace cnn {

constexpr int NL = 4;
constexpr int CIN[NL] = {2, 32, 32, 32};
constexpr int COUT[NL] = {32, 32, 32, 2};

static size_t w_off(int l) {
    size_t s = 0;
    for (int k = 0; k < l; ++k) s += (size_t)9 * CIN[k] * COUT[k] + COUT[k];
    return s;
}
static size_t b_off(int l) { return w_off(l) + (size_t)9 * CIN[l] * COUT[l]; }
static const size_t NPARAM = w_off(NL);

static int kp_of(int c) { return (9 * c + 31) / 32 * 32; }
static int padded16(int c) { return (c + 15) / 16 * 16; }

struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace cnn
}  // namespace tvs

struct tvs_cnn {
    tvs_ctx* ctx = nullptr;
    float* params = nullptr;  // FP32 master parameters
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    float* grad = nullptr;
    int64_t step = 0;
    uint16_t* wf[tvs::cnn::NL] = {};  // BF16 forward weights [coutp][kp]
    uint16_t* wf_lo[tvs::cnn::NL] = {};  // their low parts (w - bf16(w), rounded)
    uint16_t* wb[tvs::cnn::NL] = {};  // BF16 input-gradient weights [32][kp'] (layers 2..4)
    bool have_grad = false;
    bool fast = false;  // single-part BF16 forward for tvs_cnn_forward / tvs_cnn_prox
    // scratch
    enum { B_LAM, B_X1, B_X2, B_X3, B_X1L, B_X2L, B_X3L, B_QT, B_GU, B_G4, B_GA, B_GB, B_PART,
           B_LOSSP, B_LOSS, B_COUNT };
    tvs::cnn::DevBuf buf[B_COUNT];
    std::vector<float> lam_cache;
};

namespace tvs {
namespace cnn {

static void* grow(tvs_cnn* c, int which, size_t bytes) {
    DevBuf& b = c->buf[which];
    if (b.ptr && b.bytes >= bytes) return b.ptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TVS_HIP(hipStreamIsCapturing(c->ctx->stream, &cs));
    TVS_REQUIRE(cs == hipStreamCaptureStatusNone, TVS_ERR_DEVICE,
                "learned-prox scratch would have to grow during graph capture");
    if (b.ptr) {
        TVS_HIP(hipStreamSynchronize(c->ctx->stream));
        graph_cache_clear(c->ctx);
        TVS_HIP(hipFree(b.ptr));
        b.ptr = nullptr;
        b.bytes = 0;
    }
    size_t want = ((bytes < 256 ? 256 : bytes) + 255) & ~(size_t)255;
    TVS_HIP(hipMalloc(&b.ptr, want));
    b.bytes = want;
    return b.ptr;
}

static void check_batch(int n, int H, int W) {
    TVS_REQUIRE(n >= 1 && H >= 1 && W >= 1 && H <= 32768 && W <= 32768, TVS_ERR_SHAPE,
                "learned prox: need n >= 1 and 1 <= H, W <= 32768");
    TVS_REQUIRE((long long)n * H * W <= (1LL << 31), TVS_ERR_SHAPE,
                "learned prox: n H W must not exceed 2^31");
}

static void set_lam(tvs_cnn* c, int n, const double* lam_host) {
    TVS_REQUIRE(lam_host, TVS_ERR_INVALID_ARG, "null lam");
    std::vector<float> lf(n);
    for (int i = 0; i < n; ++i) {
        TVS_REQUIRE(std::isfinite(lam_host[i]) && lam_host[i] >= 0, TVS_ERR_INVALID_ARG,
                    "lam >= 0 required");
        lf[i] = (float)lam_host[i];
    }
    if (c->lam_cache == lf && c->buf[tvs_cnn::B_LAM].bytes >= n * sizeof(float)) return;
    float* d = (float*)grow(c, tvs_cnn::B_LAM, n * sizeof(float));
    TVS_HIP(hipMemcpyAsync(d, lf.data(), n * sizeof(float), hipMemcpyHostToDevice, c->ctx->stream));
    TVS_HIP(hipStreamSynchronize(c->ctx->stream));  // lf is a temporary
    c->lam_cache = lf;
}

static void pack_all(tvs_cnn* c) {
    for (int l = 0; l < NL; ++l)
        launch_pack(c->ctx, c->params + w_off(l), CIN[l], COUT[l], c->wf[l], c->wf_lo[l],
                    l > 0 ? c->wb[l] : nullptr);
}

// Forward through the four convolutions.  With proj, layer 4 writes
// P_lam(qt) into qt_dst; else the raw qt.  split selects the two-part
// (hi + lo) BF16 operands; the activations' high parts always land in
// B_X1..B_X3 (the backward pass reads them).
static void forward_convs(tvs_cnn* c, int n, int H, int W, const float* v, float* qt_dst,
                          int proj, bool split, const int* run = nullptr) {
    const size_t npx = (size_t)n * H * W;
    const float* lam = (const float*)c->buf[tvs_cnn::B_LAM].ptr;
    uint16_t* x[3];
    uint16_t* xl[3] = {nullptr, nullptr, nullptr};
    for (int l = 0; l < 3; ++l) {
        x[l] = (uint16_t*)grow(c, tvs_cnn::B_X1 + l, npx * 64);
        if (split) xl[l] = (uint16_t*)grow(c, tvs_cnn::B_X1L + l, npx * 64);
    }
    for (int l = 0; l < NL; ++l) {
        ConvArgs a;
        a.n = n;
        a.H = H;
        a.W = W;
        a.lam = lam;
        a.v = v;
        a.wt = c->wf[l];
        a.wt_lo = c->wf_lo[l];
        a.bias = c->params + b_off(l);
        a.run = run;
        if (l > 0) {
            a.in = x[l - 1];
            a.in_lo = xl[l - 1];
        }
        if (l < NL - 1) {
            a.out_bf = x[l];
            a.out_lo = xl[l];
            launch_conv(c->ctx, CIN[l], 32, l == 0 ? IN_VLAM : IN_BF16, OUT_RELU_BF16, split, a);
        } else {
            a.out_f = qt_dst;
            a.proj = proj;
            launch_conv(c->ctx, 32, 16, IN_BF16, OUT_F32_PLANAR, split, a);
        }
    }
}

static void loss_grad(tvs_cnn* c, int n, int H, int W, const float* v, int nonneg,
                      const float* zt, const float* qtg, double mu, double* loss_out) {
    const size_t npx = (size_t)n * H * W;
    float* qt = (float*)grow(c, tvs_cnn::B_QT, npx * 2 * sizeof(float));
    float* gu = (float*)grow(c, tvs_cnn::B_GU, npx * sizeof(float));
    uint16_t* g4 = (uint16_t*)grow(c, tvs_cnn::B_G4, npx * 4);
    uint16_t* gA = (uint16_t*)grow(c, tvs_cnn::B_GA, npx * 64);
    uint16_t* gB = (uint16_t*)grow(c, tvs_cnn::B_GB, npx * 64);
    const int nwg = wgrad_blocks(c->ctx, n, H, W);
    float* part = (float*)grow(c, tvs_cnn::B_PART, (size_t)nwg * 289 * 32 * sizeof(float));
    const int nhb = head_blocks(c->ctx, npx);
    double* lossp = (double*)grow(c, tvs_cnn::B_LOSSP, (size_t)nhb * sizeof(double));
    double* loss = (double*)grow(c, tvs_cnn::B_LOSS, sizeof(double));
    const float* lam = (const float*)c->buf[tvs_cnn::B_LAM].ptr;

    forward_convs(c, n, H, W, v, qt, 0, true);
    const uint16_t* x1 = (const uint16_t*)c->buf[tvs_cnn::B_X1].ptr;
    const uint16_t* x2 = (const uint16_t*)c->buf[tvs_cnn::B_X2].ptr;
    const uint16_t* x3 = (const uint16_t*)c->buf[tvs_cnn::B_X3].ptr;

    HeadArgs h;
    h.n = n;
    h.H = H;
    h.W = W;
    h.nonneg = nonneg;
    h.qt = qt;
    h.v = v;
    h.lam = lam;
    h.z_target = zt;
    h.q_target = (qtg && mu != 0.0) ? qtg : nullptr;
    h.mu = (float)mu;
    h.gu = gu;
    h.inv_npx = (float)(1.0 / (double)npx);
    h.loss_part = lossp;
    h.loss_out = loss;
    h.gq_bf = g4;
    launch_head_fwd(c->ctx, h, nhb);
    launch_head_bwd(c->ctx, h, nhb);

    WgradArgs w;
    w.n = n;
    w.H = H;
    w.W = W;
    w.v = v;
    w.lam = lam;
    w.part = part;
    // layer 4: dW from x3 and g4; input gradient masked by x3 > 0
    w.x = x3;
    w.g = g4;
    launch_wgrad(c->ctx, 3, w, c->grad + w_off(3));
    ConvArgs a;
    a.n = n;
    a.H = H;
    a.W = W;
    a.in = g4;
    a.wt = c->wb[3];
    a.mask = x3;
    a.out_bf = gA;
    launch_conv(c->ctx, 2, 32, IN_BF16, OUT_MASK_BF16, false, a);
    // layer 3
    w.x = x2;
    w.g = gA;
    launch_wgrad(c->ctx, 2, w, c->grad + w_off(2));
    a.in = gA;
    a.wt = c->wb[2];
    a.mask = x2;
    a.out_bf = gB;
    launch_conv(c->ctx, 32, 32, IN_BF16, OUT_MASK_BF16, false, a);
    // layer 2
    w.x = x1;
    w.g = gB;
    launch_wgrad(c->ctx, 1, w, c->grad + w_off(1));
    a.in = gB;
    a.wt = c->wb[1];
    a.mask = x1;
    a.out_bf = gA;
    launch_conv(c->ctx, 32, 32, IN_BF16, OUT_MASK_BF16, false, a);
    // layer 1 (input is (v, lam))
    w.x = nullptr;
    w.g = gA;
    launch_wgrad(c->ctx, 0, w, c->grad + w_off(0));
    c->have_grad = true;

    if (loss_out) {
        double s = 0;
        TVS_HIP(hipMemcpyAsync(&s, loss, sizeof(double), hipMemcpyDeviceToHost, c->ctx->stream));
        TVS_HIP(hipStreamSynchronize(c->ctx->stream));
        *loss_out = s / (2.0 * (double)npx);
    }
}

static void adam(tvs_cnn* c, const float* grad, double lr) {
    TVS_REQUIRE(grad || c->have_grad, TVS_ERR_INVALID_ARG, "no gradient to apply");
    TVS_REQUIRE(std::isfinite(lr) && lr >= 0, TVS_ERR_INVALID_ARG, "lr >= 0 required");
    const double b1 = 0.9, b2 = 0.999;
    c->step += 1;
    const double c1 = 1.0 - std::pow(b1, (double)c->step);
    const double c2 = 1.0 - std::pow(b2, (double)c->step);
    launch_adam(c->ctx, (int)NPARAM, c->params, grad ? grad : c->grad, c->adam_m, c->adam_v,
                (float)lr, (float)b1, (float)b2, (float)c1, (float)c2, 1e-8f);
    pack_all(c);
}

// He-normal initial weights from SplitMix64 (Steele, Lea and Flood, 2014)
// counters and the Box-Muller transform.
static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static std::vector<float> init_params(uint64_t seed) {
    std::vector<float> p(NPARAM, 0.f);
    const uint64_t key = mix64(seed ^ 0x6A09E667F3BCC909ULL);
    uint64_t ctr = 0;
    auto uniform = [&]() {
        ctr += 1;
        uint64_t r = mix64(key + ctr * 0x9E3779B97F4A7C15ULL);
        return ((double)(r >> 11) + 0.5) * (1.0 / 9007199254740992.0);  // (0, 1)
    };
    for (int l = 0; l < NL; ++l) {
        const double sd = std::sqrt(2.0 / (9.0 * CIN[l]));
        const size_t nw = (size_t)9 * CIN[l] * COUT[l];
        for (size_t i = 0; i < nw; i += 2) {
            const double u1 = uniform(), u2 = uniform();
            const double rad = std::sqrt(-2.0 * std::log(u1));
            p[w_off(l) + i] = (float)(sd * rad * std::cos(2.0 * M_PI * u2));
            if (i + 1 < nw) p[w_off(l) + i + 1] = (float)(sd * rad * std::sin(2.0 * M_PI * u2));
        }
    }
    return p;
}

static void upload_params(tvs_cnn* c, const float* host) {
    for (size_t i = 0; i < NPARAM; ++i)
        TVS_REQUIRE(std::isfinite(host[i]), TVS_ERR_NONFINITE, "non-finite parameter");
    hipStream_t st = c->ctx->stream;
    TVS_HIP(hipMemcpyAsync(c->params, host, NPARAM * sizeof(float), hipMemcpyHostToDevice, st));
    TVS_HIP(hipStreamSynchronize(st));
    TVS_HIP(hipMemsetAsync(c->adam_m, 0, NPARAM * sizeof(float), st));
    TVS_HIP(hipMemsetAsync(c->adam_v, 0, NPARAM * sizeof(float), st));
    c->step = 0;
    c->have_grad = false;
    pack_all(c);
}

static void destroy(tvs_cnn* c) {
    if (!c) return;
    if (c->ctx) (void)hipSetDevice(c->ctx->device);
    if (c->ctx) (void)hipStreamSynchronize(c->ctx->stream);
    for (void* p : {(void*)c->params, (void*)c->adam_m, (void*)c->adam_v, (void*)c->grad})
        if (p) (void)hipFree(p);
    for (int l = 0; l < NL; ++l) {
        if (c->wf[l]) (void)hipFree(c->wf[l]);
        if (c->wf_lo[l]) (void)hipFree(c->wf_lo[l]);
        if (c->wb[l]) (void)hipFree(c->wb[l]);
    }
    for (auto& b : c->buf)
        if (b.ptr) (void)hipFree(b.ptr);
    delete c;
}

bool fast_forward(const tvs_cnn* c) { return c->fast; }

void prepare_solver_prox(tvs_cnn* c, int H, int W, double lam) {
    TVS_REQUIRE(c && c->ctx, TVS_ERR_INVALID_ARG, "null network");
    check_batch(1, H, W);
    const size_t npx = (size_t)H * W;
    set_lam(c, 1, &lam);
    for (int l = 0; l < 3; ++l) {
        grow(c, tvs_cnn::B_X1 + l, npx * 64);
        if (!c->fast) grow(c, tvs_cnn::B_X1L + l, npx * 64);
    }
    scratch(c->ctx, S_Z, npx * sizeof(float));
    scratch(c->ctx, S_QNET, 2 * npx * sizeof(float));
    scratch(c->ctx, S_SEL, 2 * sizeof(int));
    reserve_reduce_scratch(c->ctx, npx);
}

float* enqueue_solver_prox(tvs_cnn* c, int H, int W, const float* v, double lam, int nonneg,
                           double tol, int iters, float* q, const FgpConfig& cfg, int* record) {
    tvs_ctx* ctx = c->ctx;
    const size_t npx = (size_t)H * W;
    float* qn = (float*)scratch(ctx, S_QNET, 2 * npx * sizeof(float));
    float* z = (float*)scratch(ctx, S_Z, npx * sizeof(float));
    // relative duality gaps of the network's dual (red[0], red[1]) and of the
    // previous call's dual still in q (red[2], red[3])
    double* red = (double*)scratch(ctx, S_RED, 8 * sizeof(double));
    int* sel = (int*)scratch(ctx, S_SEL, 2 * sizeof(int));
    int* run = sel + 1;
    auto gap_of = [&](float* cand, double* out) {
        Finalize<float> f{};
        f.v = v;
        f.q = cand;
        f.q_out = cand;
        f.z = z;
        f.nonneg = nonneg;
        f.mode = 0;
        launch_finalize<float>(ctx, H, W, f);
        reduce_gap<float>(ctx, H, W, v, z, cand, lam, out, out + 1);
    };
    // the previous call's dual first: when it passes the gate it is the
    // result and the network is not evaluated (its kernels return at once)
    gap_of(q, red + 2);
    launch_pregate(ctx, red, tol, run);
    forward_convs(c, 1, H, W, v, qn, 1, !c->fast, run);  // qn <- P_lam(qt)
    gap_of(qn, red);  // not read by the gate when the network was skipped
    int* flag = record;  // the per-call record doubles as this call's flag
    launch_gate(ctx, red, tol, run, flag, sel);
    launch_copy_if(ctx, 2 * npx, sel, 1, qn, q);  // start (or result): the network's dual
    float* qf = run_fgp<float>(ctx, H, W, v, lam, iters, nonneg, q, cfg, flag);
    if (qf != q) launch_copy_if(ctx, 2 * npx, flag, 0, q, qf);
    return qf;
}

}  // namespace cnn
}  // namespace tvs

using namespace tvs;
using namespace tvs::cnn;

namespace {
template <typename F>
tvs_status guarded_cnn(F&& f) {
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

void check_cnn(tvs_cnn* c) {
    TVS_REQUIRE(c && c->ctx, TVS_ERR_INVALID_ARG, "null network");
    TVS_HIP(hipSetDevice(c->ctx->device));
}
}  // namespace

extern "C" int64_t tvs_cnn_param_count(void) { return (int64_t)NPARAM; }

extern "C" tvs_status tvs_cnn_create(tvs_ctx* ctx, uint64_t seed, tvs_cnn** out) {
    tvs_cnn* c = nullptr;
    tvs_status st = guarded_cnn([&] {
        TVS_REQUIRE(ctx && out, TVS_ERR_INVALID_ARG, "null argument");
        TVS_HIP(hipSetDevice(ctx->device));
        c = new tvs_cnn();
        c->ctx = ctx;
        TVS_HIP(hipMalloc(&c->params, NPARAM * sizeof(float)));
        TVS_HIP(hipMalloc(&c->adam_m, NPARAM * sizeof(float)));
        TVS_HIP(hipMalloc(&c->adam_v, NPARAM * sizeof(float)));
        TVS_HIP(hipMalloc(&c->grad, NPARAM * sizeof(float)));
        for (int l = 0; l < NL; ++l) {
            TVS_HIP(hipMalloc(&c->wf[l], (size_t)padded16(COUT[l]) * kp_of(CIN[l]) * 2));
            TVS_HIP(hipMalloc(&c->wf_lo[l], (size_t)padded16(COUT[l]) * kp_of(CIN[l]) * 2));
            if (l > 0) TVS_HIP(hipMalloc(&c->wb[l], (size_t)32 * kp_of(COUT[l]) * 2));
        }
        std::vector<float> p = init_params(seed);
        upload_params(c, p.data());
        *out = c;
    });
    if (st != TVS_OK) destroy(c);
    return st;
}

extern "C" void tvs_cnn_destroy(tvs_cnn* cnn) { destroy(cnn); }

extern "C" tvs_status tvs_cnn_get_params(tvs_cnn* cnn, float* params_host) {
    return guarded_cnn([&] {
        check_cnn(cnn);
        TVS_REQUIRE(params_host, TVS_ERR_INVALID_ARG, "null output");
        TVS_HIP(hipMemcpyAsync(params_host, cnn->params, NPARAM * sizeof(float),
                               hipMemcpyDeviceToHost, cnn->ctx->stream));
        TVS_HIP(hipStreamSynchronize(cnn->ctx->stream));
    });
}

extern "C" tvs_status tvs_cnn_set_params(tvs_cnn* cnn, const float* params_host) {
    return guarded_cnn([&] {
        check_cnn(cnn);
        TVS_REQUIRE(params_host, TVS_ERR_INVALID_ARG, "null input");
        upload_params(cnn, params_host);
    });
}

extern "C" tvs_status tvs_cnn_forward(tvs_cnn* cnn, int n, int H, int W, const float* v,
                                      const double* lam_host, int nonneg, float* qt_out,
                                      float* z_out) {
    return guarded_cnn([&] {
        check_cnn(cnn);
        check_batch(n, H, W);
        TVS_REQUIRE(v && (qt_out || z_out), TVS_ERR_INVALID_ARG, "null pointer");
        set_lam(cnn, n, lam_host);
        const size_t npx = (size_t)n * H * W;
        float* qt = qt_out ? qt_out : (float*)grow(cnn, tvs_cnn::B_QT, npx * 2 * sizeof(float));
        forward_convs(cnn, n, H, W, v, qt, 0, !cnn->fast);
        if (z_out) {
            HeadArgs h;
            h.n = n;
            h.H = H;
            h.W = W;
            h.nonneg = nonneg ? 1 : 0;
            h.qt = qt;
            h.v = v;
            h.lam = (const float*)cnn->buf[tvs_cnn::B_LAM].ptr;
            h.z = z_out;
            launch_head_fwd(cnn->ctx, h, head_blocks(cnn->ctx, npx));
        }
    });
}

extern "C" tvs_status tvs_cnn_loss_grad(tvs_cnn* cnn, int n, int H, int W, const float* v,
                                        const double* lam_host, int nonneg,
                                        const float* z_target, const float* q_target, double mu,
                                        double* loss_out, float* grad_out) {
    return guarded_cnn([&] {
        check_cnn(cnn);
        check_batch(n, H, W);
        TVS_REQUIRE(v && z_target, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(std::isfinite(mu) && mu >= 0, TVS_ERR_INVALID_ARG, "mu >= 0 required");
        set_lam(cnn, n, lam_host);
        loss_grad(cnn, n, H, W, v, nonneg ? 1 : 0, z_target, q_target, mu, loss_out);
        if (grad_out)
            TVS_HIP(hipMemcpyAsync(grad_out, cnn->grad, NPARAM * sizeof(float),
                                   hipMemcpyDeviceToDevice, cnn->ctx->stream));
    });
}

extern "C" tvs_status tvs_cnn_adam_step(tvs_cnn* cnn, const float* grad, double lr) {
    return guarded_cnn([&] {
        check_cnn(cnn);
        adam(cnn, grad, lr);
    });
}

extern "C" tvs_status tvs_cnn_train_step(tvs_cnn* cnn, int n, int H, int W, const float* v,
                                         const double* lam_host, int nonneg,
                                         const float* z_target, const float* q_target,
                                         double mu, double lr, double* loss_out) {
    return guarded_cnn([&] {
        check_cnn(cnn);
        check_batch(n, H, W);
        TVS_REQUIRE(v && z_target, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(std::isfinite(mu) && mu >= 0, TVS_ERR_INVALID_ARG, "mu >= 0 required");
        set_lam(cnn, n, lam_host);
        loss_grad(cnn, n, H, W, v, nonneg ? 1 : 0, z_target, q_target, mu, loss_out);
        adam(cnn, nullptr, lr);
    });
}

extern "C" tvs_status tvs_cnn_prox(tvs_cnn* cnn, int H, int W, const float* v, double lam,
                                   int nonneg, double gap_tol, int fallback_iters, float* q_out,
                                   float* z_out, int* fell_back_out, double* rel_gap_out) {
    return guarded_cnn([&] {
        check_cnn(cnn);
        check_batch(1, H, W);
        TVS_REQUIRE(v && q_out && z_out, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(fallback_iters >= 0, TVS_ERR_INVALID_ARG, "fallback_iters >= 0 required");
        TVS_REQUIRE(!std::isnan(gap_tol), TVS_ERR_INVALID_ARG, "gap_tol must be a number");
        set_lam(cnn, 1, &lam);
        const int nn = nonneg ? 1 : 0;
        forward_convs(cnn, 1, H, W, v, q_out, 1, !cnn->fast);
        double g = 0, pr = 0;
        gap_host<float>(cnn->ctx, H, W, v, lam, nn, q_out, &g, &pr);
        const double rel = pr > 0 ? g / pr : g;
        const bool fb = !(rel <= gap_tol) && fallback_iters > 0;  // a NaN gap falls back
        // ... from the zero dual when the gap is not finite: such a network
        // dual (overflowed activations) is no warm start
        if (fb && !std::isfinite(rel)) launch_fill<float>(cnn->ctx, (size_t)2 * H * W, 0.0f, q_out);
        tv_prox_impl<float>(cnn->ctx, H, W, v, lam, fb ? fallback_iters : 0, nn, q_out, z_out,
                            nullptr);
        if (fell_back_out) *fell_back_out = fb ? 1 : 0;
        if (rel_gap_out) *rel_gap_out = rel;
    });
}

extern "C" tvs_status tvs_cnn_set_fast_forward(tvs_cnn* cnn, int fast) {
    return guarded_cnn([&] {
        check_cnn(cnn);
        cnn->fast = fast != 0;
    });
}

extern "C" tvs_status tvs_cnn_save(tvs_cnn* cnn, const char* path) {
    return guarded_cnn([&] {
        check_cnn(cnn);
        TVS_REQUIRE(path, TVS_ERR_INVALID_ARG, "null path");
        std::vector<float> p(NPARAM);
        TVS_HIP(hipMemcpyAsync(p.data(), cnn->params, NPARAM * sizeof(float),
                               hipMemcpyDeviceToHost, cnn->ctx->stream));
        TVS_HIP(hipStreamSynchronize(cnn->ctx->stream));
        FILE* f = std::fopen(path, "wb");
        TVS_REQUIRE(f, TVS_ERR_INVALID_ARG, std::string("cannot open ") + path);
        const int64_t cnt = (int64_t)NPARAM;
        bool ok = std::fwrite("TVSCNN01", 1, 8, f) == 8 && std::fwrite(&cnt, 8, 1, f) == 1 &&
                  std::fwrite(p.data(), sizeof(float), NPARAM, f) == NPARAM;
        ok = (std::fclose(f) == 0) && ok;
        TVS_REQUIRE(ok, TVS_ERR_DEVICE, std::string("write failed: ") + path);
    });
}

extern "C" tvs_status tvs_cnn_load(tvs_cnn* cnn, const char* path) {
    return guarded_cnn([&] {
        check_cnn(cnn);
        TVS_REQUIRE(path, TVS_ERR_INVALID_ARG, "null path");
        FILE* f = std::fopen(path, "rb");
        TVS_REQUIRE(f, TVS_ERR_INVALID_ARG, std::string("cannot open ") + path);
        char magic[8] = {};
        int64_t cnt = 0;
        std::vector<float> p(NPARAM);
        bool ok = std::fread(magic, 1, 8, f) == 8 && std::fread(&cnt, 8, 1, f) == 1;
        ok = ok && std::memcmp(magic, "TVSCNN01", 8) == 0;
        if (ok && cnt == (int64_t)NPARAM) ok = std::fread(p.data(), sizeof(float), NPARAM, f) == NPARAM;
        std::fclose(f);
        TVS_REQUIRE(ok, TVS_ERR_INVALID_ARG, std::string("not a parameter file: ") + path);
        TVS_REQUIRE(cnt == (int64_t)NPARAM, TVS_ERR_SHAPE, "parameter count mismatch");
        upload_params(cnn, p.data());
    });
}
