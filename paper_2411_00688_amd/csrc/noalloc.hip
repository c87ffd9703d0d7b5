// The allocation-free TV prox (tvs_tv_prox_noalloc): the same FGP and
// finalize kernels as tvs_tv_prox, with the work buffers (the momentum
// table and three dual fields) in one file-scope device array instead of
// context scratch, for callers that cannot allocate device memory (code
// under stream capture, serving loops, harnesses that forbid hipMalloc).
// Every call on a device shares that device's array and leaves its
// contents behind; calls that overlap on one device race.
#include <cmath>
#include <mutex>

#include "tvs_internal.hpp"

// TVS_NOALLOC_SCRATCH_BYTES (include/tvskip.h): 32 MiB per device, held
// until the process ends.
static __device__ __align__(256) unsigned char scratch[TVS_NOALLOC_SCRATCH_BYTES];

namespace tvs {
namespace {

std::mutex g_noalloc_mu;
constexpr int kMaxDevices = 64;
void* g_noalloc_ptr[kMaxDevices] = {};

// t_0 = 1, t_k = (1 + sqrt(1 + 4 t_{k-1}^2)) / 2, beta[0] = 0,
// beta[k] = (t_{k-1} - 1) / t_k: the FGP momentum table, in float64 as on
// the host, by one thread (n is the inner iteration count plus one).
template <typename T>
__global__ void beta_fill_kernel(T* beta, int n) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double t = 1.0;
    beta[0] = T(0);
    for (int k = 1; k < n; ++k) {
        const double tn = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
        beta[k] = (T)((t - 1.0) / tn);
        t = tn;
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

template <typename T>
void tv_prox_noalloc_impl(tvs_ctx* ctx, int H, int W, const T* v, double lambda, int iters,
                          int nonneg, T* q, T* z) {
    unsigned char* base = (unsigned char*)noalloc_ptr(ctx->device);
    const size_t plane = (size_t)H * W;
    const size_t beta_bytes = align256((size_t)(iters + 1) * sizeof(T));
    const size_t dual_bytes = align256(2 * plane * sizeof(T));
    TVS_REQUIRE(beta_bytes + 3 * dual_bytes <= (size_t)TVS_NOALLOC_SCRATCH_BYTES,
                TVS_ERR_INVALID_ARG,
                "image too large for the no-allocation scratch (TVS_NOALLOC_SCRATCH_BYTES: "
                "256-byte-aligned (inner_iters + 1) + 3 * 2 * H * W elements)");
    T* beta = (T*)base;
    T* bufs[3] = {(T*)(base + beta_bytes), (T*)(base + beta_bytes + dual_bytes),
                  (T*)(base + beta_bytes + 2 * dual_bytes)};
    hipLaunchKernelGGL((beta_fill_kernel<T>), dim3(1), dim3(64), 0, ctx->stream, beta, iters + 1);
    TVS_LAUNCH_CHECK();
    const FgpConfig cfg = fgp_config(ctx, H, W, (int)sizeof(T));
    T* qf = run_fgp_bufs<T>(ctx, H, W, v, lambda, iters, nonneg, q, bufs, beta, cfg, nullptr);
    Finalize<T> f{};
    f.v = v;
    f.q = qf;
    f.q_out = q;
    f.z = z;
    f.nonneg = nonneg;
    f.mode = 0;
    launch_finalize<T>(ctx, H, W, f);
}

template <typename F>
tvs_status guarded_noalloc(F&& f) {
    try {
        f();
        return TVS_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    } catch (...) {
        set_error("unexpected C++ exception");
        return TVS_ERR_DEVICE;
    }
}

}  // namespace

// Device address of this device's array (hipGetSymbolAddress with the
// device current), once per device; the array's name is only a host-side
// stand-in.
void noalloc_setup(int device) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    TVS_REQUIRE(device >= 0 && device < kMaxDevices, TVS_ERR_DEVICE, "device index too large");
    if (g_noalloc_ptr[device]) return;
    void* p = nullptr;
    // ::scratch: the array (tvs::scratch is the context's scratch allocator)
    TVS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch)));
    TVS_REQUIRE(p, TVS_ERR_DEVICE, "no device address for the no-allocation scratch");
    g_noalloc_ptr[device] = p;
}

void* noalloc_ptr(int device) {
    {
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        if (device >= 0 && device < kMaxDevices && g_noalloc_ptr[device])
            return g_noalloc_ptr[device];
    }
    noalloc_setup(device);
    return g_noalloc_ptr[device];
}

}  // namespace tvs

extern "C" tvs_status tvs_tv_prox_noalloc(tvs_ctx* ctx, tvs_dtype dtype, int H, int W,
                                          const void* v, double lambda, int inner_iters,
                                          int nonneg, void* q_inout, void* z_out) {
    return tvs::guarded_noalloc([&] {
        TVS_REQUIRE(ctx, TVS_ERR_INVALID_ARG, "null context");
        TVS_REQUIRE(dtype == TVS_F32 || dtype == TVS_F64, TVS_ERR_INVALID_ARG, "unknown dtype");
        TVS_REQUIRE(H >= 1 && W >= 1, TVS_ERR_SHAPE, "H, W >= 1 required");
        TVS_REQUIRE(v && q_inout && z_out, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(lambda >= 0 && std::isfinite(lambda), TVS_ERR_INVALID_ARG,
                    "lambda >= 0 required");
        TVS_REQUIRE(inner_iters >= 0, TVS_ERR_INVALID_ARG, "inner_iters >= 0 required");
        TVS_HIP(hipSetDevice(ctx->device));
        if (dtype == TVS_F32)
            tvs::tv_prox_noalloc_impl<float>(ctx, H, W, (const float*)v, lambda, inner_iters,
                                             nonneg ? 1 : 0, (float*)q_inout, (float*)z_out);
        else
            tvs::tv_prox_noalloc_impl<double>(ctx, H, W, (const double*)v, lambda, inner_iters,
                                              nonneg ? 1 : 0, (double*)q_inout, (double*)z_out);
    });
}
