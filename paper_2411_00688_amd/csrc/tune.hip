// FGP tile / temporal-depth autotuning.  Every compiled variant (output tile
// BW x BH, TS fused iterations per launch) is timed with HIP events on a
// seeded random image of the requested size; the fastest is kept per
// (H, W, dtype) in the context and used by every later prox evaluation.
#include <cmath>

#include "tvs_internal.hpp"

using namespace tvs;

namespace tvs {
void set_error(const std::string& msg);
}

extern "C" int tvs_fgp_variant_count(void) { return fgp_variant_count(); }

extern "C" tvs_status tvs_fgp_variant(int index, int* tile_w, int* tile_h, int* steps) {
    if (index < 0 || index >= fgp_variant_count() || !tile_w || !tile_h || !steps) {
        set_error("variant index out of range or null output");
        return TVS_ERR_INVALID_ARG;
    }
    FgpConfig c = fgp_variant(index);
    *tile_w = c.tile_w;
    *tile_h = c.tile_h;
    *steps = c.steps;
    return TVS_OK;
}

extern "C" tvs_status tvs_fgp_set_variant(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, int index) {
    if (!ctx || (dtype != TVS_F32 && dtype != TVS_F64) || index < -1 ||
        index >= fgp_variant_count()) {
        set_error("bad context, dtype or variant index");
        return TVS_ERR_INVALID_ARG;
    }
    const int bytes = dtype == TVS_F32 ? 4 : 8;
    if (index < 0) {
        ctx->fgp_tuned.erase(fgp_key(H, W, bytes));
        return TVS_OK;
    }
    FgpConfig c = fgp_variant(index);
    if (bytes == 8 && c.tile_w == 64 && c.tile_h == 32 && c.steps == 8) {
        set_error("variant not compiled for float64");
        return TVS_ERR_UNSUPPORTED;
    }
    ctx->fgp_tuned[fgp_key(H, W, bytes)] = c;
    return TVS_OK;
}

namespace {

template <typename T>
void autotune(tvs_ctx* ctx, int H, int W, int iters, int reps, int* best, double* ms_out) {
    const size_t n = (size_t)H * W;
    T *v = nullptr, *q = nullptr;
    TVS_HIP(hipMalloc(&v, n * sizeof(T)));
    TVS_HIP(hipMalloc(&q, 2 * n * sizeof(T)));
    std::vector<T> hv(n);
    for (size_t i = 0; i < n; ++i)
        hv[i] = (T)((double)(splitmix_mix(i + 1) >> 11) * (1.0 / 9007199254740992.0));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best_ms = 1e300;
    int best_i = -1;
    try {
        TVS_HIP(hipMemcpy(v, hv.data(), n * sizeof(T), hipMemcpyHostToDevice));
        TVS_HIP(hipEventCreate(&e0));
        TVS_HIP(hipEventCreate(&e1));
        for (int vi = 0; vi < fgp_variant_count(); ++vi) {
            FgpConfig c = fgp_variant(vi);
            if (sizeof(T) == 8 && c.tile_w == 64 && c.tile_h == 32 && c.steps == 8) {
                if (ms_out) ms_out[vi] = -1.0;
                continue;
            }
            launch_fill<T>(ctx, 2 * n, T(0), q);
            run_fgp<T>(ctx, H, W, v, 0.1, iters, 0, q, c);  // warm-up
            TVS_HIP(hipEventRecord(e0, ctx->stream));
            for (int r = 0; r < reps; ++r) run_fgp<T>(ctx, H, W, v, 0.1, iters, 0, q, c);
            TVS_HIP(hipEventRecord(e1, ctx->stream));
            TVS_HIP(hipEventSynchronize(e1));
            float ms = 0;
            TVS_HIP(hipEventElapsedTime(&ms, e0, e1));
            const double per_iter = (double)ms / ((double)reps * iters);
            if (ms_out) ms_out[vi] = per_iter;
            if (per_iter < best_ms) {
                best_ms = per_iter;
                best_i = vi;
            }
        }
    } catch (...) {
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
        hipFree(v);
        hipFree(q);
        throw;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    TVS_HIP(hipStreamSynchronize(ctx->stream));
    hipFree(v);
    hipFree(q);
    ctx->fgp_tuned[fgp_key(H, W, (int)sizeof(T))] = fgp_variant(best_i);
    if (best) *best = best_i;
}

}  // namespace

extern "C" tvs_status tvs_fgp_autotune(tvs_ctx* ctx, tvs_dtype dtype, int H, int W,
                                       int inner_iters, int reps, int* best_index,
                                       double* ms_per_iter_out) {
    try {
        TVS_REQUIRE(ctx, TVS_ERR_INVALID_ARG, "null context");
        TVS_REQUIRE(dtype == TVS_F32 || dtype == TVS_F64, TVS_ERR_INVALID_ARG, "bad dtype");
        TVS_REQUIRE(H >= 1 && W >= 1, TVS_ERR_SHAPE, "bad size");
        TVS_REQUIRE(inner_iters >= 1 && reps >= 1, TVS_ERR_INVALID_ARG, "inner_iters, reps >= 1");
        TVS_HIP(hipSetDevice(ctx->device));
        if (dtype == TVS_F32)
            autotune<float>(ctx, H, W, inner_iters, reps, best_index, ms_per_iter_out);
        else
            autotune<double>(ctx, H, W, inner_iters, reps, best_index, ms_per_iter_out);
        return TVS_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    } catch (...) {
        set_error("unexpected C++ exception");
        return TVS_ERR_DEVICE;
    }
}
