// Batched ProxSkip TV denoising: many independent slices of uneven sizes in
// one launch sequence per outer iteration.  Each iteration is one data-step
// launch over every tile of every slice, the FGP launches over the tiles of
// the slices whose coin came up (a work list per iteration, built on the host
// from the counter-based coin before anything runs), and one finalize launch
// over those tiles.  The whole run can be captured into one HIP graph.
//
// Every slice gets exactly the arithmetic of the single-image solver with
// A = I (same kernels' per-pixel code, same per-slice scalars), so a slice's
// result equals a separate tvs_proxskip call with that slice's parameters.
#include <algorithm>
#include <cmath>

#include "tvs_internal.hpp"

namespace tvs {
void set_error(const std::string& msg);
}

using namespace tvs;

namespace {

struct Plan {
    std::vector<int> ints;            // all per-iteration lists, packed
    std::vector<size_t> it_off;       // per iteration: offset of act / pref_fgp / pref_fin
    std::vector<int> n_act, tiles_fgp, tiles_fin;
    std::vector<int> pref_all;        // 32 x 32 tiles of every slice, cumulative
    std::vector<uint8_t> theta;       // [K][n]
    std::vector<int64_t> nprox;
};

int tiles_of(int H, int W, int bw, int bh) { return div_up(W, bw) * div_up(H, bh); }

template <typename T>
void run_batched(tvs_ctx* ctx, int n, const tvs_slice* S, const T* b, T* x, T* h, T* q,
                 const tvs_batch_params* P, int64_t* nprox_out) {
    // ------------------------------------------------------------ validation
    TVS_REQUIRE(n >= 1, TVS_ERR_SHAPE, "n_slices >= 1 required");
    TVS_REQUIRE(P->step > 0 && std::isfinite(P->step), TVS_ERR_INVALID_ARG, "step > 0 required");
    TVS_REQUIRE(P->outer_iters >= 0 && P->inner_iters >= 1 && P->k0 >= 0, TVS_ERR_INVALID_ARG,
                "outer_iters >= 0, inner_iters >= 1, k0 >= 0 required");
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) {
        order[i] = i;
        TVS_REQUIRE(S[i].H >= 1 && S[i].W >= 1 && S[i].offset >= 0, TVS_ERR_SHAPE,
                    "slice sizes >= 1 and offsets >= 0 required");
        TVS_REQUIRE(S[i].p > 0 && S[i].p <= 1, TVS_ERR_INVALID_ARG, "slice p must be in (0, 1]");
        TVS_REQUIRE(S[i].alpha >= 0 && std::isfinite(S[i].alpha), TVS_ERR_INVALID_ARG,
                    "slice alpha >= 0 required");
    }
    std::sort(order.begin(), order.end(), [&](int a, int c) { return S[a].offset < S[c].offset; });
    size_t total = 0;
    for (int k = 0; k < n; ++k) {
        const tvs_slice& s = S[order[k]];
        TVS_REQUIRE((size_t)s.offset >= total, TVS_ERR_SHAPE, "slices overlap in the pools");
        total = (size_t)s.offset + (size_t)s.H * s.W;
    }
    const int64_t K = P->outer_iters;
    const double step = P->step;
    FgpConfig cfg;
    if (P->fgp_variant >= 0) {
        TVS_REQUIRE(P->fgp_variant < fgp_variant_count(), TVS_ERR_INVALID_ARG, "bad FGP variant");
        cfg = fgp_variant(P->fgp_variant);
    } else {
        cfg = fgp_config_batched(ctx, n, (int)sizeof(T));
    }

    // --------------------------------------------------------------- plan
    Plan pl;
    pl.theta.resize((size_t)K * n);
    pl.nprox.assign(n, 0);
    for (int64_t kk = 0; kk < K; ++kk)
        for (int s = 0; s < n; ++s) {
            const int th = coin(S[s].seed, S[s].stream_id, P->k0 + kk, S[s].p);
            pl.theta[(size_t)kk * n + s] = (uint8_t)th;
            pl.nprox[s] += th;
        }
    pl.pref_all.assign(n + 1, 0);
    for (int s = 0; s < n; ++s) pl.pref_all[s + 1] = pl.pref_all[s] + tiles_of(S[s].H, S[s].W, 32, 32);
    for (int64_t kk = 0; kk < K; ++kk) {
        std::vector<int> act;
        for (int s = 0; s < n; ++s)
            if (pl.theta[(size_t)kk * n + s]) act.push_back(s);
        pl.it_off.push_back(pl.ints.size());
        pl.n_act.push_back((int)act.size());
        pl.ints.insert(pl.ints.end(), act.begin(), act.end());
        int cf = 0, cn = 0;
        pl.ints.push_back(0);
        for (int s : act) pl.ints.push_back(cf += tiles_of(S[s].H, S[s].W, cfg.tile_w, cfg.tile_h));
        pl.ints.push_back(0);
        for (int s : act) pl.ints.push_back(cn += tiles_of(S[s].H, S[s].W, 32, 32));
        pl.tiles_fgp.push_back(cf);
        pl.tiles_fin.push_back(cn);
    }
    std::vector<BSlice<T>> hs(n);
    for (int s = 0; s < n; ++s) {
        hs[s].H = S[s].H;
        hs[s].W = S[s].W;
        hs[s].off = S[s].offset;
        hs[s].lam = (T)(S[s].alpha * step / S[s].p);
        hs[s].coef = (T)(step - step / S[s].p);
        hs[s].rate = (T)(S[s].p / step);
    }

    // ---------------------------------------------- device tables, scratch
    BSlice<T>* d_sl = (BSlice<T>*)scratch(ctx, S_BSL, n * sizeof(BSlice<T>));
    int* d_pref = (int*)scratch(ctx, S_BPREF, (n + 1) * sizeof(int));
    int* d_list = (int*)scratch(ctx, S_BLIST, std::max<size_t>(pl.ints.size(), 1) * sizeof(int));
    uint8_t* d_th = (uint8_t*)scratch(ctx, S_BTHETA, std::max<size_t>(pl.theta.size(), 1));
    T* xhat = (T*)scratch(ctx, S_XHAT, total * sizeof(T));
    T* v = (T*)scratch(ctx, S_V, total * sizeof(T));
    scratch(ctx, S_Q1, 2 * total * sizeof(T));
    scratch(ctx, S_Q2, 2 * total * sizeof(T));
    scratch(ctx, S_Q3, 2 * total * sizeof(T));
    beta_table_dev<T>(ctx, P->inner_iters + 1);
    // The tables are rewritten in place: wait until launches of an earlier
    // call on this stream (which may still read them) have finished.  A copy
    // from pageable memory is not ordered after work on a non-blocking stream.
    TVS_HIP(hipStreamSynchronize(ctx->stream));
    TVS_HIP(hipMemcpy(d_sl, hs.data(), n * sizeof(BSlice<T>), hipMemcpyHostToDevice));
    TVS_HIP(hipMemcpy(d_pref, pl.pref_all.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice));
    if (!pl.ints.empty())
        TVS_HIP(hipMemcpy(d_list, pl.ints.data(), pl.ints.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!pl.theta.empty())
        TVS_HIP(hipMemcpy(d_th, pl.theta.data(), pl.theta.size(), hipMemcpyHostToDevice));

    // -------------------------------------------------------------- enqueue
    auto enqueue = [&] {
        for (int64_t kk = 0; kk < K; ++kk) {
            launch_identity_step_batched<T>(ctx, d_sl, d_pref, n, pl.pref_all[n],
                                            d_th + (size_t)kk * n, b, x, h, xhat, v, (T)step);
            if (pl.n_act[kk] == 0) continue;
            BatchLists L;
            const int* base = d_list + pl.it_off[kk];
            L.n_act = pl.n_act[kk];
            L.act = base;
            L.pref_fgp = base + L.n_act;
            L.pref_fin = base + 2 * L.n_act + 1;
            L.tiles_fgp = pl.tiles_fgp[kk];
            L.tiles_fin = pl.tiles_fin[kk];
            T* qf = run_fgp_batched<T>(ctx, d_sl, L, v, q, total, P->inner_iters, P->nonneg, cfg);
            launch_finalize_batched<T>(ctx, d_sl, L, v, qf, q, x, h, xhat, P->nonneg);
        }
    };
    if ((P->flags & TVS_FLAG_GRAPH) && K > 0) {
        // key: pools, scalars, and a digest of the slice table and coin plan
        uint64_t hsh = 1469598103934665603ULL;
        auto mixin = [&](uint64_t v) { hsh = (hsh ^ v) * 1099511628211ULL; };
        for (int s = 0; s < n; ++s) {
            mixin((uint64_t)S[s].H);
            mixin((uint64_t)S[s].W);
            mixin((uint64_t)S[s].offset);
            uint64_t a, p;
            std::memcpy(&a, &S[s].alpha, 8);
            std::memcpy(&p, &S[s].p, 8);
            mixin(a);
            mixin(p);
            mixin(S[s].seed);
            mixin(S[s].stream_id);
        }
        uint64_t st;
        std::memcpy(&st, &step, 8);
        std::vector<uint64_t> key = {0xBA7C4ULL, (uint64_t)sizeof(T), (uint64_t)(uintptr_t)b,
                                     (uint64_t)(uintptr_t)x, (uint64_t)(uintptr_t)h,
                                     (uint64_t)(uintptr_t)q, st, (uint64_t)K,
                                     (uint64_t)P->inner_iters, (uint64_t)P->nonneg,
                                     (uint64_t)P->k0, (uint64_t)cfg.tile_w, (uint64_t)cfg.tile_h,
                                     (uint64_t)cfg.steps, (uint64_t)n, hsh};
        graph_run_key(ctx, key, enqueue);
    } else {
        enqueue();
    }
    if (nprox_out)
        for (int s = 0; s < n; ++s) nprox_out[s] = pl.nprox[s];
}

// Times every compiled FGP variant on one FGP pass over the whole batch
// (every slice active), on private pools with seeded random data laid out
// back to back; keeps the fastest for this slice count.
template <typename T>
void autotune_batched(tvs_ctx* ctx, int n, const tvs_slice* S, int iters, int reps, int* best,
                      double* ms_out) {
    TVS_REQUIRE(n >= 1, TVS_ERR_SHAPE, "n_slices >= 1 required");
    std::vector<BSlice<T>> hs(n);
    size_t total = 0;
    for (int s = 0; s < n; ++s) {
        TVS_REQUIRE(S[s].H >= 1 && S[s].W >= 1, TVS_ERR_SHAPE, "slice sizes >= 1 required");
        TVS_REQUIRE(S[s].p > 0 && S[s].p <= 1 && S[s].alpha >= 0, TVS_ERR_INVALID_ARG,
                    "slice p in (0, 1] and alpha >= 0 required");
        hs[s].H = S[s].H;
        hs[s].W = S[s].W;
        hs[s].off = (int64_t)total;
        hs[s].lam = (T)(S[s].alpha / S[s].p);
        hs[s].coef = T(0);
        hs[s].rate = T(1);
        total += (size_t)S[s].H * S[s].W;
    }
    std::vector<T> hv(total);
    for (size_t i = 0; i < total; ++i)
        hv[i] = (T)((double)(splitmix_mix(i + 7) >> 11) * (1.0 / 9007199254740992.0));
    struct Tmp {
        std::vector<void*> ptrs;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Tmp() {
            for (void* p : ptrs) (void)hipFree(p);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
        void* alloc(size_t bytes) {
            void* p = nullptr;
            TVS_HIP(hipMalloc(&p, bytes));
            ptrs.push_back(p);
            return p;
        }
    } tmp;
    // The slices a prox call of the run actually covers: those whose coin is
    // 1 at each of the first kProbe outer iterations (k0 = 0), so that the
    // variant is chosen for the active sets the solve will see (a fraction p
    // of the slices), not for all slices at once.  With no active slice in
    // those iterations, every slice.
    constexpr int kProbe = 8;
    std::vector<std::vector<int>> sets;
    for (int k = 0; k < kProbe; ++k) {
        std::vector<int> a;
        for (int s = 0; s < n; ++s)
            if (coin(S[s].seed, S[s].stream_id, k, S[s].p) == 1) a.push_back(s);
        if (!a.empty()) sets.push_back(std::move(a));
    }
    if (sets.empty()) {
        sets.emplace_back();
        for (int s = 0; s < n; ++s) sets.back().push_back(s);
    }
    const int n_sets = (int)sets.size();
    T* v = (T*)tmp.alloc(total * sizeof(T));
    T* q = (T*)tmp.alloc(2 * total * sizeof(T));
    BSlice<T>* d_sl = (BSlice<T>*)tmp.alloc(n * sizeof(BSlice<T>));
    int* d_list = (int*)tmp.alloc((size_t)n_sets * (3 * n + 2) * sizeof(int));
    TVS_HIP(hipMemcpy(v, hv.data(), total * sizeof(T), hipMemcpyHostToDevice));
    TVS_HIP(hipMemcpy(d_sl, hs.data(), n * sizeof(BSlice<T>), hipMemcpyHostToDevice));
    TVS_HIP(hipEventCreate(&tmp.e0));
    TVS_HIP(hipEventCreate(&tmp.e1));
    scratch(ctx, S_Q1, 2 * total * sizeof(T));
    scratch(ctx, S_Q2, 2 * total * sizeof(T));
    scratch(ctx, S_Q3, 2 * total * sizeof(T));
    beta_table_dev<T>(ctx, iters + 1);
    double best_ms = 1e300;
    int best_i = -1;
    for (int vi = 0; vi < fgp_variant_count(); ++vi) {
        const FgpConfig c = fgp_variant(vi);
        if (find_variant_index(c, (int)sizeof(T)) < 0) {
            if (ms_out) ms_out[vi] = -1.0;
            continue;
        }
        // one work list per active set: act, FGP tile prefix, 32 x 32 prefix
        std::vector<BatchLists> Ls(n_sets);
        std::vector<int> ints((size_t)n_sets * (3 * n + 2), 0);
        for (int j = 0; j < n_sets; ++j) {
            const std::vector<int>& a = sets[j];
            const int na = (int)a.size();
            int* li = ints.data() + (size_t)j * (3 * n + 2);
            int cf = 0, cn = 0;
            for (int t = 0; t < na; ++t) li[t] = a[t];
            li[na] = 0;
            for (int t = 0; t < na; ++t)
                li[na + 1 + t] = cf += tiles_of(S[a[t]].H, S[a[t]].W, c.tile_w, c.tile_h);
            li[2 * na + 1] = 0;
            for (int t = 0; t < na; ++t) li[2 * na + 2 + t] = cn += tiles_of(S[a[t]].H, S[a[t]].W, 32, 32);
            int* dl = d_list + (size_t)j * (3 * n + 2);
            Ls[j].n_act = na;
            Ls[j].act = dl;
            Ls[j].pref_fgp = dl + na;
            Ls[j].pref_fin = dl + 2 * na + 1;
            Ls[j].tiles_fgp = cf;
            Ls[j].tiles_fin = cn;
        }
        TVS_HIP(hipMemcpy(d_list, ints.data(), ints.size() * sizeof(int), hipMemcpyHostToDevice));
        launch_fill<T>(ctx, 2 * total, T(0), q);
        for (const BatchLists& L : Ls) run_fgp_batched<T>(ctx, d_sl, L, v, q, total, iters, 0, c);  // warm-up
        TVS_HIP(hipEventRecord(tmp.e0, ctx->stream));
        for (int r = 0; r < reps; ++r)
            for (const BatchLists& L : Ls) run_fgp_batched<T>(ctx, d_sl, L, v, q, total, iters, 0, c);
        TVS_HIP(hipEventRecord(tmp.e1, ctx->stream));
        TVS_HIP(hipEventSynchronize(tmp.e1));
        float ms = 0;
        TVS_HIP(hipEventElapsedTime(&ms, tmp.e0, tmp.e1));
        // time per FGP iteration of one prox call of the run (an average active set)
        const double per_iter = (double)ms / ((double)reps * iters * n_sets);
        if (ms_out) ms_out[vi] = per_iter;
        if (per_iter < best_ms) {
            best_ms = per_iter;
            best_i = vi;
        }
    }
    TVS_HIP(hipStreamSynchronize(ctx->stream));
    TuneEntry e;
    e.cfg = fgp_variant(best_i);
    e.ms_per_iter = best_ms;
    ctx->fgp_tuned[tune_key(TK_BATCH, n, 0, (int)sizeof(T))] = e;
    if (best) *best = best_i;
}

}  // namespace

extern "C" tvs_status tvs_fgp_autotune_batched(tvs_ctx* ctx, tvs_dtype dtype, int n_slices,
                                               const tvs_slice* slices, int inner_iters, int reps,
                                               int* best_index, double* ms_per_iter_out) {
    try {
        TVS_REQUIRE(ctx && slices, TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(dtype == TVS_F32 || dtype == TVS_F64, TVS_ERR_INVALID_ARG, "bad dtype");
        TVS_REQUIRE(inner_iters >= 1 && reps >= 1, TVS_ERR_INVALID_ARG, "inner_iters, reps >= 1");
        TVS_HIP(hipSetDevice(ctx->device));
        if (dtype == TVS_F32)
            autotune_batched<float>(ctx, n_slices, slices, inner_iters, reps, best_index,
                                    ms_per_iter_out);
        else
            autotune_batched<double>(ctx, n_slices, slices, inner_iters, reps, best_index,
                                     ms_per_iter_out);
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

extern "C" tvs_status tvs_proxskip_batched(tvs_ctx* ctx, tvs_dtype dtype, int n_slices,
                                           const tvs_slice* slices, const void* b_pool,
                                           void* x_pool, void* h_pool, void* q_pool,
                                           const tvs_batch_params* params, int64_t* n_prox_out) {
    try {
        TVS_REQUIRE(ctx && slices && b_pool && x_pool && h_pool && q_pool && params,
                    TVS_ERR_INVALID_ARG, "null pointer");
        TVS_REQUIRE(dtype == TVS_F32 || dtype == TVS_F64, TVS_ERR_INVALID_ARG, "bad dtype");
        TVS_HIP(hipSetDevice(ctx->device));
        if (dtype == TVS_F32)
            run_batched<float>(ctx, n_slices, slices, (const float*)b_pool, (float*)x_pool,
                               (float*)h_pool, (float*)q_pool, params, n_prox_out);
        else
            run_batched<double>(ctx, n_slices, slices, (const double*)b_pool, (double*)x_pool,
                                (double*)h_pool, (double*)q_pool, params, n_prox_out);
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

extern "C" tvs_status tvs_fgp_set_variant_batched(tvs_ctx* ctx, tvs_dtype dtype, int n_slices,
                                                  int index) {
    if (!ctx || (dtype != TVS_F32 && dtype != TVS_F64) || index < -1 ||
        index >= fgp_variant_count() || n_slices < 1) {
        set_error("bad context, dtype, slice count or variant index");
        return TVS_ERR_INVALID_ARG;
    }
    const int bytes = dtype == TVS_F32 ? 4 : 8;
    if (index < 0) {
        ctx->fgp_tuned.erase(tune_key(TK_BATCH, n_slices, 0, bytes));
        return TVS_OK;
    }
    FgpConfig c = fgp_variant(index);
    if (find_variant_index(c, bytes) < 0) {
        set_error("variant not compiled for float64");
        return TVS_ERR_UNSUPPORTED;
    }
    TuneEntry e;
    e.cfg = c;
    ctx->fgp_tuned[tune_key(TK_BATCH, n_slices, 0, bytes)] = e;
    return TVS_OK;
}
