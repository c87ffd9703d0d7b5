// FGP tile / temporal-depth autotuner.  Every compiled variant (output tile
// BW x BH, TS fused iterations per launch, 256 threads) is timed with HIP
// events on a seeded random image of the requested size; the fastest is kept
// in the context for that exact size and for its size class (each side
// rounded up to a power of two), and used by every later prox evaluation of
// a matching size.  The table can be saved to and loaded from a JSON file,
// keyed by the GPU architecture.
#include <cmath>
#include <cstdio>
#include <fstream>
#include <sstream>

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

static tvs_status fail(tvs_status st, const char* msg) {
    set_error(msg);
    return st;
}

template <typename F>
static tvs_status guarded_tune(F&& f) {
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

extern "C" tvs_status tvs_fgp_set_variant(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, int index) {
    if (!ctx || (dtype != TVS_F32 && dtype != TVS_F64) || index < -1 ||
        index >= fgp_variant_count() || H < 1 || W < 1)
        return fail(TVS_ERR_INVALID_ARG, "bad context, dtype, size or variant index");
    const int bytes = dtype == TVS_F32 ? 4 : 8;
    if (index < 0) {
        ctx->fgp_tuned.erase(tune_key(TK_IMAGE, H, W, bytes));
        return TVS_OK;
    }
    TuneEntry e;
    e.cfg = fgp_variant(index);
    if (find_variant_index(e.cfg, bytes) < 0)
        return fail(TVS_ERR_UNSUPPORTED, "variant not compiled for float64");
    ctx->fgp_tuned[tune_key(TK_IMAGE, H, W, bytes)] = e;
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
        // Three rounds over all variants, each variant's best round kept:
        // interleaving the rounds spreads clock ramps and neighbours' noise
        // over every variant instead of charging it to the first ones.
        const int nv = fgp_variant_count();
        std::vector<double> t(nv, 1e300);
        for (int round = 0; round < 3; ++round) {
            for (int vi = 0; vi < nv; ++vi) {
                FgpConfig c = fgp_variant(vi);
                if (find_variant_index(c, (int)sizeof(T)) < 0) continue;
                launch_fill<T>(ctx, 2 * n, T(0), q);
                run_fgp<T>(ctx, H, W, v, 0.1, iters, 0, q, c);  // warm-up
                TVS_HIP(hipEventRecord(e0, ctx->stream));
                for (int r = 0; r < reps; ++r) run_fgp<T>(ctx, H, W, v, 0.1, iters, 0, q, c);
                TVS_HIP(hipEventRecord(e1, ctx->stream));
                TVS_HIP(hipEventSynchronize(e1));
                float ms = 0;
                TVS_HIP(hipEventElapsedTime(&ms, e0, e1));
                const double per_iter = (double)ms / ((double)reps * iters);
                if (per_iter < t[vi]) t[vi] = per_iter;
            }
        }
        for (int vi = 0; vi < nv; ++vi) {
            const bool ok = find_variant_index(fgp_variant(vi), (int)sizeof(T)) >= 0;
            if (ms_out) ms_out[vi] = ok ? t[vi] : -1.0;
            if (ok && t[vi] < best_ms) {
                best_ms = t[vi];
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
    TuneEntry e;
    e.cfg = fgp_variant(best_i);
    e.ms_per_iter = best_ms;
    ctx->fgp_tuned[tune_key(TK_IMAGE, H, W, (int)sizeof(T))] = e;
    ctx->fgp_tuned[tune_key(TK_CLASS, size_class(H), size_class(W), (int)sizeof(T))] = e;
    if (best) *best = best_i;
}

}  // namespace

extern "C" tvs_status tvs_fgp_autotune(tvs_ctx* ctx, tvs_dtype dtype, int H, int W,
                                       int inner_iters, int reps, int* best_index,
                                       double* ms_per_iter_out) {
    return guarded_tune([&] {
        TVS_REQUIRE(ctx, TVS_ERR_INVALID_ARG, "null context");
        TVS_REQUIRE(dtype == TVS_F32 || dtype == TVS_F64, TVS_ERR_INVALID_ARG, "bad dtype");
        TVS_REQUIRE(H >= 1 && W >= 1, TVS_ERR_SHAPE, "bad size");
        TVS_REQUIRE(inner_iters >= 1 && reps >= 1, TVS_ERR_INVALID_ARG, "inner_iters, reps >= 1");
        TVS_HIP(hipSetDevice(ctx->device));
        if (dtype == TVS_F32)
            autotune<float>(ctx, H, W, inner_iters, reps, best_index, ms_per_iter_out);
        else
            autotune<double>(ctx, H, W, inner_iters, reps, best_index, ms_per_iter_out);
    });
}

static void query_out(tvs_ctx* ctx, uint64_t key, const FgpConfig& c, int bytes, int* index,
                      double* ms) {
    *index = find_variant_index(c, bytes);
    if (ms) {
        auto it = ctx->fgp_tuned.find(key);
        *ms = it != ctx->fgp_tuned.end() ? it->second.ms_per_iter : -1.0;
    }
}

extern "C" tvs_status tvs_fgp_query(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, int* index,
                                    double* ms_per_iter) {
    if (!ctx || (dtype != TVS_F32 && dtype != TVS_F64) || H < 1 || W < 1 || !index)
        return fail(TVS_ERR_INVALID_ARG, "bad context, dtype, size or null output");
    const int bytes = dtype == TVS_F32 ? 4 : 8;
    const FgpConfig c = fgp_config(ctx, H, W, bytes);
    uint64_t key = tune_key(TK_IMAGE, H, W, bytes);
    if (!ctx->fgp_tuned.count(key)) key = tune_key(TK_CLASS, size_class(H), size_class(W), bytes);
    query_out(ctx, key, c, bytes, index, ms_per_iter);
    return TVS_OK;
}

extern "C" tvs_status tvs_fgp_query_batched(tvs_ctx* ctx, tvs_dtype dtype, int n_slices,
                                            int* index, double* ms_per_iter) {
    if (!ctx || (dtype != TVS_F32 && dtype != TVS_F64) || n_slices < 1 || !index)
        return fail(TVS_ERR_INVALID_ARG, "bad context, dtype, slice count or null output");
    const int bytes = dtype == TVS_F32 ? 4 : 8;
    query_out(ctx, tune_key(TK_BATCH, n_slices, 0, bytes), fgp_config_batched(ctx, n_slices, bytes),
              bytes, index, ms_per_iter);
    return TVS_OK;
}

extern "C" tvs_status tvs_tune_clear(tvs_ctx* ctx) {
    if (!ctx) return fail(TVS_ERR_INVALID_ARG, "null context");
    ctx->fgp_tuned.clear();
    return TVS_OK;
}

// ------------------------------------------------------------ tuning files
namespace {

const char* kFormat = "tvskip-fgp-tune/1";
const char* kKinds[3] = {"image", "class", "batch"};

std::string device_arch(tvs_ctx* ctx) {
    hipDeviceProp_t prop;
    TVS_HIP(hipGetDeviceProperties(&prop, ctx->device));
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// A JSON value: enough of the grammar for the tuning file (objects, arrays,
// strings without escapes other than \" and \\, numbers, true/false/null).
struct JVal {
    enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
    double num = 0;
    bool b = false;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal* get(const std::string& k) const {
        for (const auto& kv : obj)
            if (kv.first == k) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const std::string& s;
    size_t i = 0;
    explicit JParser(const std::string& text) : s(text) {}
    [[noreturn]] void bad(const char* what) {
        throw Error{TVS_ERR_INVALID_ARG, std::string("tuning file: ") + what + " at byte " +
                                             std::to_string(i)};
    }
    void ws() {
        while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\t' || s[i] == '\r')) ++i;
    }
    bool lit(const char* w) {
        const size_t n = std::strlen(w);
        if (s.compare(i, n, w) == 0) {
            i += n;
            return true;
        }
        return false;
    }
    std::string string() {
        if (i >= s.size() || s[i] != '"') bad("expected a string");
        ++i;
        std::string out;
        while (i < s.size() && s[i] != '"') {
            if (s[i] == '\\') {
                if (i + 1 >= s.size() || (s[i + 1] != '"' && s[i + 1] != '\\')) bad("escape");
                ++i;
            }
            out.push_back(s[i++]);
        }
        if (i >= s.size()) bad("unterminated string");
        ++i;
        return out;
    }
    JVal value(int depth) {
        if (depth > 16) bad("nesting too deep");
        ws();
        JVal v;
        if (i >= s.size()) bad("unexpected end");
        const char c = s[i];
        if (c == '{') {
            v.kind = JVal::OBJ;
            ++i;
            ws();
            if (i < s.size() && s[i] == '}') {
                ++i;
                return v;
            }
            for (;;) {
                ws();
                std::string k = string();
                ws();
                if (i >= s.size() || s[i] != ':') bad("expected ':'");
                ++i;
                v.obj.emplace_back(k, value(depth + 1));
                ws();
                if (i < s.size() && s[i] == ',') { ++i; continue; }
                if (i < s.size() && s[i] == '}') { ++i; break; }
                bad("expected ',' or '}'");
            }
        } else if (c == '[') {
            v.kind = JVal::ARR;
            ++i;
            ws();
            if (i < s.size() && s[i] == ']') {
                ++i;
                return v;
            }
            for (;;) {
                v.arr.push_back(value(depth + 1));
                ws();
                if (i < s.size() && s[i] == ',') { ++i; continue; }
                if (i < s.size() && s[i] == ']') { ++i; break; }
                bad("expected ',' or ']'");
            }
        } else if (c == '"') {
            v.kind = JVal::STR;
            v.str = string();
        } else if (lit("true")) {
            v.kind = JVal::BOOL;
            v.b = true;
        } else if (lit("false")) {
            v.kind = JVal::BOOL;
        } else if (lit("null")) {
            v.kind = JVal::NUL;
        } else {
            const char* begin = s.c_str() + i;
            char* end = nullptr;
            v.num = std::strtod(begin, &end);
            if (end == begin) bad("expected a value");
            v.kind = JVal::NUM;
            i += (size_t)(end - begin);
        }
        return v;
    }
};

int int_field(const JVal& e, const char* k) {
    const JVal* v = e.get(k);
    if (!v || v->kind != JVal::NUM || v->num != std::floor(v->num) || v->num < 0 ||
        v->num > 2147483647.0)
        throw Error{TVS_ERR_INVALID_ARG, std::string("tuning file: entry field ") + k +
                                             " missing or not a non-negative integer"};
    return (int)v->num;
}

}  // namespace

extern "C" tvs_status tvs_tune_save(tvs_ctx* ctx, const char* path) {
    return guarded_tune([&] {
        TVS_REQUIRE(ctx && path, TVS_ERR_INVALID_ARG, "null argument");
        std::ostringstream o;
        o.precision(17);
        o << "{\n  \"format\": \"" << kFormat << "\",\n  \"arch\": \"" << device_arch(ctx)
          << "\",\n  \"entries\": [";
        bool first = true;
        for (const auto& kv : ctx->fgp_tuned) {
            const uint64_t k = kv.first;
            const int bytes = (int)(k & 15), kind = (int)((k >> 4) & 3);
            const int b = (int)((k >> 6) & 0xFFFFFFFULL), a = (int)(k >> 34);
            const TuneEntry& e = kv.second;
            o << (first ? "\n" : ",\n") << "    {\"kind\": \"" << kKinds[kind] << "\", \"dtype\": \""
              << (bytes == 4 ? "f32" : "f64") << "\", ";
            if (kind == TK_BATCH)
                o << "\"n_slices\": " << a;
            else
                o << "\"H\": " << a << ", \"W\": " << b;
            o << ", \"tile_w\": " << e.cfg.tile_w << ", \"tile_h\": " << e.cfg.tile_h
              << ", \"steps\": " << e.cfg.steps << ", \"ms_per_iter\": " << e.ms_per_iter << "}";
            first = false;
        }
        o << (first ? "]\n}\n" : "\n  ]\n}\n");
        const std::string tmp = std::string(path) + ".tmp";
        {
            std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
            TVS_REQUIRE(f.good(), TVS_ERR_INVALID_ARG, std::string("cannot write ") + tmp);
            f << o.str();
            f.close();
            TVS_REQUIRE(f.good(), TVS_ERR_DEVICE, std::string("write failed: ") + tmp);
        }
        TVS_REQUIRE(std::rename(tmp.c_str(), path) == 0, TVS_ERR_DEVICE,
                    std::string("cannot rename to ") + path);
    });
}

extern "C" tvs_status tvs_tune_load(tvs_ctx* ctx, const char* path) {
    return guarded_tune([&] {
        TVS_REQUIRE(ctx && path, TVS_ERR_INVALID_ARG, "null argument");
        std::ifstream f(path, std::ios::binary);
        TVS_REQUIRE(f.good(), TVS_ERR_INVALID_ARG, std::string("cannot open ") + path);
        std::stringstream ss;
        ss << f.rdbuf();
        const std::string text = ss.str();
        TVS_REQUIRE(text.size() < (1u << 24), TVS_ERR_INVALID_ARG, "tuning file too large");
        JParser P(text);
        const JVal root = P.value(0);
        P.ws();
        if (P.i != text.size()) P.bad("trailing data");
        TVS_REQUIRE(root.kind == JVal::OBJ, TVS_ERR_INVALID_ARG, "tuning file: not an object");
        const JVal* fmt = root.get("format");
        TVS_REQUIRE(fmt && fmt->kind == JVal::STR && fmt->str == kFormat, TVS_ERR_INVALID_ARG,
                    "tuning file: unknown format");
        const JVal* arch = root.get("arch");
        TVS_REQUIRE(arch && arch->kind == JVal::STR, TVS_ERR_INVALID_ARG, "tuning file: no arch");
        TVS_REQUIRE(arch->str == device_arch(ctx), TVS_ERR_UNSUPPORTED,
                    "tuning file was made on " + arch->str + ", this device is " + device_arch(ctx));
        const JVal* ents = root.get("entries");
        TVS_REQUIRE(ents && ents->kind == JVal::ARR, TVS_ERR_INVALID_ARG, "tuning file: no entries");
        std::map<uint64_t, TuneEntry> add;  // validate everything before changing the context
        for (const JVal& e : ents->arr) {
            TVS_REQUIRE(e.kind == JVal::OBJ, TVS_ERR_INVALID_ARG, "tuning file: entry not an object");
            const JVal* kind = e.get("kind");
            const JVal* dt = e.get("dtype");
            TVS_REQUIRE(kind && kind->kind == JVal::STR && dt && dt->kind == JVal::STR,
                        TVS_ERR_INVALID_ARG, "tuning file: entry without kind or dtype");
            int kd = -1;
            for (int k = 0; k < 3; ++k)
                if (kind->str == kKinds[k]) kd = k;
            TVS_REQUIRE(kd >= 0, TVS_ERR_INVALID_ARG, "tuning file: unknown kind " + kind->str);
            TVS_REQUIRE(dt->str == "f32" || dt->str == "f64", TVS_ERR_INVALID_ARG,
                        "tuning file: dtype must be f32 or f64");
            const int bytes = dt->str == "f32" ? 4 : 8;
            TuneEntry te;
            te.cfg.tile_w = int_field(e, "tile_w");
            te.cfg.tile_h = int_field(e, "tile_h");
            te.cfg.steps = int_field(e, "steps");
            TVS_REQUIRE(find_variant_index(te.cfg, bytes) >= 0, TVS_ERR_UNSUPPORTED,
                        "tuning file: FGP variant not compiled in this library");
            const JVal* ms = e.get("ms_per_iter");
            if (ms && ms->kind == JVal::NUM) te.ms_per_iter = ms->num;
            uint64_t key;
            if (kd == TK_BATCH) {
                const int ns = int_field(e, "n_slices");
                TVS_REQUIRE(ns >= 1, TVS_ERR_INVALID_ARG, "tuning file: n_slices >= 1");
                key = tune_key(TK_BATCH, ns, 0, bytes);
            } else {
                const int H = int_field(e, "H"), W = int_field(e, "W");
                TVS_REQUIRE(H >= 1 && W >= 1 && H < (1 << 28) && W < (1 << 28), TVS_ERR_INVALID_ARG,
                            "tuning file: bad image size");
                key = tune_key(kd, H, W, bytes);
            }
            add[key] = te;
        }
        for (const auto& kv : add) ctx->fgp_tuned[kv.first] = kv.second;
    });
}
