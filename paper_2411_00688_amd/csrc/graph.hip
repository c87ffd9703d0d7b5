// HIP-graph capture of a solver run.  The coin schedule is known on the host,
// so a whole run (every data step, FGP launch and dual step) is one fixed
// sequence of kernels; capturing it turns thousands of launches into one
// graph launch.  Graphs are cached per context under the full call key
// (operator, buffers, dtype and every parameter), so an identical later call
// relaunches the instantiated graph.
#include "tvs_internal.hpp"

namespace tvs {

struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static uint64_t bits(double d) {
    uint64_t u;
    std::memcpy(&u, &d, sizeof(u));
    return u;
}

std::vector<uint64_t> graph_key(const tvs_op* op, bool pdhg, int dtype, const void* b,
                                      const tvs_state* st, const tvs_params* P) {
    return {(uint64_t)(uintptr_t)op, (uint64_t)pdhg, (uint64_t)dtype, (uint64_t)(uintptr_t)b,
            (uint64_t)(uintptr_t)st->x, (uint64_t)(uintptr_t)st->h, (uint64_t)(uintptr_t)st->q,
            (uint64_t)(uintptr_t)st->y, bits(P->alpha), bits(P->step), bits(P->dual_step),
            bits(P->p), (uint64_t)P->outer_iters, (uint64_t)P->inner_iters, (uint64_t)P->nonneg,
            P->seed, P->stream_id, (uint64_t)P->k0, (uint64_t)P->flags};
}

static void destroy_entry(GraphEntry* e) {
    if (e->exec) hipGraphExecDestroy(e->exec);
    if (e->graph) hipGraphDestroy(e->graph);
    delete e;
}

void graph_cache_clear(tvs_ctx* ctx) {
    for (GraphEntry* e : ctx->graphs) destroy_entry(e);
    ctx->graphs.clear();
}

void graph_run(tvs_ctx* ctx, const tvs_op* op, bool pdhg, int dtype, const void* b,
               const tvs_state* st, const tvs_params* P, const std::function<void()>& enqueue) {
    graph_run_key(ctx, graph_key(op, pdhg, dtype, b, st, P), enqueue);
}

void graph_run_key(tvs_ctx* ctx, const std::vector<uint64_t>& key,
                   const std::function<void()>& enqueue) {
    for (GraphEntry* e : ctx->graphs) {
        if (e->key == key) {
            TVS_HIP(hipGraphLaunch(e->exec, ctx->stream));
            return;
        }
    }
    hipStream_t cap = nullptr;
    TVS_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipStream_t saved = ctx->stream;
    ctx->stream = cap;
    hipGraph_t graph = nullptr;
    hipError_t err = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) {
        ctx->stream = saved;
        hipStreamDestroy(cap);
        TVS_HIP(err);
    }
    try {
        enqueue();
    } catch (...) {
        hipStreamEndCapture(cap, &graph);
        if (graph) hipGraphDestroy(graph);
        ctx->stream = saved;
        hipStreamDestroy(cap);
        throw;
    }
    err = hipStreamEndCapture(cap, &graph);
    ctx->stream = saved;
    hipStreamDestroy(cap);
    TVS_HIP(err);
    auto* e = new GraphEntry();
    e->key = key;
    e->graph = graph;
    err = hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        destroy_entry(e);
        TVS_HIP(err);
    }
    const size_t kMaxGraphs = 8;
    if (ctx->graphs.size() >= kMaxGraphs) {
        TVS_HIP(hipStreamSynchronize(ctx->stream));
        destroy_entry(ctx->graphs.front());
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back(e);
    TVS_HIP(hipGraphLaunch(e->exec, ctx->stream));
}

}  // namespace tvs
