// Internal declarations of the gfx950 TV-skip library: context, operators,
// scratch memory and the host-side launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/tvskip.h"

namespace tvs {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);

struct Error {
    tvs_status status;
    std::string msg;
};

#define TVS_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess)                                                  \
            throw ::tvs::Error{e_ == hipErrorOutOfMemory ? TVS_ERR_OOM          \
                                                         : TVS_ERR_DEVICE,     \
                               std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define TVS_LAUNCH_CHECK() TVS_HIP(hipGetLastError())

#define TVS_REQUIRE(cond, st, msg)                                             \
    do {                                                                       \
        if (!(cond)) throw ::tvs::Error{(st), (msg)};                          \
    } while (0)

// ------------------------------------------------------------------ scratch
// Grow-only device buffers owned by the context, one per named slot.  A slot
// is never shrunk, so pointers stay valid until the slot grows.
struct Scratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};

enum Slot : int {
    S_XHAT = 0, S_V, S_XBAR, S_XBART, S_Q1, S_Q2, S_Q3, S_RES, S_TMP, S_BETAF,
    S_PART, S_RED, S_BETA, S_Z, S_NORMV, S_OBJ, S_TR_IMG, S_PARTIMG, S_XBARP, S_XBARTP,
    S_PADX, S_BSL, S_BLIST, S_BTHETA, S_BPREF, S_GATE, S_QNET, S_SEL,
    S_SB, S_SY, S_SDY, S_SZ, S_SZB, S_FX1, S_FX2, S_HZERO, S_COUNT
};

struct GraphEntry;

struct FgpConfig {
    int tile_w = 32, tile_h = 32, steps = 4;
};

// Autotuner entries: per exact image size, per size class (each side rounded
// up to a power of two, at least 16) and per batched slice count.
enum TuneKind : int { TK_IMAGE = 0, TK_CLASS = 1, TK_BATCH = 2 };

struct TuneEntry {
    FgpConfig cfg;
    double ms_per_iter = -1.0;  // measured time per FGP iteration, -1 if set by hand
};

inline uint64_t tune_key(int kind, int a, int b, int dtype_bytes) {
    return ((uint64_t)(uint32_t)a << 34) | ((uint64_t)(uint32_t)b << 6) |
           ((uint64_t)(uint32_t)kind << 4) | (uint64_t)(uint32_t)dtype_bytes;
}

inline int size_class(int x) {
    int c = 16;
    while (c < x && c < (1 << 30)) c <<= 1;
    return c;
}

}  // namespace tvs

struct tvs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    tvs::Scratch slots[tvs::S_COUNT];
    int n_cu = 0;
    // FGP momentum table: beta[k] for k < beta_len (float and double copies)
    int beta_len = 0;
    // FGP tile / temporal-depth choices (tune_key -> entry), set by the
    // autotuner, by hand or from a tuning file
    std::map<uint64_t, tvs::TuneEntry> fgp_tuned;
    // cached graphs of solver runs
    std::vector<tvs::GraphEntry*> graphs;
};

namespace tvs {

void* scratch(tvs_ctx* ctx, Slot s, size_t bytes);

enum OpKind { OP_IDENTITY = 0, OP_BLUR = 1, OP_JOSEPH = 2 };

// Per-angle Joseph geometry.  For a ray (a, d) the sampled step index s runs
// over image rows (cls 0) or columns (cls 1); the continuous interpolation
// coordinate at step s is u = A d + B s + C.  The projector and the
// backprojector evaluate u with exactly the same arithmetic, so the two are
// exact transposes of each other:
//  - float64 data: u = fma(A, d, fma(B, s, C)) in float64, floor / fraction;
//  - float32 data: u in 32.32 fixed point, U = u 2^32 = Aq d + Bq s + Cq with
//    integer-valued float64 coefficients (Aq = round(A 2^32) ...).  Every
//    intermediate is an integer below 2^52, so all float64 sums and products
//    are exact, either kernel may step U incrementally, and floor(u) and the
//    fraction are read from the bits of U + 1.5 2^52.  Rounding the
//    coefficients moves a sample by less than 2e-7 pixel.
struct JAngle {
    double A, B, C;    // coefficients of u
    double inv_A;      // 1 / A
    double half_span;  // 1 / |A|
    double wgt;        // pixel / max(|cos|, |sin|)
    double Aq, Bq, Cq; // integer-valued 32.32 fixed-point copies of A, B, C
    long long Aqi, Bqi, Cqi;  // the same integers as int64
    float inv_Af, half_spanf;
    int cls;           // 0: steps over rows, interpolates columns; 1: the reverse
    int n_cand;        // candidate rays per pixel in the backprojector
};

struct JosephGeom {
    int n_ang = 0, n_det = 0;
    double pixel = 0, det_spacing = 0;
    JAngle* ang = nullptr;   // device table
    std::vector<JAngle> host;
    // the ray-driven float32 backprojector applies (joseph_rd_angle_ok for
    // every angle)
    bool rd_ok = false;
    // the paired-ray float32 projector applies: adjacent rays 1 to 2 pixels
    // apart along the interpolation axis for every angle (1 <= |A| < 2 in
    // the 32.32 coefficient), so a ray's right neighbour pair is 1 or 2
    // pixels past the left ray's
    bool pair_ok = false;
    // angle groups of the ray-driven backprojector, chosen on first use
    mutable int rd_groups = 0;
    // angle-subset operators of the stochastic-angle method (sub_n of them,
    // owned), each subset's first row in the permuted sinogram, and the
    // permutation (permuted row -> angle) on the device
    int sub_n = 0;
    std::vector<tvs_op*> subsets;
    std::vector<int> sub_off;
    int* sub_perm = nullptr;
};

struct BlurGeom {
    int kh = 0, kw = 0;
    float* k_f = nullptr;   // device kernel (row-major kh x kw)
    double* k_d = nullptr;
};

}  // namespace tvs

struct tvs_op {
    tvs_ctx* ctx = nullptr;
    int kind = 0;
    int H = 0, W = 0;
    tvs::JosephGeom joseph;
    tvs::BlurGeom blur;
    size_t out_size() const {
        return kind == tvs::OP_JOSEPH ? (size_t)joseph.n_ang * joseph.n_det
                                      : (size_t)H * W;
    }
};

namespace tvs {

// One slice of the batched form: size, element offset in the pools (the
// slice's dual planes start at 2 * off in the dual pool) and its per-slice
// scalars lambda = alpha gamma / p, coef = gamma - gamma / p, rate = p / gamma.
template <typename T>
struct BSlice {
    int H, W;
    long long off;
    T lam, coef, rate;
};

// ---------------------------------------------------------------- epilogues
// What a per-pixel data-fidelity kernel does with s = (grad f) or (A^T y) at
// a pixel, shared by all operators.
template <typename T>
struct PrimalStep {
    // w = x - step * s;  xhat = w + step * h
    // theta = 1: v = w + coef * h  (stored), xhat stored
    // theta = 0: x <- xhat (in place); pdhg: xbar = 2 xhat - x_old (+ transpose)
    T* x;
    const T* h;
    T* xhat;
    T* v;
    T* xbar;       // element (0, 0) of xbar, row stride xbar_ld
    T* xbarT;      // element (0, 0) of the transposed xbar, row stride xbarT_ld
    int xbar_ld, xbarT_ld;
    T step, coef;
    int theta;
    int pdhg;
    int xcopy;     // pdhg and xcopy: the padded copies take xhat itself (no extrapolation)
};

// Backprojector epilogue of the stochastic-angle method: s = A_j^T dy;
// z += s; zbar = z + nsub s.
template <typename T>
struct ZAcc {
    T* z;
    T* zbar;
    T nsub;
};

// ------------------------------------------------------------------ launchers
// All launchers enqueue on ctx->stream and throw tvs::Error on failure.

// D, div (standalone, unit tests and reductions)
template <typename T> void launch_grad(tvs_ctx* ctx, int H, int W, const T* u, T* q);
template <typename T> void launch_div(tvs_ctx* ctx, int H, int W, const T* q, T* u);

// FGP on the dual: runs `iters` iterations from the warm dual in q_inout and
// returns the buffer holding the final dual (q_inout or a scratch buffer);
// launch_finalize then forms z and copies the dual back into q_inout.
// FGP configuration for one H x W image: the exact-size entry, else the size
// class entry, else the default.  fgp_config_batched: per slice count.
FgpConfig fgp_config(tvs_ctx* ctx, int H, int W, int dtype_bytes);
FgpConfig fgp_config_batched(tvs_ctx* ctx, int n_slices, int dtype_bytes);
int find_variant_index(const FgpConfig& c, int dtype_bytes);  // -1 if not compiled
int fgp_variant_count();
FgpConfig fgp_variant(int index);
template <typename T>
T* run_fgp(tvs_ctx* ctx, int H, int W, const T* v, double lambda, int iters, int nonneg,
           T* q_inout, const FgpConfig& cfg, const int* run_flag = nullptr);
// The same on caller-given work buffers (three fields of 2 H W elements) and
// momentum table (iters + 1 entries); allocates nothing.
template <typename T>
T* run_fgp_bufs(tvs_ctx* ctx, int H, int W, const T* v, double lambda, int iters, int nonneg,
                T* q_inout, T* const* work, const T* beta, const FgpConfig& cfg,
                const int* run_flag = nullptr);
// The allocation-free prox's static device array: its device address on
// `device` (looked up once per device, with the device current).
void noalloc_setup(int device);
void* noalloc_ptr(int device);

// z = P_X(v + div q) and the ProxSkip / PDHGSkip bookkeeping after a prox.
template <typename T>
struct Finalize {
    const T* v;
    const T* q;      // final dual (may differ from q_out)
    T* q_out;        // caller's dual buffer; written if != q
    T* z;            // standalone prox output (or nullptr)
    T* x;            // solver: x_{k+1} = z (old x read first for pdhg)
    T* h;            // h += rate (z - xhat)
    const T* xhat;
    T* xbar;         // pdhg: 2 z - x_old (row stride xbar_ld)
    T* xbarT;        // pdhg: transposed copy (row stride xbarT_ld)
    int xbar_ld, xbarT_ld;
    T rate;
    T c1, c2;        // mode 4: xbar = c1 z - c2 x_old
    int nonneg;
    int mode;        // 0: prox only, 1: proxskip, 2: pdhgskip, 3: stochastic angles (xbar = z),
                     // 4: pdhgskip-1 (no control variate)
};
template <typename T> void launch_finalize(tvs_ctx* ctx, int H, int W, const Finalize<T>& f);

// ProxSkip data step for A = I:  s = x - b, then PrimalStep.
template <typename T>
void launch_identity_step(tvs_ctx* ctx, int H, int W, const T* b, const PrimalStep<T>& ps);
// PDHGSkip data step for A = I:  s = y, then PrimalStep.
template <typename T>
void launch_identity_adj_step(tvs_ctx* ctx, int H, int W, const T* y, const PrimalStep<T>& ps);
// y = (y + tau (xbar - b)) / (1 + tau), pointwise (A = I).
template <typename T>
void launch_dual_prox_pointwise(tvs_ctx* ctx, size_t n, const T* xb, const T* b, T* y, T tau);
// Pointwise: out = x - b (residual for A = I) etc.
template <typename T>
void launch_axpby(tvs_ctx* ctx, size_t n, T a, const T* x, T bcoef, const T* y, T* out);
template <typename T> void launch_copy(tvs_ctx* ctx, size_t n, const T* x, T* y);
template <typename T> void launch_fill(tvs_ctx* ctx, size_t n, T val, T* y);
// FISTA's extrapolation: out = x + beta (x - xprev).
template <typename T>
void launch_fista_extrap(tvs_ctx* ctx, size_t n, const T* x, const T* xprev, T beta, T* out);
template <typename T>
void launch_permute_rows(tvs_ctx* ctx, int rows, int cols, const int* perm, const T* src, T* dst,
                         bool scatter);
template <typename T> void launch_transpose(tvs_ctx* ctx, int H, int W, const T* x, T* xT);

// Blur: out = A x (- b if b), or A^T y followed by a PrimalStep.
template <typename T>
void launch_blur(tvs_ctx* ctx, const tvs_op* op, bool adjoint, const T* x, const T* b, T* out);
template <typename T>
void launch_blur_dual_prox(tvs_ctx* ctx, const tvs_op* op, const T* xbar, const T* b, T* y, T tau);
template <typename T>
void launch_blur_adjoint_step(tvs_ctx* ctx, const tvs_op* op, const T* r, const PrimalStep<T>& ps);

// Joseph: forward with epilogue (store, residual, dual prox), adjoint with
// epilogue (store, primal step).  The projector reads the image through two
// zero-padded copies, row-major (row stride W + 2 JPAD) and transposed (row
// stride H + 2 JPAD), each with JPAD zero columns on both sides of every row,
// so that samples falling just outside the image read zeros instead of
// being masked; x and xT point at element (0, 0) of each copy.
constexpr int JPAD = 4;
enum FwdEpi { FWD_STORE = 0, FWD_RESIDUAL = 1, FWD_DUAL_PROX = 2, FWD_DUAL_PROX_DELTA = 3 };
// FWD_DUAL_PROX_DELTA: the dual prox of FWD_DUAL_PROX, and dy = y_new - y_old.
template <typename T>
void launch_joseph_fwd(tvs_ctx* ctx, const tvs_op* op, const T* x, const T* xT, const T* b,
                       T* y, int epi, T tau, T* dy = nullptr);
// Writes both padded copies of the H x W image x (pads included).
template <typename T>
void launch_pad_copy(tvs_ctx* ctx, int H, int W, const T* x, T* xp, T* xTp);
int joseph_rd_groups(const tvs_ctx* ctx, const tvs_op* op);
int joseph_rd_max_angles();
void joseph_upload(tvs_op* op);
void joseph_make_subsets(tvs_op* op, int n);
void joseph_free_subsets(tvs_op* op);
bool joseph_rd_angle_ok(const JAngle& e);
template <typename T>
void launch_joseph_adj(tvs_ctx* ctx, const tvs_op* op, const T* y, T* x_out,
                       const PrimalStep<T>* ps, const ZAcc<T>* za = nullptr);

// Reductions (deterministic two-stage, float64 accumulation).  Each returns
// a device pointer to one double holding the result.
template <typename T>
double* reduce_sq_diff(tvs_ctx* ctx, size_t n, const T* a, const T* b, double* out_dev);
template <typename T>
double* reduce_tv(tvs_ctx* ctx, int H, int W, const T* u, double* out_dev);
template <typename T>
void reduce_gap(tvs_ctx* ctx, int H, int W, const T* v, const T* z, const T* q, double lam,
                double* gap_dev, double* primal_dev);
// grows the reduction scratch so that the reductions over n elements can
// later be enqueued during graph capture
void reserve_reduce_scratch(tvs_ctx* ctx, size_t n);
template <typename T>
double* reduce_dot(tvs_ctx* ctx, size_t n, const T* a, const T* b, double* out_dev);
// out[0] = a*x[0] + b*y[0] on the device (scalars combined in float64)
void launch_combine(tvs_ctx* ctx, const double* x, double a, const double* y, double b, double* out);

// host helpers
uint64_t splitmix_mix(uint64_t z);
int coin(uint64_t seed, uint64_t stream, int64_t k, double p);
// the skipping inner solver draws its coins on stream stream_id xor 2^62
constexpr uint64_t INNER_STREAM = 1ULL << 62;
int subset_draw(uint64_t seed, uint64_t stream, int64_t k, int n);
const double* beta_table_host(int n);

template <typename T> const T* beta_table_dev(tvs_ctx* ctx, int n);

// batched form (kernels_fgp.hip, kernels_ops.hip)
struct BatchLists {
    const int* act;         // active slice ids of this iteration
    const int* pref_fgp;    // cumulative FGP tile counts (n_act + 1)
    const int* pref_fin;    // cumulative 32 x 32 tile counts (n_act + 1)
    int n_act, tiles_fgp, tiles_fin;
};
template <typename T>
T* run_fgp_batched(tvs_ctx* ctx, const BSlice<T>* sl, const BatchLists& L, const T* v_pool,
                   T* q_pool, size_t total_px, int iters, int nonneg, const FgpConfig& cfg);
template <typename T>
void launch_finalize_batched(tvs_ctx* ctx, const BSlice<T>* sl, const BatchLists& L, const T* v,
                             const T* q, T* q_out, T* x, T* h, const T* xhat, int nonneg);
template <typename T>
void launch_identity_step_batched(tvs_ctx* ctx, const BSlice<T>* sl, const int* pref_all, int n,
                                  int tiles, const uint8_t* theta, const T* b, T* x, const T* h,
                                  T* xhat, T* v, T step);

// graphs (graph.hip)
// Runs `enqueue` captured into a HIP graph (cached under the call's key) on
// ctx->stream.  All scratch memory must already be allocated.
void graph_run(tvs_ctx* ctx, const tvs_op* op, bool pdhg, int dtype, const void* b,
               const tvs_state* st, const tvs_params* P, const std::function<void()>& enqueue);
std::vector<uint64_t> graph_key(const tvs_op* op, bool pdhg, int dtype, const void* b,
                                const tvs_state* st, const tvs_params* P);
void graph_run_key(tvs_ctx* ctx, const std::vector<uint64_t>& key,
                   const std::function<void()>& enqueue);
void graph_cache_clear(tvs_ctx* ctx);

// TV prox and its duality gap on one image (api.hip); gap_host synchronises
template <typename T>
void gap_host(tvs_ctx* ctx, int H, int W, const T* v, double lam, int nonneg, const T* q,
              double* gap, double* primal);
template <typename T>
void tv_prox_impl(tvs_ctx* ctx, int H, int W, const T* v, double lambda, int iters, int nonneg,
                  T* q, T* z, double* rel_gap);

// TV prox by ProxSkip on its dual (light_prox.hip): iters steps (coins
// theta[0 .. iters)) with step 1/8 and projection probability p_in from the
// warm (q, h) (the constrained dual when nonneg).  h ends in h; returns the
// buffer that holds the final dual (q or a scratch buffer).  Enqueue only.
template <typename T>
T* run_tv_prox_skip(tvs_ctx* ctx, int H, int W, const T* v, double lam, int nonneg, int iters,
                    double p_in, const uint8_t* theta, T* q, T* h);

// Optional parts of a solver run: the learned prox or the skipping inner
// solver in place of FGP, and the recording of the prox inputs.
struct SolveExt {
    tvs_cnn* cnn = nullptr;
    double gap_tol = 0.0;
    void* v_record = nullptr;   // device, max_record x H x W, the solver's dtype
    int64_t max_record = 0;
    int* gate = nullptr;        // device, one int per prox call (learned prox)
    double inner_p = 0.0;       // > 0: the prox by run_tv_prox_skip
    void* inner_h = nullptr;    // its control variate, device [2][H][W]
    const uint8_t* inner_theta = nullptr;  // host, inner_iters coins per prox call
};

// learned prox (kernels_cnn.hip)
namespace cnn {
constexpr int CONV_NT = 256;   // threads per block of the convolution kernels
constexpr int CONV_TILE = 16;  // forward / input-gradient output tile edge
constexpr int WG_TH = 8;       // rows of a weight-gradient tile (16 columns)
enum { IN_VLAM = 0, IN_BF16 = 1 };
enum { OUT_RELU_BF16 = 0, OUT_F32_PLANAR = 1, OUT_MASK_BF16 = 2 };

struct ConvArgs {
    int n = 0, H = 0, W = 0;
    const float* v = nullptr;       // IN_VLAM: [n][H][W]
    const float* lam = nullptr;     // [n] (device)
    const uint16_t* in = nullptr;   // IN_BF16: [n][H][W][cin] bf16
    const uint16_t* in_lo = nullptr;// split: low parts of in
    const uint16_t* wt = nullptr;   // [coutp][kp] bf16
    const uint16_t* wt_lo = nullptr;// split: low parts of wt
    const float* bias = nullptr;    // forward: [cout]
    uint16_t* out_bf = nullptr;     // [n][H][W][32] bf16
    uint16_t* out_lo = nullptr;     // split OUT_RELU_BF16: low parts
    const uint16_t* mask = nullptr; // OUT_MASK_BF16: keep where mask > 0
    float* out_f = nullptr;         // OUT_F32_PLANAR: [n][2][H][W]
    int proj = 0;                   // OUT_F32_PLANAR: project onto the lam ball
    int tiles_x = 0, tiles_y = 0, n_tiles = 0;
    const int* run = nullptr;       // device flag (nullable): 0 = return at once
};
struct WgradArgs {
    int n = 0, H = 0, W = 0;
    const float* v = nullptr;       // IN_VLAM input
    const float* lam = nullptr;
    const uint16_t* x = nullptr;    // IN_BF16 input [n][H][W][cin]
    const uint16_t* g = nullptr;    // output gradient [n][H][W][cout]
    float* part = nullptr;          // [blocks][(9 cin + 1) cout]
    int tiles_x = 0, tiles_y = 0, n_tiles = 0;
};
struct HeadArgs {
    int n = 0, H = 0, W = 0, nonneg = 0;
    const float* qt = nullptr;      // [n][2][H][W]
    const float* v = nullptr;       // [n][H][W]
    const float* lam = nullptr;     // [n]
    float* z = nullptr;             // nullable
    const float* z_target = nullptr;// training only
    const float* q_target = nullptr;// training, optional dual target [n][2][H][W]
    float mu = 0.f;                 // weight of the dual term
    float* gu = nullptr;            // training: dL/du [n][H][W]
    float inv_npx = 0.f;
    double* loss_part = nullptr;    // [blocks]
    double* loss_out = nullptr;     // sum of squared errors
    uint16_t* gq_bf = nullptr;      // backward: [n][H][W][2] bf16
};
void launch_conv(tvs_ctx* ctx, int cin, int coutp, int in_mode, int out_mode, bool split,
                 ConvArgs a);
int wgrad_blocks(const tvs_ctx* ctx, int n, int H, int W);
void launch_wgrad(tvs_ctx* ctx, int layer, WgradArgs a, float* grad_out);
int head_blocks(const tvs_ctx* ctx, size_t tot);
void launch_head_fwd(tvs_ctx* ctx, HeadArgs a, int nblk);
void launch_head_bwd(tvs_ctx* ctx, HeadArgs a, int nblk);
void launch_adam(tvs_ctx* ctx, int n, float* p, const float* grad, float* m, float* v, float lr,
                 float b1, float b2, float c1, float c2, float eps);
void launch_pack(tvs_ctx* ctx, const float* w, int cin, int cout, uint16_t* wf, uint16_t* wf_lo,
                 uint16_t* wb);
void launch_pregate(tvs_ctx* ctx, const double* red, double tol, int* run);
void launch_gate(tvs_ctx* ctx, const double* red, double tol, const int* run, int* flag, int* sel);
void launch_copy_if(tvs_ctx* ctx, size_t n, const int* flag, int when, const float* src,
                    float* dst);
// Learned prox inside a solver run (capturable): allocations and lam set up
// by prepare_solver_prox before capture; enqueue_solver_prox computes
// P_lam(net(v)) and gates on its relative duality gap (device side): at most
// tol, it becomes the dual; above, `iters` FGP iterations run, warm-started
// from whichever of it and the previous call's dual in q has the smaller
// relative gap.  Returns the buffer holding the final dual; *record (device)
// gets 1 if FGP ran.
void prepare_solver_prox(tvs_cnn* c, int H, int W, double lam);
bool fast_forward(const tvs_cnn* c);
float* enqueue_solver_prox(tvs_cnn* c, int H, int W, const float* v, double lam, int nonneg,
                           double tol, int iters, float* q, const FgpConfig& cfg, int* record);
}  // namespace cnn

__host__ __device__ inline int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }

// The GPU deals workgroups to its 8 XCDs (each with its own L2) round-robin
// by linear workgroup id.  For a 1-D launch of n_tiles workgroups this maps
// workgroup L to a tile so that each XCD works through one contiguous range
// of tiles (row-major), and tiles that share halo cache lines meet in the
// same L2.  A bijection on [0, n_tiles).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int L, int n_tiles) {
    const int x = L % kXcds, k = L / kXcds;
    const int base = n_tiles / kXcds, rem = n_tiles % kXcds;
    return x * base + (x < rem ? x : rem) + k;
}

}  // namespace tvs
