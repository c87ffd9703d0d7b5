/*
 * tvskip.h -- C ABI of the MI355X (gfx950) library for ProxSkip and
 * PDHGSkip-2 on TV-regularised imaging inverse problems.
 *
 * The problem (eq. (5) of Papoutsellis, Kereta and Papafitsoros, "Why do we
 * regularise in every iteration for imaging inverse problems?"):
 *
 *     argmin_u  1/2 |A u - b|_2^2 + alpha TV(u)        (optionally u >= 0,
 *                                                      the CT problem of Sec. 3.3)
 *
 * solved by ProxSkip (Alg. "ProxSkip") or PDHGSkip-2 (Alg. "PDHGSkip-2"),
 * whose randomly skipped TV prox is evaluated by an inner FGP loop (the
 * paper's accelerated projected gradient on the dual, "AProjGD", Sec. 2-3).
 *
 * Conventions shared by every call:
 *  - Images are row-major H x W; pixel (i, j) is row i, column j.  A TV dual
 *    field is two planes [2][H][W]: plane 0 the row (y) component, plane 1
 *    the column (x) component, matching D u = (D_y u, D_x u).  A CT sinogram
 *    is row-major [n_ang][n_det].
 *  - Array arguments named as device buffers are device pointers on the
 *    context's device, contiguous, of the element type `dtype` (float or
 *    double).  The caller owns them; the library never frees caller memory.
 *    Arguments typed `const double*` with a `_host` suffix and every scalar
 *    output are host memory.
 *  - Work is ordered on the context's HIP stream.  Calls return once the work
 *    is enqueued, except where they fill host outputs (reports, traces, gaps,
 *    norms, objectives): those synchronise the stream before returning.
 *  - Every call returns a tvs_status; on failure tvs_last_error() (per host
 *    thread) holds a message.  No call aborts or throws across the ABI.
 *    On failure no output is guaranteed to be written, and device buffers
 *    passed as in/out may hold partial results.
 *  - One context per host thread at a time.
 */
#ifndef TVSKIP_H
#define TVSKIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tvs_status {
    TVS_OK = 0,
    TVS_ERR_INVALID_ARG = 1, /* null pointer, bad scalar (p outside (0, 1], ...) */
    TVS_ERR_SHAPE = 2,       /* sizes out of range or inconsistent */
    TVS_ERR_DEVICE = 3,      /* a HIP runtime call failed */
    TVS_ERR_OOM = 4,         /* device allocation failed */
    TVS_ERR_NONFINITE = 5,   /* a checked result is NaN or infinite */
    TVS_ERR_UNSUPPORTED = 6  /* combination not implemented */
} tvs_status;

typedef enum tvs_dtype { TVS_F32 = 0, TVS_F64 = 1 } tvs_dtype;

typedef struct tvs_ctx tvs_ctx;
typedef struct tvs_op tvs_op;

/* ------------------------------------------------------------------ context
 * Binds a device and a HIP stream (hipStream_t passed as void*; NULL is the
 * null stream).  The context owns its scratch memory (grown on demand, freed
 * by tvs_ctx_destroy). */
tvs_status tvs_ctx_create(int device, void* hip_stream, tvs_ctx** out);
void tvs_ctx_destroy(tvs_ctx* ctx);
tvs_status tvs_ctx_set_stream(tvs_ctx* ctx, void* hip_stream);
/* Message of the last failing call on this host thread ("" if none). */
const char* tvs_last_error(void);
/* Blocks until all work enqueued on the context's stream has finished. */
tvs_status tvs_sync(tvs_ctx* ctx);

/* ---------------------------------------------------------------- operators
 * A: X -> Y.  X is H x W.  Y is H x W (identity, blur) or n_ang x n_det (CT).
 * An operator copies its tables to the device and keeps a pointer to ctx; it
 * must be destroyed before the context. */

/* A = I (the denoising problems of Sec. 2 and the batched denoising form). */
tvs_status tvs_op_identity(tvs_ctx* ctx, int H, int W, tvs_op** out);

/* A = periodic convolution (deblurring, Sec. 3.1):
 *   (A x)_{i,j} = sum_{m,n} k_{m,n} x_{(i-m) mod H, (j-n) mod W},
 * k_{m,n} = kernel_host[(m + kh/2) * kw + (n + kw/2)]; kh, kw odd, <= 17 and
 * <= H, W.  The adjoint is the correlation with the same kernel. */
tvs_status tvs_op_blur_periodic(tvs_ctx* ctx, int H, int W, const double* kernel_host,
                                int kh, int kw, tvs_op** out);

/* A = parallel-beam discrete Radon transform (CT, Sec. 3.3), discretised as
 * Joseph's ray-driven projector with linear interpolation:
 *   pixel centres ((j - (W-1)/2) pixel, ((H-1)/2 - i) pixel), bins
 *   s_b = (b - (n_det-1)/2) det_spacing, ray {x cos t + y sin t = s_b}.
 *   A ray with |cos t| >= |sin t| is sampled once per image row, otherwise
 *   once per column, interpolating linearly between the two nearest pixel
 *   centres of that row (column), weighted by pixel / max(|cos t|, |sin t|).
 * The adjoint is its exact transpose (same interpolation weights), without
 * atomics: for float32 with det_spacing >= pixel / max(|cos t|, |sin t|)
 * over all angles (so neighbouring rays are at least one pixel apart), a
 * ray-driven scatter into LDS tiles plus a fixed-order sum of per-angle-group
 * partial images; otherwise (and for float64) a gather over pixels.  In
 * float32 the ray positions are 32.32 fixed-point integers shared by both
 * directions, so the transpose is exact there too.  angles_host: n_ang
 * radians.  Requires pixel / 4 <= det_spacing <= 4 pixel, 1 <= n_ang <= 65535
 * and n_det, H, W <= 32768 (TVS_ERR_SHAPE / TVS_ERR_INVALID_ARG otherwise). */
tvs_status tvs_op_ct_joseph(tvs_ctx* ctx, int H, int W, int n_ang,
                            const double* angles_host, int n_det, double pixel,
                            double det_spacing, tvs_op** out);

/* Angle groups of the float32 ray-driven backprojector of a Joseph operator
 * (a tuning control; the result does not depend on it beyond the order of
 * the float32 sums): one workgroup per (52 x 52 tile, group), group g
 * holding angles g, g + groups, ...; the groups' partial images are summed in
 * a fixed order.  groups = 0 restores the automatic choice (the count that
 * balances the most loaded compute unit).  Otherwise 1 <= ceil(n_ang / 36)
 * <= groups <= n_ang (TVS_ERR_INVALID_ARG; also for an operator that is not
 * Joseph).  Waits for the device and drops the context's captured graphs. */
tvs_status tvs_op_joseph_set_groups(tvs_op* op, int groups);
/* The group count the backprojector uses (-1 if op is not Joseph). */
int tvs_op_joseph_groups(const tvs_op* op);

void tvs_op_destroy(tvs_op* op);
/* Output size (number of elements of Y). */
size_t tvs_op_out_size(const tvs_op* op);
/* y = A x  (x: device, H*W; y: device, out_size). */
tvs_status tvs_op_apply(tvs_op* op, tvs_dtype dtype, const void* x, void* y);
/* x = A^T y. */
tvs_status tvs_op_adjoint(tvs_op* op, tvs_dtype dtype, const void* y, void* x);
/* |A|_2 by `iters` power iterations on A^T A in float64 from a start vector
 * seeded by `seed` (step sizes with sigma tau |K|^2 <= 1, Sec. 3.3). */
tvs_status tvs_op_norm(tvs_op* op, int iters, uint64_t seed, double* norm_out);

/* ----------------------------------------------------- TV building blocks
 * D u = (D_y u, D_x u): forward differences, zero in the last row / column
 * (Neumann, the TV definition before eq. (5)).  div = -D^T (Sec. 2.1). */
tvs_status tvs_grad(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, const void* u, void* q);
tvs_status tvs_div(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, const void* q, void* u);

/* TV prox  z = argmin 1/2 |z - v|^2 + lambda TV(z) (+ z >= 0 if nonneg),
 * by `inner_iters` FGP iterations on the dual (Dual-ROF, eq. (6)):
 *   z = P_X(v + div r);  q_k = P_lambda(r + D z / 8);
 *   t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2;
 *   r = q_k + ((t_k - 1) / t_{k+1}) (q_k - q_{k-1}),
 * P_lambda the pixelwise projection onto the lambda ball (eq. (7)), warm
 * started from q_inout (2*H*W, device, in/out: warm dual in, final dual out);
 * t restarts at 1 on every call.  z_out: device, H*W.  rel_gap_out
 * (nullable, host): gap(q) / P(z) of the returned pair, which synchronises. */
tvs_status tvs_tv_prox(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, const void* v,
                       double lambda, int inner_iters, int nonneg, void* q_inout,
                       void* z_out, double* rel_gap_out);

/* The TV prox of tvs_tv_prox (same kernels, same results bit for bit) for
 * callers that cannot allocate device memory: code under HIP stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  It allocates
 * nothing: its work buffers (the momentum table and three dual fields) live
 * in one static device array of TVS_NOALLOC_SCRATCH_BYTES per device, held
 * until the process ends, whose device address the context creation looks
 * up.  Requires 256-byte-aligned (inner_iters + 1) + 3 * (2 H W) elements of
 * dtype to fit (float32: about 1.39 million pixels, e.g. 1024 x 1024;
 * float64 about 0.69 million, e.g. 800 x 800); larger sizes return
 * TVS_ERR_INVALID_ARG before anything is enqueued.  No rel_gap output (that
 * would need a reduction buffer and a host wait).  Every call on a device
 * shares that device's array: calls that overlap on one device (other
 * streams, other threads) race; calls in one stream are ordered.  Arguments
 * as tvs_tv_prox; enqueues on the context's stream and does not wait. */
#define TVS_NOALLOC_SCRATCH_BYTES (32u << 20)
tvs_status tvs_tv_prox_noalloc(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, const void* v,
                               double lambda, int inner_iters, int nonneg, void* q_inout,
                               void* z_out);

/* Duality gap of the TV prox at dual point q: with z = P_X(v + div q),
 *   gap = sum_i lambda |(D z)_i| - <(D z)_i, q_i>,  P(z) = 1/2|z - v|^2 + lambda TV(z).
 * Host outputs (nullable); synchronises. */
tvs_status tvs_tv_gap(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, const void* v,
                      double lambda, int nonneg, const void* q, double* gap_out,
                      double* primal_out);

/* Phi(x) = 1/2 |A x - b|^2 + alpha TV(x) (eq. (5), without the u >= 0
 * indicator).  x: device H*W; b: device out_size.  Synchronises. */
tvs_status tvs_objective(tvs_op* op, tvs_dtype dtype, const void* b, const void* x,
                         double alpha, double* out);

/* ------------------------------------------------------------- FGP tuning
 * The FGP kernel is compiled for several output tiles (tile_w x tile_h) and
 * temporal depths (steps: FGP iterations fused per launch, with a halo of
 * `steps` pixels), each with 256 threads; the variants with tile_w >= 240
 * are row-walking strips for large images (a workgroup walks 256 columns,
 * storing tile_w of them, down tile_h rows).  The context keeps a tuning table:
 * entries per exact size (H, W, dtype), per size class (H and W each
 * rounded up to a power of two, at least 16; written by the autotuner next
 * to the exact entry) and per batched slice count.  An H x W prox uses the
 * exact entry, else its size class entry, else the default (32 x 32, 4
 * steps). */
int tvs_fgp_variant_count(void);
/* Shape of variant `index` (host outputs). */
tvs_status tvs_fgp_variant(int index, int* tile_w, int* tile_h, int* steps);
/* Use variant `index` for (H, W, dtype) from now on; index -1 restores the
 * default. */
tvs_status tvs_fgp_set_variant(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, int index);
/* Times every variant on a seeded random H x W image (inner_iters FGP
 * iterations, `reps` repetitions, HIP events; three rounds over all variants,
 * each variant's best round counted), keeps the fastest and returns
 * it in *best_index (nullable); ms_per_iter_out (nullable, host, variant
 * count doubles) gets each variant's milliseconds per FGP iteration (-1 if
 * not available for the dtype).  Synchronises; allocates temporary device
 * memory. */
tvs_status tvs_fgp_autotune(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, int inner_iters,
                            int reps, int* best_index, double* ms_per_iter_out);
/* The variant an H x W prox would use now (*index, host) and its measured
 * milliseconds per FGP iteration (*ms_per_iter, nullable; -1 when set by
 * hand or the default). */
tvs_status tvs_fgp_query(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, int* index,
                         double* ms_per_iter);
/* Remove every tuning entry of the context. */
tvs_status tvs_tune_clear(tvs_ctx* ctx);
/* Save the tuning table as JSON: {"format": "tvskip-fgp-tune/1", "arch":
 * <GPU architecture, e.g. "gfx950">, "entries": [{"kind": "image" | "class" |
 * "batch", "dtype": "f32" | "f64", "H", "W" (image, class) or "n_slices"
 * (batch), "tile_w", "tile_h", "steps", "ms_per_iter"}, ...]}.  Written to
 * path + ".tmp" and renamed. */
tvs_status tvs_tune_save(tvs_ctx* ctx, const char* path);
/* Load a tuning file: entries replace those with the same key.  A file made
 * on another architecture is TVS_ERR_UNSUPPORTED, a malformed one
 * TVS_ERR_INVALID_ARG (the table is unchanged in both cases), an entry naming
 * a variant this library does not compile TVS_ERR_UNSUPPORTED. */
tvs_status tvs_tune_load(tvs_ctx* ctx, const char* path);

/* --------------------------------------------------------------------- coin
 * theta_k ~ Bernoulli(p), i.i.d. in k (Alg. "ProxSkip", Alg. "PDHGSkip-2"),
 * as a pure function of (seed, stream_id, k): SplitMix64 (Steele, Lea and
 * Flood 2014, output mix of Stafford's variant 13): key = mix(seed ^
 * mix(stream_id + G)), r = mix(key + (k + 1) G), theta = [(r >> 11) <
 * floor(p 2^53)], G = 0x9E3779B97F4A7C15.  Returns 0 or 1, or -1 if p is
 * outside (0, 1] or k < 0.  Host only. */
int tvs_coin(uint64_t seed, uint64_t stream_id, int64_t k, double p);

/* ------------------------------------------------------------------ solvers */
typedef struct tvs_params {
    double alpha;        /* TV weight, >= 0 */
    double step;         /* gamma (ProxSkip) or sigma (PDHGSkip), > 0 */
    double dual_step;    /* tau (PDHGSkip), > 0; ignored by ProxSkip */
    double p;            /* prox probability, (0, 1]; p = 1 gives PGD / PDHG */
    int64_t outer_iters; /* K >= 0 */
    int32_t inner_iters; /* FGP iterations per prox call, >= 1 */
    int32_t nonneg;      /* 1: add u >= 0 to g */
    uint64_t seed;       /* coin seed */
    uint64_t stream_id;  /* coin stream */
    int64_t k0;          /* index of the first coin draw (resume) */
    int32_t flags;       /* TVS_FLAG_* */
    int32_t reserved;
} tvs_params;

/* Capture the whole launch sequence into a HIP graph and launch it as one
 * graph; an identical later call (same op, buffers, params) relaunches the
 * cached graph. */
#define TVS_FLAG_GRAPH 1

/* Iterate state, caller-owned device buffers, in/out.  x, h: H*W; q: 2*H*W
 * (the warm FGP dual); y: out_size (PDHGSkip only, NULL for ProxSkip).
 * Initial values in, values after the last iteration out. */
typedef struct tvs_state {
    void* x;
    void* h;
    void* q;
    void* y;
} tvs_state;

typedef struct tvs_report {
    int64_t n_prox;     /* number of prox evaluations (theta_k = 1) */
    int64_t iters;      /* outer iterations done */
} tvs_report;

/* ProxSkip (Alg. "ProxSkip") with f = 1/2|A . - b|^2, g = alpha TV (+ u >= 0):
 *   xhat = x_k - gamma (grad f(x_k) - h_k)
 *   theta_k = 1: x_{k+1} = prox_{(gamma/p) g}(xhat - (gamma/p) h_k), by FGP
 *   theta_k = 0: x_{k+1} = xhat
 *   h_{k+1} = h_k + (p/gamma)(x_{k+1} - xhat)
 * b: device out_size.  obj_trace (nullable, host, outer_iters doubles):
 * Phi(x_{k+1}) per iteration (adds work; synchronises).  theta_trace
 * (nullable, host, outer_iters bytes).  report (nullable, host). */
tvs_status tvs_proxskip(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                        const tvs_params* params, double* obj_trace,
                        uint8_t* theta_trace, tvs_report* report);

/* PDHGSkip-2 (Alg. "PDHGSkip-2") with K = A, f = 1/2|. - b|^2, g = alpha TV
 * (+ u >= 0), reading the dual update at K xbar_{k+1} and the control-variate
 * update at xhat_k:
 *   xhat = x_k - sigma (A^T y_k - h_k)
 *   theta_k = 1: x_{k+1} = prox_{(sigma/p) g}(xhat - (sigma/p) h_k), by FGP
 *   theta_k = 0: x_{k+1} = xhat
 *   xbar = 2 x_{k+1} - x_k;  y_{k+1} = (y_k + tau (A xbar - b)) / (1 + tau)
 *   h_{k+1} = h_k + (p/sigma)(x_{k+1} - xhat)
 * Same arguments as tvs_proxskip; state->y is required. */
tvs_status tvs_pdhgskip(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                        const tvs_params* params, double* obj_trace,
                        uint8_t* theta_trace, tvs_report* report);

/* The paper's comparison methods on the same kernels.
 * FISTA (Alg. "FISTA", its momentum read as Beck and Teboulle's):
 *   ybar = x_k + ((t_k - 1) / t_{k+1}) (x_k - x_{k-1}),
 *   x_{k+1} = prox_{gamma g}(ybar - gamma A^T (A ybar - b)) by FGP (warm dual),
 * t_1 = 1 and x_{k-1} = x_k at the start of every call (momentum restarted).
 * params: alpha, step = gamma, outer/inner iterations, nonneg, flags (p,
 * seed, stream_id, k0, dual_step ignored; p must still be in (0, 1]).
 * state: x, q (h, y unused).  ISTA is tvs_proxskip at p = 1. */
tvs_status tvs_fista(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                     const tvs_params* params, double* obj_trace, tvs_report* report);

/* PDHGSkip-1 (Alg. "PDHGSkip-1", the bracket read as K(x_{k+1} + xhat_k),
 * omega + 1 = 1/p):
 *   theta_k = 1: x+ = prox_{sigma g}(x_k - sigma A^T y_k) by FGP,
 *                e = (1 + 1/p) x+ - x_k / p (= x_{k+1} + xhat_k), x_{k+1} = x+
 *   theta_k = 0: x_{k+1} = e = x_k (no A^T, no prox)
 *   y_{k+1} = (y_k + tau (A e - b)) / (1 + tau).
 * At p = 1 this is PDHG.  Arguments as tvs_pdhgskip (state h unused). */
tvs_status tvs_pdhgskip1(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                         const tvs_params* params, double* obj_trace, uint8_t* theta_trace,
                         tvs_report* report);

/* Stochastic angle subsets with the skipped prox (the paper's "Discussion
 * and Future work": a random subset of the projection angles per iteration
 * in addition to the random prox).  Reading: SPDHG (Chambolle, Ehrhardt,
 * Richtarik, Schoenlieb, SIAM J. Optim. 2018) over n_subsets interleaved
 * angle subsets (subset j: angles j, j + n, ...; f_j = 1/2|. - b_j|^2,
 * uniform sampling, dual extrapolation 1/p_j = n), with the primal prox of
 * g skipped as in PDHGSkip-2:
 *   xhat = x_k - sigma (zbar_k - h_k)
 *   theta_k = 1: x_{k+1} = prox_{(sigma/p) g}(xhat - (sigma/p) h_k), by FGP
 *   theta_k = 0: x_{k+1} = xhat
 *   h_{k+1} = h_k + (p/sigma)(x_{k+1} - xhat)
 *   j = j_k:  y_j = (y_j + tau (A_j x_{k+1} - b_j)) / (1 + tau)
 *   z += A_j^T dy_j;  zbar = z + n A_j^T dy_j   (dy_j: the change of y_j)
 * with z = zbar = A^T y at the start of every call.  j_k = tvs_subset(seed,
 * stream_id, k, n_subsets).  Step sizes (caller's choice; SPDHG's condition
 * sigma tau |A_j|^2 < 1/n): params->step = sigma, params->dual_step = tau.
 * Joseph operators only (TVS_ERR_UNSUPPORTED otherwise); 1 <= n_subsets <=
 * min(n_ang, 1024) (TVS_ERR_INVALID_ARG).  state->y is required (natural
 * angle order).  subset_trace (nullable, host, outer_iters int32): j_k.
 * Other arguments as tvs_pdhgskip; TVS_FLAG_GRAPH captures the run. */
tvs_status tvs_spdhgskip(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                         const tvs_params* params, int n_subsets, double* obj_trace,
                         uint8_t* theta_trace, int32_t* subset_trace, tvs_report* report);

/* The angle subset drawn at outer iteration k of tvs_spdhgskip: SplitMix64
 * as tvs_coin on the stream stream_id xor 2^63, j_k = floor((r >> 11) n /
 * 2^53) (uniform on 0..n-1).  -1 if n < 1, n > 1024 or k < 0.  Host, pure. */
int tvs_subset(uint64_t seed, uint64_t stream_id, int64_t k, int n);

/* ------------------------------------------------ light-prox problems
 * ProxSkip on the dual of TV denoising, Sec. 2.1-2.2:
 *
 *   min_{|q_i| <= alpha}  F(q) = 1/2 |div q + b|^2 + eps / (2 alpha) |q|^2
 *
 * (eps = 0: Dual-ROF, eq. (6) up to its constant; eps > 0: Dual-Huber-ROF of
 * Sec. 2.2, strongly convex with mu = eps / alpha).  grad F(q) = -D(div q +
 * b) + mu q; the prox is the projection onto the alpha-ball (eq. (7), read as
 * the projection onto radius alpha), so the prox step does not depend on
 * gamma / p.  Step of Alg. "ProxSkip": w = q - step grad F(q), qhat = w + step
 * h; if theta_k: q = P(w + (step - step / p) h), h += (p / step)(q - qhat);
 * else q = qhat.  p = 1 is ProjGD (Sec. 2.1) bitwise.  The primal iterate is
 * u = b + div q (tvs_div).  b: [H][W], q and h: [2][H][W], device, dtype,
 * q and h in/out (start from zeros for a fresh run).  The coin is the stream
 * of tvs_coin(seed, stream_id, k0 + k, p).  theta_trace (nullable, host,
 * outer_iters bytes), n_prox_out (nullable, host).  Eight steps are fused
 * per kernel launch; TVS_FLAG_GRAPH captures the run in one HIP graph. */
typedef struct tvs_dual_rof_params {
    double alpha;        /* radius of the dual ball (the TV weight), >= 0 */
    double eps;          /* Huber smoothing, >= 0 */
    double step;         /* gamma > 0, e.g. 1 / (8 + eps / alpha) */
    double p;            /* projection probability in (0, 1] */
    int64_t outer_iters;
    uint64_t seed, stream_id;
    int64_t k0;          /* first coin index */
    int32_t flags;       /* TVS_FLAG_GRAPH */
    int32_t reserved;
} tvs_dual_rof_params;

tvs_status tvs_dual_rof_proxskip(tvs_ctx* ctx, tvs_dtype dtype, int H, int W, const void* b,
                                 void* q, void* h, const tvs_dual_rof_params* params,
                                 uint8_t* theta_trace, int64_t* n_prox_out);

/* ---------------------------------------------------------- batched form
 * Many independent ProxSkip TV-denoising problems (A = I, Sec. 2; e.g. the
 * slices of a volume or a stack of images) of uneven sizes, solved together: each
 * outer iteration is one data-step launch over every slice, FGP launches over
 * the slices whose coin came up (work lists built on the host from the
 * counter-based coin), and one finalize launch; with TVS_FLAG_GRAPH the whole
 * run is one HIP graph.  Each slice gets the same arithmetic as tvs_proxskip
 * with tvs_op_identity and that slice's alpha, p, seed and stream.
 *
 * Pools (device, dtype elements): slice s occupies [offset, offset + H*W) of
 * b_pool, x_pool and h_pool (row-major H x W) and [2 offset, 2 offset +
 * 2 H W) of q_pool (two planes y, x).  Slices must not overlap.  x, h, q are
 * in/out.  n_prox_out (nullable, host, n_slices int64): prox calls per slice. */
typedef struct tvs_slice {
    int32_t H, W;
    int64_t offset;      /* element offset of the slice in the pools */
    double alpha, p;     /* TV weight and prox probability of the slice */
    uint64_t seed, stream_id;
} tvs_slice;

typedef struct tvs_batch_params {
    double step;         /* gamma (1 = 1/L for A = I) */
    int64_t outer_iters;
    int32_t inner_iters;
    int32_t nonneg;
    int64_t k0;          /* first coin index */
    int32_t flags;       /* TVS_FLAG_GRAPH */
    int32_t fgp_variant; /* FGP tile variant index, -1: the context's choice */
} tvs_batch_params;

tvs_status tvs_proxskip_batched(tvs_ctx* ctx, tvs_dtype dtype, int n_slices,
                                const tvs_slice* slices, const void* b_pool, void* x_pool,
                                void* h_pool, void* q_pool, const tvs_batch_params* params,
                                int64_t* n_prox_out);
/* FGP tile variant used by tvs_proxskip_batched for batches of n_slices
 * slices in this context (-1 restores the default). */
tvs_status tvs_fgp_set_variant_batched(tvs_ctx* ctx, tvs_dtype dtype, int n_slices, int index);
/* Times every FGP variant on the FGP passes a run of these slices makes at
 * its first 8 outer iterations (k0 = 0): each pass covers the slices whose
 * coin (seed, stream_id, p) is 1 at that iteration, or every slice when
 * none is; seeded random data on private pools, offsets ignored.  Keeps the
 * fastest for n_slices slices; ms_per_iter_out gets each variant's time per
 * FGP iteration of one such pass (-1 if not compiled for the dtype).
 * Outputs as tvs_fgp_autotune. */
tvs_status tvs_fgp_autotune_batched(tvs_ctx* ctx, tvs_dtype dtype, int n_slices,
                                    const tvs_slice* slices, int inner_iters, int reps,
                                    int* best_index, double* ms_per_iter_out);
/* The variant a batch of n_slices slices would use now. */
tvs_status tvs_fgp_query_batched(tvs_ctx* ctx, tvs_dtype dtype, int n_slices, int* index,
                                 double* ms_per_iter);

/* ------------------------------------------------------------ learned prox
 * A learned replacement for the inner TV-prox solver of Sec. 3 (the prox of
 * eq. (3) with R = TV).  A 3x3 convolutional network, channels 2 -> 32 ->
 * 32 -> 32 -> 2 with ReLU between layers and zero padding, maps the prox
 * input v and a constant map of the prox weight lam to a dual field qt
 * [2][H][W]; the prox output is recovered as the dual method recovers it
 * (u = b + div q, Sec. 2.1, with the ball projection of eq. (7)):
 *
 *     q = P_lam(qt),   z = P_X(v + div q)      (P_X = max(., 0) if nonneg)
 *
 * so every prediction has an exact duality gap and is a valid warm start for
 * FGP.  Convolutions run on the BF16 matrix cores with FP32 accumulation;
 * the master parameters, the gradient and Adam run in FP32.  The CNN works
 * on float32 data only.  The forward pass carries every operand as two BF16
 * parts (x = hi + lo) and takes three products per K slice (hi hi, hi lo,
 * lo hi), which brings its error near FP32's; the backward pass uses single
 * BF16 operands.  tvs_cnn_set_fast_forward switches the forward and prox
 * calls (not training) to single BF16 operands.
 *
 * Parameter vector (float32, tvs_cnn_param_count() = 19682 entries): for
 * layer l = 1..4 with (C_in, C_out) = (2,32), (32,32), (32,32), (32,2):
 * W_l[9][C_in][C_out] then b_l[C_out]; tap t = 3 * (row offset + 1) +
 * (column offset + 1), out(p) = b + sum_t sum_ci W[t][ci][co] in(p + o_t).
 *
 * Batches: v, z_target [n][H][W] and qt [n][2][H][W] are float32 device
 * buffers; lam_host is n doubles on the host.  Training loss:
 * L = sum [(z - z_target)^2 + mu |q - q_target|^2] / (2 n H W), the dual
 * term optional (q_target [n][2][H][W] device float32, NULL or mu = 0 drops
 * it); it fixes the dual where z alone leaves it free (D z = 0).  A tvs_cnn belongs to one context
 * and uses its stream; it owns its parameters and scratch (grow-only). */
typedef struct tvs_cnn tvs_cnn;

/* New network, He-normal weights from a counter-based generator keyed by
 * seed (zero biases), Adam state cleared. */
tvs_status tvs_cnn_create(tvs_ctx* ctx, uint64_t seed, tvs_cnn** out);
void tvs_cnn_destroy(tvs_cnn* cnn);
int64_t tvs_cnn_param_count(void);
/* Copy the FP32 master parameters to / from host memory (param_count
 * floats).  Setting parameters clears the Adam state and step count. */
tvs_status tvs_cnn_get_params(tvs_cnn* cnn, float* params_host);
tvs_status tvs_cnn_set_params(tvs_cnn* cnn, const float* params_host);
/* Forward pass: qt_out (nullable) gets the raw network output, z_out
 * (nullable) the prox estimate z.  Sizes: n >= 1, 1 <= H, W <= 32768,
 * n H W <= 2^31. */
tvs_status tvs_cnn_forward(tvs_cnn* cnn, int n, int H, int W, const float* v,
                           const double* lam_host, int nonneg, float* qt_out, float* z_out);
/* Loss (host, nullable) and its gradient with respect to the parameters
 * (grad_out: device float32[param_count], nullable; the gradient is also kept
 * for tvs_cnn_adam_step).  Synchronises when loss_out is set. */
tvs_status tvs_cnn_loss_grad(tvs_cnn* cnn, int n, int H, int W, const float* v,
                             const double* lam_host, int nonneg, const float* z_target,
                             const float* q_target, double mu, double* loss_out,
                             float* grad_out);
/* One Adam step (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8) with the
 * gradient grad (device float32[param_count]) or, when grad is NULL, the one
 * kept by the last tvs_cnn_loss_grad. */
tvs_status tvs_cnn_adam_step(tvs_cnn* cnn, const float* grad, double lr);
/* tvs_cnn_loss_grad followed by tvs_cnn_adam_step. */
tvs_status tvs_cnn_train_step(tvs_cnn* cnn, int n, int H, int W, const float* v,
                              const double* lam_host, int nonneg, const float* z_target,
                              const float* q_target, double mu, double lr, double* loss_out);
/* Learned prox of one H x W image with a duality-gap gate: the network's
 * dual q = P_lam(qt) is written to q_out [2][H][W]; if its relative gap
 * gap(q) / P(z_q) (the gap of eq. (6) in the form gap(q) = sum_i lam
 * |(D z_q)_i| - <(D z_q)_i, q_i>, P the prox objective) exceeds gap_tol
 * (or is NaN) and fallback_iters > 0, FGP runs fallback_iters iterations
 * warm-started from q (from zero when the gap is not finite) and q_out gets
 * its final dual.  z_out gets
 * P_X(v + div q_out).  fell_back_out (nullable) is set to 1 when FGP ran;
 * rel_gap_out (nullable) gets the network's relative gap.  Synchronises
 * (the gate is decided on the host). */
tvs_status tvs_cnn_prox(tvs_cnn* cnn, int H, int W, const float* v, double lam, int nonneg,
                        double gap_tol, int fallback_iters, float* q_out, float* z_out,
                        int* fell_back_out, double* rel_gap_out);
/* ------------------------------------------- solver runs with extensions
 * tvs_proxskip / tvs_pdhgskip with two optional parts, set in a
 * tvs_solve_ext (NULL: the plain call):
 *  - cnn != NULL: every prox call of the run is the learned prox with the
 *    duality-gap gate of tvs_cnn_prox, decided on the device (so the run
 *    stays one HIP graph with TVS_FLAG_GRAPH).  The previous call's dual
 *    (the warm dual the plain run reuses; zero at the first call unless the
 *    state brings one) is checked first: when its relative gap at the new
 *    prox input is at most gap_tol it is the call's dual, and neither the
 *    network nor FGP runs.  Otherwise the network's dual P_lam(qt) becomes
 *    the call's dual when its relative gap is at most gap_tol; else
 *    params->inner_iters FGP iterations run, warm-started from whichever of
 *    the two duals has the smaller relative gap.  A NaN gap falls back.
 *    float32 only (TVS_ERR_UNSUPPORTED else).
 *  - inner_p > 0 (skipping inside the inner solver, the paper's
 *    "Discussion and Future work"): every prox call solves the TV prox by
 *    params->inner_iters steps of ProxSkip on its dual instead of FGP (the
 *    dual of Sec. 2.1 with eps = 0; with nonneg the constrained dual, whose
 *    gradient is -D max(v + div q, 0)), step 1/8 and projection probability
 *    inner_p, warm-started from (state->q, inner_h).  inner_h: device, dtype,
 *    [2][H][W], the inner control variate, kept across calls and runs like q
 *    (zero it for a cold start).  The inner coin of step i of the call at
 *    outer iteration k (k0 included) is the coin of tvs_proxskip on stream
 *    stream_id xor 2^62 at index k inner_iters + i, so a resumed run draws
 *    the same schedule.  float32 and float64; excludes cnn
 *    (TVS_ERR_INVALID_ARG); inner_p outside (0, 1] or a NULL inner_h is
 *    TVS_ERR_INVALID_ARG.  inner_p = 0: FGP as in the plain call.
 *  - v_record != NULL: the prox inputs v (the argument of the prox in
 *    Alg. "ProxSkip" / "PDHGSkip-2") of the first max_record prox calls are
 *    copied to v_record (device, dtype, max_record x H x W), the pairs that
 *    train the network.
 * Outputs: n_fallback = calls where FGP ran, n_recorded = inputs stored,
 * n_inner_proj = projections the skipping inner solver made. */
typedef struct tvs_solve_ext {
    tvs_cnn* cnn;
    double gap_tol;
    void* v_record;
    int64_t max_record;
    int64_t n_fallback;   /* out */
    int64_t n_recorded;   /* out */
    double inner_p;
    void* inner_h;
    int64_t n_inner_proj; /* out */
} tvs_solve_ext;

tvs_status tvs_proxskip_ex(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                           const tvs_params* params, tvs_solve_ext* ext, double* obj_trace,
                           uint8_t* theta_trace, tvs_report* report);
tvs_status tvs_pdhgskip_ex(tvs_op* op, tvs_dtype dtype, const void* b, tvs_state* state,
                           const tvs_params* params, tvs_solve_ext* ext, double* obj_trace,
                           uint8_t* theta_trace, tvs_report* report);

/* fast != 0: tvs_cnn_forward and tvs_cnn_prox use single-part BF16
 * operands (one product per K slice, about three times fewer matrix-core
 * operations, BF16-level error); 0 (the default): two-part operands.  Also
 * applies to the learned prox inside tvs_proxskip_ex / tvs_pdhgskip_ex. */
tvs_status tvs_cnn_set_fast_forward(tvs_cnn* cnn, int fast);
/* Save / load the parameters as a little-endian binary file: the 8 bytes
 * "TVSCNN01", an int64 parameter count, then the float32 parameters.
 * Loading clears the Adam state; a file of another count is TVS_ERR_SHAPE. */
tvs_status tvs_cnn_save(tvs_cnn* cnn, const char* path);
tvs_status tvs_cnn_load(tvs_cnn* cnn, const char* path);

#ifdef __cplusplus
}
#endif
#endif /* TVSKIP_H */
