/*
 * oracle.h -- plain CPU FP64 reference ("oracle") of the ProxSkip / PDHGSkip
 * TV-regularised imaging iterations (Papoutsellis, Kereta, Papafitsoros,
 * "Why do we regularise in every iteration for imaging inverse problems?").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this code.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may use it.  It shares no code, header, table or
 * constant generator with the GPU library.
 *
 * Conventions (all arrays row-major, float64):
 *   image  u[H][W];   pixel (i, j) = row i, column j.
 *   dual   q[2][H][W]; plane 0 = y (row) component, plane 1 = x (column)
 *          component, matching D u = (D_y u, D_x u) of the problem statement
 *          in the paper's introduction (the TV definition before eq. (5)).
 *   CT sinogram y[n_ang][n_det].
 */
#ifndef TVS_ORACLE_H
#define TVS_ORACLE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- discrete operators (TV definition before eq. (5); Sec. 2.1) ---- */
void orc_grad(int H, int W, const double* u, double* q);
void orc_div(int H, int W, const double* q, double* u);
double orc_tv(int H, int W, const double* u);
void orc_proj_ball(size_t n, const double* w, double lam, double* out);

/* ---- TV prox by FGP ("AProjGD", Sec. 2.1-2.2, Sec. 3.1) ---- */
void orc_fgp(int H, int W, const double* v, double lam, int iters, int nonneg,
             double* q_inout, double* z_out);
double orc_tv_gap(int H, int W, const double* v, double lam, int nonneg,
                  const double* q, double* primal_out);

/* ---- forward operators A ---- */
enum { ORC_IDENTITY = 0, ORC_BLUR = 1, ORC_JOSEPH = 2 };
typedef struct {
    int kind;
    int H, W;
    /* blur: kernel[kh][kw], odd sizes, centre (kh/2, kw/2) */
    const double* kernel;
    int kh, kw;
    /* Joseph parallel beam */
    int n_ang;
    const double* angles;
    int n_det;
    double pixel, det_spacing;
} orc_op;

size_t orc_op_out_size(const orc_op* A);
void orc_op_apply(const orc_op* A, const double* x, double* y);
void orc_op_adjoint(const orc_op* A, const double* y, double* x);
double orc_objective(const orc_op* A, const double* b, const double* x, double alpha);

/* ---- coin stream ---- */
uint64_t orc_splitmix64_mix(uint64_t z);
int orc_coin(uint64_t seed, uint64_t stream_id, int64_t k, double p);

/* ---- outer algorithms ---- */
typedef struct {
    double alpha;      /* TV weight */
    double step;       /* gamma (ProxSkip / PGD) or sigma (PDHGSkip / PDHG) */
    double dual_step;  /* tau (PDHGSkip / PDHG) */
    double p;          /* prox probability, (0, 1] */
    int64_t outer_iters;
    int32_t inner_iters;
    int32_t nonneg;
    uint64_t seed, stream_id;
    int64_t k0;        /* first coin index */
} orc_params;

/* Alg. "ProxSkip".  x, h, q are in/out.  theta_trace (nullable) gets theta_k,
 * obj_trace (nullable) gets Phi(x_{k+1}).  Returns the number of prox calls. */
int64_t orc_proxskip(const orc_op* A, const double* b, double* x, double* h,
                     double* q, const orc_params* P, uint8_t* theta_trace,
                     double* obj_trace);
/* Alg. "PGD/ISTA/FBS" with the same FGP prox (written separately). */
void orc_pgd(const orc_op* A, const double* b, double* x, double* q,
             const orc_params* P, double* obj_trace);
/* Alg. "PDHGSkip-2".  y is the dual (data-space) iterate. */
int64_t orc_pdhgskip(const orc_op* A, const double* b, double* x, double* h,
                     double* y, double* q, const orc_params* P,
                     uint8_t* theta_trace, double* obj_trace);
/* PDHG (Chambolle-Pock) with the same FGP prox (written separately). */
void orc_pdhg(const orc_op* A, const double* b, double* x, double* y,
              double* q, const orc_params* P, double* obj_trace);

/* Stochastic angle subsets (the paper's "Discussion and Future work"):
 * subset j of n holds the angles a with a mod n = j; the subset drawn at
 * outer iteration k is orc_subset(seed, stream_id, k, n), uniform on
 * {0, ..., n-1}, from the coin's generator on stream stream_id xor 2^63. */
int orc_subset(uint64_t seed, uint64_t stream_id, int64_t k, int n);
/* The rows of A (Joseph) for angle subset j of n: y_j has
 * ceil((n_ang - j) / n) rows, row i = angle j + i n. */
void orc_subset_apply(const orc_op* A, int n, int j, const double* x, double* yj);
void orc_subset_adjoint(const orc_op* A, int n, int j, const double* yj, double* x);
/* SPDHG (Chambolle, Ehrhardt, Richtarik, Schoenlieb 2018) over angle subsets
 * with the prox of g skipped as in Alg. "PDHGSkip-2".  y (full sinogram, in
 * natural angle order), x, h, q are in/out; every call starts from
 * z = zbar = A^T y.  subset_trace (nullable) gets j_k.  Returns the number
 * of prox calls. */
int64_t orc_spdhgskip(const orc_op* A, const double* b, int n_sub, double* x, double* h,
                      double* y, double* q, const orc_params* P, uint8_t* theta_trace,
                      int32_t* subset_trace, double* obj_trace);

/* Alg. "FISTA" (read as Beck and Teboulle's: t_{k+1} = (1 + sqrt(1 + 4
 * t_k^2)) / 2, xbar = x_k + ((t_k - 1) / t_{k+1})(x_k - x_{k-1}),
 * x_{k+1} = prox_{gamma g}(xbar - gamma grad f(xbar))) with the same FGP
 * prox, warm started.  Every call restarts the momentum (t_1 = 1,
 * x_{k-1} = x_k).  x, q in/out. */
void orc_fista(const orc_op* A, const double* b, double* x, double* q,
               const orc_params* P, double* obj_trace);
/* Alg. "PDHGSkip-1" (Condat et al.'s skipped PDHG, with the bracket read as
 * K(x_{k+1} + xhat_k) and omega + 1 = 1/p):
 *   theta_k = 1: x+ = prox_{sigma g}(x_k - sigma K^T y_k); else x+ = x_k;
 *   e = x_{k+1} + xhat_k = (1 + 1/p) x+ - x_k / p (theta_k = 1), x_k (theta_k = 0);
 *   y_{k+1} = (y_k + tau (K e - b)) / (1 + tau).
 * x, y, q in/out.  Returns the number of prox calls. */
int64_t orc_pdhgskip1(const orc_op* A, const double* b, double* x, double* y,
                      double* q, const orc_params* P, uint8_t* theta_trace,
                      double* obj_trace);

/* Operator norm by power iteration on A^T A from a seeded start vector. */
double orc_op_norm(const orc_op* A, int iters, uint64_t seed);

/* Reference minimiser by diagonally preconditioned explicit PDHG with
 * K = [A; D] (the paper's reference solver of Sec. 3.1).  Runs `iters`
 * iterations; obj_every > 0 records Phi every obj_every iterations. */
void orc_pdhg_explicit(const orc_op* A, const double* b, double alpha,
                       int nonneg, int64_t iters, double* x, double* y1,
                       double* y2, int64_t obj_every, double* obj_trace);

/* ---- light-prox problems (Sec. 2.1-2.2): ProxSkip on Dual-ROF and
 * Dual-Huber-ROF (eps > 0), and ProjGD written separately ---- */
int64_t orc_dual_rof_proxskip(int H, int W, const double* b, double alpha, double eps,
                              double gamma, double p, int64_t K, uint64_t seed,
                              uint64_t stream, int64_t k0, double* q, double* h,
                              uint8_t* theta_trace, const double* u_ref, double* err_trace);
void orc_dual_rof_projgd(int H, int W, const double* b, double alpha, double eps, double gamma,
                         int64_t K, double* q);

/* ---- skipping inside the inner solver ("Discussion and Future work"): the
 * TV prox by ProxSkip on its dual (step 1/8, projection probability p_in,
 * with u >= 0 the constrained dual, gradient -D P_X(v + div q)); q, h
 * ([2][H][W]) in/out, z_out = P_X(v + div q).  Returns the projections. */
int64_t orc_tv_prox_skip(int H, int W, const double* v, double lam, int nonneg, int iters,
                         double p_in, uint64_t seed, uint64_t stream, int64_t k0, double* q,
                         double* h, double* z_out);
/* ProxSkip / PDHGSkip-2 with that prox: inner_iters inner steps per call,
 * inner coins on stream stream_id xor 2^62 at indices k inner_iters + i
 * (k the outer iteration), inner control variate h_in kept across calls.
 * n_proj_out (nullable) gets the inner projections; returns the prox calls. */
int64_t orc_proxskip_inner(const orc_op* A, const double* b, double* x, double* h, double* q,
                           double* h_in, double p_in, const orc_params* P,
                           uint8_t* theta_trace, double* obj_trace, int64_t* n_proj_out);
int64_t orc_pdhgskip_inner(const orc_op* A, const double* b, double* x, double* h, double* y,
                           double* q, double* h_in, double p_in, const orc_params* P,
                           uint8_t* theta_trace, double* obj_trace, int64_t* n_proj_out);

/* ---- learned TV prox (cnn.c): 2 -> 32 -> 32 -> 32 -> 2, 3x3, dual output ---- */
#define ORC_CNN_LAYERS 4
size_t orc_cnn_param_count(void);
/* v: [n][H][W], lam: [n]; qt_out (nullable): [n][2][H][W] raw network output;
 * z_out (nullable): [n][H][W] = P_X(v + div P_lam(qt)). */
void orc_cnn_forward(int n, int H, int W, const double* v, const double* lam, int nonneg,
                     const double* params, double* qt_out, double* z_out);
/* Loss sum [(z - z_target)^2 + mu |q - q_target|^2] / (2 n H W), q =
 * P_lam(qt), q_target [n][2][H][W] nullable, and its gradient (nullable). */
double orc_cnn_loss_grad(int n, int H, int W, const double* v, const double* lam,
                         int nonneg, const double* params, const double* z_target,
                         const double* q_target, double mu, double* grad);
void orc_adam_step(size_t n, double* params, const double* grad, double* m, double* v,
                   int64_t step, double lr, double beta1, double beta2, double eps);

#ifdef __cplusplus
}
#endif
#endif
