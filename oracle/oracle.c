/*
 * oracle.c -- plain CPU FP64 reference of the ProxSkip / PDHGSkip TV hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product library.  Every function
 * writes out the definition it follows, in the paper's order and notation,
 * with no blocking, fusion or reordering; OpenMP is used only to split
 * independent rows (or rays) across threads, never to reorder a sum.
 *
 * Readings of passages that the paper leaves open (boundary conventions,
 * the projection formula, the PDHGSkip indices, the coin) are stated at
 * each function.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* images smaller than this run single-threaded (a parallel region costs
 * more than the loop) */
#define ORC_PAR_MIN 16384

#define AT(a, i, j) ((a)[(size_t)(i) * (size_t)W + (size_t)(j)])

static double* dalloc(size_t n) {
    double* p = (double*)calloc(n ? n : 1, sizeof(double));
    if (!p) abort();
    return p;
}

/* ------------------------------------------------------------------------
 * Discrete gradient D = (D_y, D_x): forward differences under Neumann
 * boundary conditions (TV definition before eq. (5)).  Reading: the
 * difference is zero in the last row (D_y) and last column (D_x).
 * ------------------------------------------------------------------------ */
void orc_grad(int H, int W, const double* u, double* q) {
    double* qy = q;
    double* qx = q + (size_t)H * W;
#pragma omp parallel for schedule(static) if ((size_t)H * W >= ORC_PAR_MIN)
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            AT(qy, i, j) = (i < H - 1) ? AT(u, i + 1, j) - AT(u, i, j) : 0.0;
            AT(qx, i, j) = (j < W - 1) ? AT(u, i, j + 1) - AT(u, i, j) : 0.0;
        }
    }
}

/* Discrete divergence div = -D^T (Sec. 2.1, below eq. (6)).  Writing out
 * -D^T q entry by entry for the forward differences above: each pixel
 * receives +q at its own position (if that difference exists) and -q from
 * the pixel before it (if that difference exists). */
void orc_div(int H, int W, const double* q, double* out) {
    const double* qy = q;
    const double* qx = q + (size_t)H * W;
#pragma omp parallel for schedule(static) if ((size_t)H * W >= ORC_PAR_MIN)
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            double d = 0.0;
            if (i < H - 1) d += AT(qy, i, j);
            if (i > 0) d -= AT(qy, i - 1, j);
            if (j < W - 1) d += AT(qx, i, j);
            if (j > 0) d -= AT(qx, i, j - 1);
            AT(out, i, j) = d;
        }
    }
}

/* Isotropic TV(u) = sum_i |((D_y u)_i, (D_x u)_i)|_2 (before eq. (5)). */
double orc_tv(int H, int W, const double* u) {
    double s = 0.0;
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            double dy = (i < H - 1) ? AT(u, i + 1, j) - AT(u, i, j) : 0.0;
            double dx = (j < W - 1) ? AT(u, i, j + 1) - AT(u, i, j) : 0.0;
            s += sqrt(dy * dy + dx * dx);
        }
    }
    return s;
}

/* Pixelwise projection onto {q : |q_i|_2 <= lam}, eq. (7).  The printed
 * formula x / max{alpha, |x|} is garbled (it maps onto the unit ball and
 * divides by alpha inside it); the reading used is the projection onto the
 * ball of radius lam:  q_i * min(1, lam / |q_i|), taken with the strict
 * branch |q_i| > lam so that lam = 0 or q_i = 0 never divides 0 by 0. */
void orc_proj_ball(size_t n, const double* w, double lam, double* out) {
#pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (long long i = 0; i < (long long)n; ++i) {
        double wy = w[i], wx = w[n + i];
        double nrm = sqrt(wy * wy + wx * wx);
        double s = (nrm > lam) ? lam / nrm : 1.0;
        out[i] = wy * s;
        out[n + i] = wx * s;
    }
}

static void proj_x(size_t n, double* z, int nonneg) {
    if (!nonneg) return;
    for (size_t i = 0; i < n; ++i) z[i] = (z[i] > 0.0) ? z[i] : 0.0;
}

/* ------------------------------------------------------------------------
 * TV prox  z = argmin_z 1/2 |z - v|^2 + lam TV(z) (+ indicator z >= 0),
 * eq. (3) with R = TV, solved on the dual (Dual-ROF, eq. (6)) by the
 * accelerated projected gradient iteration the paper calls AProjGD:
 * projected gradient (Sec. 2.1, step 1/L with L = |D|^2 <= 8, Sec. 2.1)
 * plus the FISTA momentum (Alg. "FISTA"; Sec. 2.2 describes AProjGD as GD
 * with the FISTA acceleration step).  This is Beck and Teboulle's FGP.
 *
 * Reading of the momentum (the printed FISTA extrapolation is garbled): the
 * Beck-Teboulle sequence  t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2,
 * r_{k+1} = q_k + ((t_k - 1) / t_{k+1}) (q_k - q_{k-1}), t_1 = 1.
 * Warm start (Sec. 3.1): q_inout carries the dual between calls; t and the
 * previous dual restart at every call.  nonneg adds the projection P_X onto
 * z >= 0 inside the primal map (the CT problem of Sec. 3.3).
 * ------------------------------------------------------------------------ */
void orc_fgp(int H, int W, const double* v, double lam, int iters, int nonneg,
             double* q, double* z) {
    size_t n = (size_t)H * W;
    double* q_prev = dalloc(2 * n);
    double* r = dalloc(2 * n);
    double* g = dalloc(2 * n);
    double* q_new = dalloc(2 * n);
    double* dv = dalloc(n);
    double* zz = dalloc(n);
    memcpy(q_prev, q, 2 * n * sizeof(double));
    memcpy(r, q, 2 * n * sizeof(double));
    double t = 1.0;
    for (int k = 0; k < iters; ++k) {
        /* primal point of the current dual point: z = P_X(v + div r) */
        orc_div(H, W, r, dv);
        for (size_t i = 0; i < n; ++i) zz[i] = v[i] + dv[i];
        proj_x(n, zz, nonneg);
        /* projected gradient step on the dual, step 1/8 */
        orc_grad(H, W, zz, g);
        for (size_t i = 0; i < 2 * n; ++i) q_new[i] = r[i] + 0.125 * g[i];
        orc_proj_ball(n, q_new, lam, q_new);
        /* FISTA momentum */
        double t_next = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
        double beta = (t - 1.0) / t_next;
        for (size_t i = 0; i < 2 * n; ++i) r[i] = q_new[i] + beta * (q_new[i] - q_prev[i]);
        memcpy(q_prev, q_new, 2 * n * sizeof(double));
        t = t_next;
    }
    memcpy(q, q_prev, 2 * n * sizeof(double));
    /* primal solution from the dual: u = b + div q (Sec. 2.1) */
    orc_div(H, W, q, dv);
    for (size_t i = 0; i < n; ++i) z[i] = v[i] + dv[i];
    proj_x(n, z, nonneg);
    free(q_prev); free(r); free(g); free(q_new); free(dv); free(zz);
}

/* Duality gap of the TV prox at the dual point q (the paper cites duality-gap
 * checks of the inner solver in Sec. 3.3 without a formula; derived here).
 * With z_q = P_X(v + div q):
 *   primal P(z) = 1/2 |z - v|^2 + lam TV(z),
 *   gap(q) = P(z_q) - D(q) = sum_i lam |(D z_q)_i| - <(D z_q)_i, q_i>  >= 0
 * for |q_i| <= lam (the 1/2|z - v|^2 terms cancel, also with z >= 0).
 * Returns the gap; *primal_out (nullable) gets P(z_q). */
double orc_tv_gap(int H, int W, const double* v, double lam, int nonneg,
                  const double* q, double* primal_out) {
    size_t n = (size_t)H * W;
    double* z = dalloc(n);
    double* g = dalloc(2 * n);
    orc_div(H, W, q, z);
    for (size_t i = 0; i < n; ++i) z[i] += v[i];
    proj_x(n, z, nonneg);
    orc_grad(H, W, z, g);
    double gap = 0.0, tv = 0.0, fid = 0.0;
    for (size_t i = 0; i < n; ++i) {
        double gy = g[i], gx = g[n + i];
        double nrm = sqrt(gy * gy + gx * gx);
        gap += lam * nrm - (gy * q[i] + gx * q[n + i]);
        tv += nrm;
        fid += (z[i] - v[i]) * (z[i] - v[i]);
    }
    if (primal_out) *primal_out = 0.5 * fid + lam * tv;
    free(z); free(g);
    return gap;
}

/* ------------------------------------------------------------------------
 * Forward operators A and their adjoints.
 * ------------------------------------------------------------------------ */
size_t orc_op_out_size(const orc_op* A) {
    if (A->kind == ORC_JOSEPH) return (size_t)A->n_ang * A->n_det;
    return (size_t)A->H * A->W;
}

static int pmod(int a, int m) { int r = a % m; return r < 0 ? r + m : r; }

/* Periodic convolution (the deblurring operator of Sec. 3.1; the paper does
 * not fix the kernel or boundary, the workload fixes a periodic one):
 *   (A x)_{i,j} = sum_{m,n} k_{m,n} x_{(i-m) mod H, (j-n) mod W},
 * with k_{m,n} = kernel[m + kh/2][n + kw/2]. */
static void blur_apply(const orc_op* A, const double* x, double* y) {
    int H = A->H, W = A->W, ch = A->kh / 2, cw = A->kw / 2;
#pragma omp parallel for schedule(static) if ((size_t)H * W >= ORC_PAR_MIN)
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            double s = 0.0;
            for (int a = 0; a < A->kh; ++a)
                for (int c = 0; c < A->kw; ++c)
                    s += A->kernel[a * A->kw + c] * AT(x, pmod(i - (a - ch), H), pmod(j - (c - cw), W));
            AT(y, i, j) = s;
        }
    }
}

/* Adjoint of the periodic convolution: correlation with the same kernel,
 *   (A^T y)_{i,j} = sum_{m,n} k_{m,n} y_{(i+m) mod H, (j+n) mod W}. */
static void blur_adjoint(const orc_op* A, const double* y, double* x) {
    int H = A->H, W = A->W, ch = A->kh / 2, cw = A->kw / 2;
#pragma omp parallel for schedule(static) if ((size_t)H * W >= ORC_PAR_MIN)
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            double s = 0.0;
            for (int a = 0; a < A->kh; ++a)
                for (int c = 0; c < A->kw; ++c)
                    s += A->kernel[a * A->kw + c] * AT(y, pmod(i + (a - ch), H), pmod(j + (c - cw), W));
            AT(x, i, j) = s;
        }
    }
}

/* Discrete Radon transform of the CT experiment (Sec. 3.3), which the paper
 * does not discretise; the reading is Joseph's ray-driven projector:
 *   pixel centres (x_j, y_i) = ((j - (W-1)/2) d, ((H-1)/2 - i) d), d = pixel;
 *   bin centres s_b = (b - (n_det-1)/2) ds;  ray {x cos t + y sin t = s_b}.
 *   If |cos t| >= |sin t| the ray is sampled once per row i at
 *   x = (s_b - y_i sin t) / cos t, i.e. at the continuous column
 *   c = x / d + (W-1)/2, linearly interpolated between columns floor(c) and
 *   floor(c) + 1 (weights 1 - f, f with f = c - floor(c); a column outside
 *   the image contributes 0), and the sum is weighted by d / |cos t|.
 *   Otherwise the roles of rows and columns swap: sampled once per column j
 *   at the continuous row r = (H-1)/2 - y / d with y = (s_b - x_j cos t) /
 *   sin t, weighted by d / |sin t|. */
static void joseph_apply(const orc_op* A, const double* x, double* y) {
    int H = A->H, W = A->W, na = A->n_ang, nd = A->n_det;
    double px = A->pixel, ds = A->det_spacing;
#pragma omp parallel for schedule(static) if ((size_t)H * W >= ORC_PAR_MIN)
    for (long long ray = 0; ray < (long long)na * nd; ++ray) {
        int a = (int)(ray / nd), b = (int)(ray % nd);
        double c = cos(A->angles[a]), s = sin(A->angles[a]);
        double sb = (b - (nd - 1) / 2.0) * ds;
        double acc = 0.0, wgt;
        if (fabs(c) >= fabs(s)) {
            wgt = px / fabs(c);
            for (int i = 0; i < H; ++i) {
                double yi = ((H - 1) / 2.0 - i) * px;
                double xx = (sb - yi * s) / c;
                double cc = xx / px + (W - 1) / 2.0;
                double fl = floor(cc), f = cc - fl;
                long j0 = (long)fl;
                if (j0 >= 0 && j0 < W) acc += (1.0 - f) * AT(x, i, j0);
                if (j0 + 1 >= 0 && j0 + 1 < W) acc += f * AT(x, i, j0 + 1);
            }
        } else {
            wgt = px / fabs(s);
            for (int j = 0; j < W; ++j) {
                double xj = (j - (W - 1) / 2.0) * px;
                double yy = (sb - xj * c) / s;
                double rr = (H - 1) / 2.0 - yy / px;
                double fl = floor(rr), f = rr - fl;
                long i0 = (long)fl;
                if (i0 >= 0 && i0 < H) acc += (1.0 - f) * AT(x, i0, j);
                if (i0 + 1 >= 0 && i0 + 1 < H) acc += f * AT(x, i0 + 1, j);
            }
        }
        y[ray] = acc * wgt;
    }
}

/* Exact transpose of joseph_apply, by scattering every sample's two weights
 * back into the image.  Angles are visited in order; within an angle the
 * threads own disjoint rows (row-stepping rays) or columns (column-stepping
 * rays), so no two threads touch one pixel and the sum order is fixed. */
static void joseph_adjoint(const orc_op* A, const double* y, double* x) {
    int H = A->H, W = A->W, na = A->n_ang, nd = A->n_det;
    double px = A->pixel, ds = A->det_spacing;
    memset(x, 0, (size_t)H * W * sizeof(double));
    for (int a = 0; a < na; ++a) {
        double c = cos(A->angles[a]), s = sin(A->angles[a]);
        if (fabs(c) >= fabs(s)) {
            double wgt = px / fabs(c);
#pragma omp parallel for schedule(static) if ((size_t)H * W >= ORC_PAR_MIN)
            for (int i = 0; i < H; ++i) {
                double yi = ((H - 1) / 2.0 - i) * px;
                for (int b = 0; b < nd; ++b) {
                    double sb = (b - (nd - 1) / 2.0) * ds;
                    double xx = (sb - yi * s) / c;
                    double cc = xx / px + (W - 1) / 2.0;
                    double fl = floor(cc), f = cc - fl;
                    long j0 = (long)fl;
                    double val = wgt * y[(size_t)a * nd + b];
                    if (j0 >= 0 && j0 < W) AT(x, i, j0) += (1.0 - f) * val;
                    if (j0 + 1 >= 0 && j0 + 1 < W) AT(x, i, j0 + 1) += f * val;
                }
            }
        } else {
            double wgt = px / fabs(s);
#pragma omp parallel for schedule(static) if ((size_t)H * W >= ORC_PAR_MIN)
            for (int j = 0; j < W; ++j) {
                double xj = (j - (W - 1) / 2.0) * px;
                for (int b = 0; b < nd; ++b) {
                    double sb = (b - (nd - 1) / 2.0) * ds;
                    double yy = (sb - xj * c) / s;
                    double rr = (H - 1) / 2.0 - yy / px;
                    double fl = floor(rr), f = rr - fl;
                    long i0 = (long)fl;
                    double val = wgt * y[(size_t)a * nd + b];
                    if (i0 >= 0 && i0 < H) AT(x, i0, j) += (1.0 - f) * val;
                    if (i0 + 1 >= 0 && i0 + 1 < H) AT(x, i0 + 1, j) += f * val;
                }
            }
        }
    }
}

void orc_op_apply(const orc_op* A, const double* x, double* y) {
    if (A->kind == ORC_BLUR) blur_apply(A, x, y);
    else if (A->kind == ORC_JOSEPH) joseph_apply(A, x, y);
    else memcpy(y, x, (size_t)A->H * A->W * sizeof(double));
}

void orc_op_adjoint(const orc_op* A, const double* y, double* x) {
    if (A->kind == ORC_BLUR) blur_adjoint(A, y, x);
    else if (A->kind == ORC_JOSEPH) joseph_adjoint(A, y, x);
    else memcpy(x, y, (size_t)A->H * A->W * sizeof(double));
}

/* Phi(x) = 1/2 |A x - b|^2 + alpha TV(x), eq. (5) (the non-negativity
 * indicator of the CT problem is not added). */
double orc_objective(const orc_op* A, const double* b, const double* x, double alpha) {
    size_t m = orc_op_out_size(A);
    double* Ax = dalloc(m);
    orc_op_apply(A, x, Ax);
    double s = 0.0;
    for (size_t i = 0; i < m; ++i) s += (Ax[i] - b[i]) * (Ax[i] - b[i]);
    free(Ax);
    return 0.5 * s + alpha * orc_tv(A->H, A->W, x);
}

/* ------------------------------------------------------------------------
 * Coin theta_k ~ Bernoulli(p), i.i.d. over k (Alg. "ProxSkip", Alg.
 * "PDHGSkip-2").  Counter-based so that theta_k is a pure function of
 * (seed, stream, k):  SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) with
 * the "variant 13" output mix of D. Stafford (2011), as in S. Vigna's public
 * domain splitmix64.  The stream key is mix(seed xor mix(stream + G)); the
 * k-th draw is the generator output at position k + 1 from that key,
 * mix(key + (k + 1) G); theta_k = [ (r >> 11) < floor(p 2^53) ].
 * ------------------------------------------------------------------------ */
#define ORC_GOLDEN 0x9E3779B97F4A7C15ULL

uint64_t orc_splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int orc_coin(uint64_t seed, uint64_t stream_id, int64_t k, double p) {
    if (!(p > 0.0 && p <= 1.0) || k < 0) return -1;
    uint64_t key = orc_splitmix64_mix(seed ^ orc_splitmix64_mix(stream_id + ORC_GOLDEN));
    uint64_t r = orc_splitmix64_mix(key + (uint64_t)(k + 1) * ORC_GOLDEN);
    uint64_t T = (uint64_t)floor(p * 9007199254740992.0); /* p * 2^53 */
    return (r >> 11) < T ? 1 : 0;
}

/* ------------------------------------------------------------------------
 * Outer algorithms.
 * ------------------------------------------------------------------------ */

/* grad f(x) = A^T (A x - b) for f = 1/2 |A x - b|^2 (eq. (5)). */
static void data_grad(const orc_op* A, const double* b, const double* x,
                      double* res, double* g) {
    size_t m = orc_op_out_size(A);
    orc_op_apply(A, x, res);
    for (size_t i = 0; i < m; ++i) res[i] -= b[i];
    orc_op_adjoint(A, res, g);
}

/* ProxSkip (Alg. "ProxSkip") with g = alpha TV (+ z >= 0), prox by FGP.
 *   xhat_{k+1} = x_k - gamma (grad f(x_k) - h_k)
 *   theta_k = 1:  x_{k+1} = prox_{(gamma/p) g}(xhat_{k+1} - (gamma/p) h_k)
 *   theta_k = 0:  x_{k+1} = xhat_{k+1}
 *   h_{k+1} = h_k + (p/gamma)(x_{k+1} - xhat_{k+1})  (unchanged when skipped)
 * The prox argument is formed as w + (gamma - gamma/p) h_k with
 * w = x_k - gamma grad f(x_k); it equals xhat - (gamma/p) h in exact
 * arithmetic and is exactly w at p = 1, where the paper states that ProxSkip
 * and PGD coincide (Sec. 2.1). */
int64_t orc_proxskip(const orc_op* A, const double* b, double* x, double* h,
                     double* q, const orc_params* P, uint8_t* theta_trace,
                     double* obj_trace) {
    int H = A->H, W = A->W;
    size_t n = (size_t)H * W, m = orc_op_out_size(A);
    double gamma = P->step, p = P->p;
    double lam = P->alpha * gamma / p;
    double coef = gamma - gamma / p;
    double rate = p / gamma;
    double* res = dalloc(m);
    double* g = dalloc(n);
    double* w = dalloc(n);
    double* xhat = dalloc(n);
    double* v = dalloc(n);
    double* z = dalloc(n);
    int64_t nprox = 0;
    for (int64_t kk = 0; kk < P->outer_iters; ++kk) {
        int64_t k = P->k0 + kk;
        data_grad(A, b, x, res, g);
        for (size_t i = 0; i < n; ++i) {
            w[i] = x[i] - gamma * g[i];
            xhat[i] = w[i] + gamma * h[i];
        }
        int th = orc_coin(P->seed, P->stream_id, k, p);
        if (th) {
            for (size_t i = 0; i < n; ++i) v[i] = w[i] + coef * h[i];
            orc_fgp(H, W, v, lam, P->inner_iters, P->nonneg, q, z);
            for (size_t i = 0; i < n; ++i) {
                h[i] = h[i] + rate * (z[i] - xhat[i]);
                x[i] = z[i];
            }
            ++nprox;
        } else {
            memcpy(x, xhat, n * sizeof(double));
        }
        if (theta_trace) theta_trace[kk] = (uint8_t)th;
        if (obj_trace) obj_trace[kk] = orc_objective(A, b, x, P->alpha);
    }
    free(res); free(g); free(w); free(xhat); free(v); free(z);
    return nprox;
}

/* PGD / ISTA / FBS (Alg. "PGD/ISTA/FBS"):
 *   x_{k+1} = prox_{gamma g}(x_k - gamma grad f(x_k)), same warm-started FGP. */
void orc_pgd(const orc_op* A, const double* b, double* x, double* q,
             const orc_params* P, double* obj_trace) {
    int H = A->H, W = A->W;
    size_t n = (size_t)H * W, m = orc_op_out_size(A);
    double gamma = P->step;
    double lam = P->alpha * gamma;
    double* res = dalloc(m);
    double* g = dalloc(n);
    double* w = dalloc(n);
    for (int64_t k = 0; k < P->outer_iters; ++k) {
        data_grad(A, b, x, res, g);
        for (size_t i = 0; i < n; ++i) w[i] = x[i] - gamma * g[i];
        orc_fgp(H, W, w, lam, P->inner_iters, P->nonneg, q, x);
        if (obj_trace) obj_trace[k] = orc_objective(A, b, x, P->alpha);
    }
    free(res); free(g); free(w);
}

/* PDHGSkip-2 (Alg. "PDHGSkip-2") with K = A, f = 1/2 |. - b|^2, g = alpha TV
 * (+ z >= 0), the implicit formulation of Sec. 3.2.
 * Reading of two printed indices: the dual update uses K xbar_{k+1} (the
 * extrapolation just formed) and the control-variate update uses xhat_k (the
 * point formed in the same iteration); with these, p = 1 gives PDHG.
 *   xhat_k = x_k - sigma (K^T y_k - h_k)
 *   theta_k = 1: x_{k+1} = prox_{(sigma/p) g}(xhat_k - (sigma/p) h_k)
 *   theta_k = 0: x_{k+1} = xhat_k
 *   xbar = 2 x_{k+1} - x_k
 *   y_{k+1} = prox_{tau f*}(y_k + tau K xbar) = (y_k + tau (K xbar - b)) / (1 + tau)
 *   h_{k+1} = h_k + (p/sigma)(x_{k+1} - xhat_k)
 * The prox argument is formed as w + (sigma - sigma/p) h_k with
 * w = x_k - sigma K^T y_k, as in ProxSkip. */
int64_t orc_pdhgskip(const orc_op* A, const double* b, double* x, double* h,
                     double* y, double* q, const orc_params* P,
                     uint8_t* theta_trace, double* obj_trace) {
    int H = A->H, W = A->W;
    size_t n = (size_t)H * W, m = orc_op_out_size(A);
    double sigma = P->step, tau = P->dual_step, p = P->p;
    double lam = P->alpha * sigma / p;
    double coef = sigma - sigma / p;
    double rate = p / sigma;
    double* kty = dalloc(n);
    double* w = dalloc(n);
    double* xhat = dalloc(n);
    double* v = dalloc(n);
    double* z = dalloc(n);
    double* xbar = dalloc(n);
    double* kx = dalloc(m);
    int64_t nprox = 0;
    for (int64_t kk = 0; kk < P->outer_iters; ++kk) {
        int64_t k = P->k0 + kk;
        orc_op_adjoint(A, y, kty);
        for (size_t i = 0; i < n; ++i) {
            w[i] = x[i] - sigma * kty[i];
            xhat[i] = w[i] + sigma * h[i];
        }
        int th = orc_coin(P->seed, P->stream_id, k, p);
        if (th) {
            for (size_t i = 0; i < n; ++i) v[i] = w[i] + coef * h[i];
            orc_fgp(H, W, v, lam, P->inner_iters, P->nonneg, q, z);
            for (size_t i = 0; i < n; ++i) h[i] = h[i] + rate * (z[i] - xhat[i]);
            ++nprox;
        } else {
            memcpy(z, xhat, n * sizeof(double));
        }
        for (size_t i = 0; i < n; ++i) {
            xbar[i] = 2.0 * z[i] - x[i];
            x[i] = z[i];
        }
        orc_op_apply(A, xbar, kx);
        for (size_t i = 0; i < m; ++i) y[i] = (y[i] + tau * (kx[i] - b[i])) / (1.0 + tau);
        if (theta_trace) theta_trace[kk] = (uint8_t)th;
        if (obj_trace) obj_trace[kk] = orc_objective(A, b, x, P->alpha);
    }
    free(kty); free(w); free(xhat); free(v); free(z); free(xbar); free(kx);
    return nprox;
}

/* ------------------------------------------------------------------------
 * Stochastic angle subsets with the prox skip: the paper's "Discussion and
 * Future work" proposes drawing a random subset of the projection angles
 * per iteration in addition to the random prox.  The reading: SPDHG
 * (Chambolle, Ehrhardt, Richtarik and Schoenlieb, SIAM J. Optim. 28(4),
 * 2018), a published stochastic primal-dual method, with f = sum_j f_j,
 * f_j(y_j) = 1/2 |y_j - b_j|^2 over the angle subsets j, uniform sampling
 * (p_j = 1/n) and its dual extrapolation, and the primal prox of g skipped
 * with a control variate exactly as in Alg. "PDHGSkip-2":
 *   w = x_k - sigma zbar_k;  xhat = w + sigma h_k
 *   theta_k = 1: x_{k+1} = prox_{(sigma/p) g}(w + (sigma - sigma/p) h_k),
 *                h_{k+1} = h_k + (p/sigma)(x_{k+1} - xhat)
 *   theta_k = 0: x_{k+1} = xhat
 *   j = j_k:  y_j+ = prox_{tau f_j*}(y_j + tau A_j x_{k+1})
 *                  = (y_j + tau (A_j x_{k+1} - b_j)) / (1 + tau)
 *   delta = A_j^T (y_j+ - y_j);  z_{k+1} = z_k + delta;
 *   zbar_{k+1} = z_{k+1} + n delta   (the extrapolation 1 / p_j)
 * and z_0 = zbar_0 = A^T y_0.  The subset draw comes from the coin's
 * counter-based generator on the stream stream_id xor 2^63:
 *   j_k = floor((r_k >> 11) n / 2^53), exact in 64-bit integers.
 * ------------------------------------------------------------------------ */
int orc_subset(uint64_t seed, uint64_t stream_id, int64_t k, int n) {
    if (n < 1 || k < 0) return -1;
    uint64_t s2 = stream_id ^ 0x8000000000000000ULL;
    uint64_t key = orc_splitmix64_mix(seed ^ orc_splitmix64_mix(s2 + ORC_GOLDEN));
    uint64_t r = orc_splitmix64_mix(key + (uint64_t)(k + 1) * ORC_GOLDEN);
    return (int)(((r >> 11) * (uint64_t)n) >> 53);
}

/* The Joseph operator restricted to the angles j, j + n, ... */
static orc_op subset_op(const orc_op* A, int n, int j, double* ang) {
    orc_op S = *A;
    int c = 0;
    for (int a = j; a < A->n_ang; a += n) ang[c++] = A->angles[a];
    S.n_ang = c;
    S.angles = ang;
    return S;
}

void orc_subset_apply(const orc_op* A, int n, int j, const double* x, double* yj) {
    double* ang = dalloc((size_t)A->n_ang);
    orc_op S = subset_op(A, n, j, ang);
    orc_op_apply(&S, x, yj);
    free(ang);
}

void orc_subset_adjoint(const orc_op* A, int n, int j, const double* yj, double* x) {
    double* ang = dalloc((size_t)A->n_ang);
    orc_op S = subset_op(A, n, j, ang);
    orc_op_adjoint(&S, yj, x);
    free(ang);
}

int64_t orc_spdhgskip(const orc_op* A, const double* b, int n_sub, double* x, double* h,
                      double* y, double* q, const orc_params* P, uint8_t* theta_trace,
                      int32_t* subset_trace, double* obj_trace) {
    int H = A->H, W = A->W, nd = A->n_det;
    size_t n = (size_t)H * W;
    double sigma = P->step, tau = P->dual_step, p = P->p;
    double lam = P->alpha * sigma / p;
    double coef = sigma - sigma / p;
    double rate = p / sigma;
    int rows_max = (A->n_ang + n_sub - 1) / n_sub;
    double* z = dalloc(n);
    double* zbar = dalloc(n);
    double* w = dalloc(n);
    double* xhat = dalloc(n);
    double* v = dalloc(n);
    double* xn = dalloc(n);
    double* delta = dalloc(n);
    double* kx = dalloc((size_t)rows_max * nd);
    double* dy = dalloc((size_t)rows_max * nd);
    orc_op_adjoint(A, y, z);
    memcpy(zbar, z, n * sizeof(double));
    int64_t nprox = 0;
    for (int64_t kk = 0; kk < P->outer_iters; ++kk) {
        int64_t k = P->k0 + kk;
        for (size_t i = 0; i < n; ++i) {
            w[i] = x[i] - sigma * zbar[i];
            xhat[i] = w[i] + sigma * h[i];
        }
        int th = orc_coin(P->seed, P->stream_id, k, p);
        if (th) {
            for (size_t i = 0; i < n; ++i) v[i] = w[i] + coef * h[i];
            orc_fgp(H, W, v, lam, P->inner_iters, P->nonneg, q, xn);
            for (size_t i = 0; i < n; ++i) h[i] = h[i] + rate * (xn[i] - xhat[i]);
            ++nprox;
        } else {
            memcpy(xn, xhat, n * sizeof(double));
        }
        memcpy(x, xn, n * sizeof(double));
        int j = orc_subset(P->seed, P->stream_id, k, n_sub);
        orc_subset_apply(A, n_sub, j, x, kx);
        int r = 0;
        for (int a = j; a < A->n_ang; a += n_sub, ++r) {
            for (int d = 0; d < nd; ++d) {
                size_t o = (size_t)a * nd + d, oj = (size_t)r * nd + d;
                double yn = (y[o] + tau * (kx[oj] - b[o])) / (1.0 + tau);
                dy[oj] = yn - y[o];
                y[o] = yn;
            }
        }
        orc_subset_adjoint(A, n_sub, j, dy, delta);
        for (size_t i = 0; i < n; ++i) {
            z[i] = z[i] + delta[i];
            zbar[i] = z[i] + (double)n_sub * delta[i];
        }
        if (theta_trace) theta_trace[kk] = (uint8_t)th;
        if (subset_trace) subset_trace[kk] = j;
        if (obj_trace) obj_trace[kk] = orc_objective(A, b, x, P->alpha);
    }
    free(z); free(zbar); free(w); free(xhat); free(v); free(xn); free(delta); free(kx); free(dy);
    return nprox;
}

/* ------------------------------------------------------------------------
 * Alg. "FISTA" with the FGP prox.  The printed momentum (a_k = t_{k-1} /
 * t_{k+1} and x_k - x_{k+1}) is read as Beck and Teboulle's (t_k - 1) /
 * t_{k+1} applied to x_k - x_{k-1}:
 *   xbar = x_k + beta_k (x_k - x_{k-1}),  beta_k = (t_k - 1) / t_{k+1},
 *   x_{k+1} = prox_{gamma g}(xbar - gamma A^T (A xbar - b)),
 * t_1 = 1 and x_0 = x_{-1} = x at the start of each call (so beta_1 = 0,
 * the first step is a plain proximal gradient step).
 * ------------------------------------------------------------------------ */
void orc_fista(const orc_op* A, const double* b, double* x, double* q,
               const orc_params* P, double* obj_trace) {
    int H = A->H, W = A->W;
    size_t n = (size_t)H * W, m = orc_op_out_size(A);
    double gamma = P->step, lam = P->alpha * P->step;
    double* xprev = dalloc(n);
    double* xbar = dalloc(n);
    double* g = dalloc(n);
    double* v = dalloc(n);
    double* xn = dalloc(n);
    double* res = dalloc(m);
    memcpy(xprev, x, n * sizeof(double));
    double t = 1.0;
    for (int64_t k = 0; k < P->outer_iters; ++k) {
        double tn = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
        double beta = (t - 1.0) / tn;
        for (size_t i = 0; i < n; ++i) xbar[i] = x[i] + beta * (x[i] - xprev[i]);
        data_grad(A, b, xbar, res, g);
        for (size_t i = 0; i < n; ++i) v[i] = xbar[i] - gamma * g[i];
        orc_fgp(H, W, v, lam, P->inner_iters, P->nonneg, q, xn);
        memcpy(xprev, x, n * sizeof(double));
        memcpy(x, xn, n * sizeof(double));
        t = tn;
        if (obj_trace) obj_trace[k] = orc_objective(A, b, x, P->alpha);
    }
    free(xprev); free(xbar); free(g); free(v); free(xn); free(res);
}

/* ------------------------------------------------------------------------
 * Alg. "PDHGSkip-1" (the skipped PDHG of Condat et al. that the paper
 * compares with): B_p(z) = z / p with probability p, else 0;
 *   xhat_k = B_p(prox_{sigma g}(x_k - sigma K^T y_k) - x_k)
 *   x_{k+1} = x_k + xhat_k / (1 + omega),  omega + 1 = 1/p (the paper's choice)
 *   y_{k+1} = prox_{tau f*}(y_k + tau K(x_{k+1} + xhat_k))   (bracket read as
 *             K applied to x_{k+1} + xhat_k).
 * With omega + 1 = 1/p, x_{k+1} = prox(...) when theta_k = 1 and x_k
 * otherwise; x_{k+1} + xhat_k = (1 + 1/p) x+ - x_k / p, which is 2 x+ - x_k
 * bit for bit at p = 1, so the method is PDHG there.  On skipped iterations
 * neither K^T y nor the prox is needed.
 * ------------------------------------------------------------------------ */
int64_t orc_pdhgskip1(const orc_op* A, const double* b, double* x, double* y,
                      double* q, const orc_params* P, uint8_t* theta_trace,
                      double* obj_trace) {
    int H = A->H, W = A->W;
    size_t n = (size_t)H * W, m = orc_op_out_size(A);
    double sigma = P->step, tau = P->dual_step, p = P->p;
    double lam = P->alpha * sigma;
    double c1 = 1.0 + 1.0 / p, c2 = 1.0 / p;
    double* kty = dalloc(n);
    double* w = dalloc(n);
    double* xn = dalloc(n);
    double* e = dalloc(n);
    double* ke = dalloc(m);
    int64_t nprox = 0;
    for (int64_t kk = 0; kk < P->outer_iters; ++kk) {
        int64_t k = P->k0 + kk;
        int th = orc_coin(P->seed, P->stream_id, k, p);
        if (th) {
            orc_op_adjoint(A, y, kty);
            for (size_t i = 0; i < n; ++i) w[i] = x[i] - sigma * kty[i];
            orc_fgp(H, W, w, lam, P->inner_iters, P->nonneg, q, xn);
            for (size_t i = 0; i < n; ++i) {
                e[i] = c1 * xn[i] - c2 * x[i];
                x[i] = xn[i];
            }
            ++nprox;
        } else {
            memcpy(e, x, n * sizeof(double));
        }
        orc_op_apply(A, e, ke);
        for (size_t i = 0; i < m; ++i) y[i] = (y[i] + tau * (ke[i] - b[i])) / (1.0 + tau);
        if (theta_trace) theta_trace[kk] = (uint8_t)th;
        if (obj_trace) obj_trace[kk] = orc_objective(A, b, x, P->alpha);
    }
    free(kty); free(w); free(xn); free(e); free(ke);
    return nprox;
}

/* PDHG (Chambolle-Pock), primal step first, in the same notation:
 *   x_{k+1} = prox_{sigma g}(x_k - sigma K^T y_k);  xbar = 2 x_{k+1} - x_k;
 *   y_{k+1} = (y_k + tau (K xbar - b)) / (1 + tau). */
void orc_pdhg(const orc_op* A, const double* b, double* x, double* y,
              double* q, const orc_params* P, double* obj_trace) {
    int H = A->H, W = A->W;
    size_t n = (size_t)H * W, m = orc_op_out_size(A);
    double sigma = P->step, tau = P->dual_step;
    double lam = P->alpha * sigma;
    double* kty = dalloc(n);
    double* w = dalloc(n);
    double* xn = dalloc(n);
    double* xbar = dalloc(n);
    double* kx = dalloc(m);
    for (int64_t k = 0; k < P->outer_iters; ++k) {
        orc_op_adjoint(A, y, kty);
        for (size_t i = 0; i < n; ++i) w[i] = x[i] - sigma * kty[i];
        orc_fgp(H, W, w, lam, P->inner_iters, P->nonneg, q, xn);
        for (size_t i = 0; i < n; ++i) {
            xbar[i] = 2.0 * xn[i] - x[i];
            x[i] = xn[i];
        }
        orc_op_apply(A, xbar, kx);
        for (size_t i = 0; i < m; ++i) y[i] = (y[i] + tau * (kx[i] - b[i])) / (1.0 + tau);
        if (obj_trace) obj_trace[k] = orc_objective(A, b, x, P->alpha);
    }
    free(kty); free(w); free(xn); free(xbar); free(kx);
}

/* |A|_2 by power iteration on A^T A (used for sigma tau |K|^2 <= 1,
 * Sec. 3.3).  Start vector: uniform [-1/2, 1/2) values from the SplitMix64
 * stream of `seed`. */
double orc_op_norm(const orc_op* A, int iters, uint64_t seed) {
    size_t n = (size_t)A->H * A->W, m = orc_op_out_size(A);
    double* x = dalloc(n);
    double* Ax = dalloc(m);
    double* y = dalloc(n);
    for (size_t i = 0; i < n; ++i)
        x[i] = (double)(orc_splitmix64_mix(seed + (uint64_t)(i + 1) * ORC_GOLDEN) >> 11) *
                   (1.0 / 9007199254740992.0) - 0.5;
    double nrm = 0.0;
    for (size_t i = 0; i < n; ++i) nrm += x[i] * x[i];
    nrm = sqrt(nrm);
    for (size_t i = 0; i < n; ++i) x[i] /= nrm;
    double est = 0.0;
    for (int it = 0; it < iters; ++it) {
        orc_op_apply(A, x, Ax);
        orc_op_adjoint(A, Ax, y);
        double s = 0.0;
        for (size_t i = 0; i < n; ++i) s += y[i] * y[i];
        s = sqrt(s);              /* |A^T A x| with |x| = 1 */
        est = s;
        for (size_t i = 0; i < n; ++i) x[i] = y[i] / s;
    }
    free(x); free(Ax); free(y);
    return sqrt(est);
}

/* Reference minimiser of eq. (5) (+ z >= 0) by PDHG with diagonal
 * preconditioning on the explicit formulation (Sec. 3.2: K = [A; D],
 * f(s, t) = 1/2 |s - b|^2 + alpha |t|_{2,1}, g = 0 or the indicator of
 * z >= 0; Sec. 3.1 uses this method for its "exact" solutions).
 * Preconditioners (Pock and Chambolle, ICCV 2011, exponent 1):
 *   T_j = 1 / sum_i |K_ij|,  Sigma_i = 1 / sum_j |K_ij|;
 * every row of D has two entries of magnitude 1, so Sigma = 1/2 on the D
 * block (the same for both components of a pixel, so that the prox of
 * f2* stays the pixelwise projection onto the alpha ball). */
void orc_pdhg_explicit(const orc_op* A, const double* b, double alpha,
                       int nonneg, int64_t iters, double* x, double* y1,
                       double* y2, int64_t obj_every, double* obj_trace) {
    int H = A->H, W = A->W;
    size_t n = (size_t)H * W, m = orc_op_out_size(A);
    double* T = dalloc(n);
    double* S1 = dalloc(m);
    double* ones_n = dalloc(n);
    double* ones_m = dalloc(m);
    double* tmp_n = dalloc(n);
    double* tmp_m = dalloc(m);
    double* xn = dalloc(n);
    double* xbar = dalloc(n);
    double* g = dalloc(2 * n);
    for (size_t i = 0; i < n; ++i) ones_n[i] = 1.0;
    for (size_t i = 0; i < m; ++i) ones_m[i] = 1.0;
    /* |A| row and column sums (the Joseph weights are >= 0; for the blur the
     * kernel's absolute sum is every row and column sum). */
    if (A->kind == ORC_BLUR) {
        double ks = 0.0;
        for (int i = 0; i < A->kh * A->kw; ++i) ks += fabs(A->kernel[i]);
        for (size_t i = 0; i < n; ++i) { tmp_n[i] = ks; tmp_m[i] = ks; }
    } else {
        orc_op_adjoint(A, ones_m, tmp_n); /* column sums */
        orc_op_apply(A, ones_n, tmp_m);   /* row sums */
    }
    for (int i = 0; i < H; ++i) {
        for (int j = 0; j < W; ++j) {
            int cnt = (i < H - 1) + (i > 0) + (j < W - 1) + (j > 0);
            double cs = AT(tmp_n, i, j) + cnt;
            AT(T, i, j) = cs > 0 ? 1.0 / cs : 0.0;
        }
    }
    for (size_t i = 0; i < m; ++i) S1[i] = tmp_m[i] > 0 ? 1.0 / tmp_m[i] : 0.0;
    const double S2 = 0.5;
    int64_t rec = 0;
    for (int64_t k = 0; k < iters; ++k) {
        /* K^T y = A^T y1 + D^T y2 = A^T y1 - div y2 */
        orc_op_adjoint(A, y1, tmp_n);
        orc_div(H, W, y2, xn);
        for (size_t i = 0; i < n; ++i) {
            double v = x[i] - T[i] * (tmp_n[i] - xn[i]);
            if (nonneg && !(v > 0.0)) v = 0.0;
            xbar[i] = 2.0 * v - x[i];
            x[i] = v;
        }
        orc_op_apply(A, xbar, tmp_m);
        for (size_t i = 0; i < m; ++i)
            y1[i] = (y1[i] + S1[i] * (tmp_m[i] - b[i])) / (1.0 + S1[i]);
        orc_grad(H, W, xbar, g);
        for (size_t i = 0; i < 2 * n; ++i) g[i] = y2[i] + S2 * g[i];
        orc_proj_ball(n, g, alpha, y2);
        if (obj_every > 0 && obj_trace && (k + 1) % obj_every == 0)
            obj_trace[rec++] = orc_objective(A, b, x, alpha);
    }
    free(T); free(S1); free(ones_n); free(ones_m); free(tmp_n); free(tmp_m);
    free(xn); free(xbar); free(g);
}

/* ------------------------------------------------------------------------
 * The light-prox problems of Sec. 2.1-2.2: the dual of TV denoising
 * (Dual-ROF, and with eps > 0 the Dual-Huber-ROF of Sec. 2.2),
 *   min_{|q_i| <= alpha} F(q) = 1/2 |div q + b|^2 (+ eps / (2 alpha) |q|^2),
 * whose gradient is grad F(q) = -D(div q + b) + (eps / alpha) q and whose
 * nonsmooth part is the indicator of the alpha-ball set C, with prox the
 * projection P_C of eq. (7) (reading: the projection onto the alpha-ball).
 * The primal iterate is u_k = b + div q_k.
 * ------------------------------------------------------------------------ */
static void dual_rof_grad(int H, int W, const double* b, double alpha, double eps,
                          const double* q, double* u, double* g) {
    size_t n = (size_t)H * W;
    orc_div(H, W, q, u);
    for (size_t i = 0; i < n; ++i) u[i] += b[i];
    orc_grad(H, W, u, g);
    double mu = alpha > 0 ? eps / alpha : 0.0;
    for (size_t i = 0; i < 2 * n; ++i) g[i] = -g[i] + mu * q[i];
}

/* ProxSkip (Alg. "ProxSkip") with f = F, psi = indicator of C: the prox of
 * (gamma / p) psi is P_C whatever the scale.  q, h ([2][H][W]) are in/out;
 * err_trace (nullable, K values) gets |u_{k+1} - u_ref| / |u_ref| when u_ref
 * is given.  The prox argument is formed as w + (gamma - gamma / p) h with
 * w = q - gamma grad F(q), so p = 1 reproduces ProjGD bitwise.  Returns the
 * number of projections. */
int64_t orc_dual_rof_proxskip(int H, int W, const double* b, double alpha, double eps,
                              double gamma, double p, int64_t K, uint64_t seed,
                              uint64_t stream, int64_t k0, double* q, double* h,
                              uint8_t* theta_trace, const double* u_ref, double* err_trace) {
    size_t n = (size_t)H * W;
    double* u = dalloc(n);
    double* g = dalloc(2 * n);
    double* qhat = dalloc(2 * n);
    double* v = dalloc(2 * n);
    double coef = gamma - gamma / p, rate = p / gamma;
    double nref = 0.0;
    if (u_ref)
        for (size_t i = 0; i < n; ++i) nref += u_ref[i] * u_ref[i];
    nref = sqrt(nref);
    int64_t nprox = 0;
    for (int64_t kk = 0; kk < K; ++kk) {
        dual_rof_grad(H, W, b, alpha, eps, q, u, g);
        int th = orc_coin(seed, stream, k0 + kk, p);
        for (size_t i = 0; i < 2 * n; ++i) {
            double w = q[i] - gamma * g[i];
            qhat[i] = w + gamma * h[i];
            v[i] = w + coef * h[i];
        }
        if (th) {
            orc_proj_ball(n, v, alpha, q);
            for (size_t i = 0; i < 2 * n; ++i) h[i] = h[i] + rate * (q[i] - qhat[i]);
            ++nprox;
        } else {
            memcpy(q, qhat, 2 * n * sizeof(double));
        }
        if (theta_trace) theta_trace[kk] = (uint8_t)th;
        if (err_trace && u_ref) {
            orc_div(H, W, q, u);
            double e = 0.0;
            for (size_t i = 0; i < n; ++i) {
                double d = b[i] + u[i] - u_ref[i];
                e += d * d;
            }
            err_trace[kk] = sqrt(e) / nref;
        }
    }
    free(u); free(g); free(qhat); free(v);
    return nprox;
}

/* ProjGD (Chambolle's projected gradient, Sec. 2.1), written separately:
 *   q_{k+1} = P_C(q_k + gamma (D(div q_k + b) - (eps / alpha) q_k)). */
void orc_dual_rof_projgd(int H, int W, const double* b, double alpha, double eps, double gamma,
                         int64_t K, double* q) {
    size_t n = (size_t)H * W;
    double* u = dalloc(n);
    double* g = dalloc(2 * n);
    double* t = dalloc(2 * n);
    for (int64_t k = 0; k < K; ++k) {
        dual_rof_grad(H, W, b, alpha, eps, q, u, g);
        for (size_t i = 0; i < 2 * n; ++i) t[i] = q[i] - gamma * g[i];
        orc_proj_ball(n, t, alpha, q);
    }
    free(u); free(g); free(t);
}

/* ------------------------------------------------------------------------
 * Skipping inside the inner solver (the paper's "Discussion and Future
 * work"): the TV prox z = argmin 1/2 |z - v|^2 + lam TV(z) (+ z >= 0) solved
 * by ProxSkip on its dual instead of FGP.  The dual (Sec. 2.1; with z >= 0
 * the constrained dual of Beck and Teboulle 2009) is
 *   min_{|q_i| <= lam} F(q),  grad F(q) = -D P_X(v + div q),
 * P_X = max(., 0) when nonneg, else the identity (then F is the Dual-ROF
 * objective 1/2 |v + div q|^2); its nonsmooth part is the indicator of the
 * lam-ball, whose prox is the projection of eq. (7).  ProxSkip (Alg.
 * "ProxSkip") with step 1/8 (|D|^2 <= 8, the step FGP takes) and
 * projection probability p_in, from the warm (q, h); z = P_X(v + div q).
 * The coin of inner step i is orc_coin(seed, stream, k0 + i, p_in).
 * Returns the number of projections.
 * ------------------------------------------------------------------------ */
int64_t orc_tv_prox_skip(int H, int W, const double* v, double lam, int nonneg, int iters,
                         double p_in, uint64_t seed, uint64_t stream, int64_t k0, double* q,
                         double* h, double* z_out) {
    size_t n = (size_t)H * W;
    const double gamma = 0.125, coef = gamma - gamma / p_in, rate = p_in / gamma;
    double* u = dalloc(n);
    double* g = dalloc(2 * n);
    double* qhat = dalloc(2 * n);
    double* w2 = dalloc(2 * n);
    int64_t nproj = 0;
    for (int it = 0; it < iters; ++it) {
        /* grad F(q) = -D P_X(v + div q) */
        orc_div(H, W, q, u);
        for (size_t i = 0; i < n; ++i) {
            u[i] += v[i];
            if (nonneg && u[i] < 0.0) u[i] = 0.0;
        }
        orc_grad(H, W, u, g);
        int th = orc_coin(seed, stream, k0 + it, p_in);
        for (size_t i = 0; i < 2 * n; ++i) {
            double w = q[i] + gamma * g[i];      /* q - gamma grad F(q) */
            qhat[i] = w + gamma * h[i];
            w2[i] = w + coef * h[i];
        }
        if (th) {
            orc_proj_ball(n, w2, lam, q);
            for (size_t i = 0; i < 2 * n; ++i) h[i] = h[i] + rate * (q[i] - qhat[i]);
            ++nproj;
        } else {
            memcpy(q, qhat, 2 * n * sizeof(double));
        }
    }
    orc_div(H, W, q, u);
    for (size_t i = 0; i < n; ++i) {
        double zi = v[i] + u[i];
        z_out[i] = (nonneg && zi < 0.0) ? 0.0 : zi;
    }
    free(u); free(g); free(qhat); free(w2);
    return nproj;
}

/* The inner coins of the prox call at outer iteration k come from the
 * coin's generator on stream stream_id xor 2^62, indices k K_in + i, so a
 * run resumed at k0 draws the same inner schedule. */
#define ORC_INNER_STREAM 0x4000000000000000ULL

/* Alg. "ProxSkip" with the TV prox by orc_tv_prox_skip (K_in = inner_iters
 * inner ProxSkip steps, projection probability p_in, inner control variate
 * h_in [2][H][W] kept across calls like the dual q).  n_proj_out (nullable)
 * gets the number of inner projections.  Returns the number of prox calls. */
int64_t orc_proxskip_inner(const orc_op* A, const double* b, double* x, double* h, double* q,
                           double* h_in, double p_in, const orc_params* P,
                           uint8_t* theta_trace, double* obj_trace, int64_t* n_proj_out) {
    int H = A->H, W = A->W;
    size_t n = (size_t)H * W, m = orc_op_out_size(A);
    double gamma = P->step, p = P->p;
    double lam = P->alpha * gamma / p;
    double coef = gamma - gamma / p;
    double rate = p / gamma;
    double* res = dalloc(m);
    double* g = dalloc(n);
    double* w = dalloc(n);
    double* xhat = dalloc(n);
    double* v = dalloc(n);
    double* z = dalloc(n);
    int64_t nprox = 0, nproj = 0;
    for (int64_t kk = 0; kk < P->outer_iters; ++kk) {
        int64_t k = P->k0 + kk;
        data_grad(A, b, x, res, g);
        for (size_t i = 0; i < n; ++i) {
            w[i] = x[i] - gamma * g[i];
            xhat[i] = w[i] + gamma * h[i];
        }
        int th = orc_coin(P->seed, P->stream_id, k, p);
        if (th) {
            for (size_t i = 0; i < n; ++i) v[i] = w[i] + coef * h[i];
            nproj += orc_tv_prox_skip(H, W, v, lam, P->nonneg, P->inner_iters, p_in, P->seed,
                                      P->stream_id ^ ORC_INNER_STREAM, k * P->inner_iters, q,
                                      h_in, z);
            for (size_t i = 0; i < n; ++i) {
                h[i] = h[i] + rate * (z[i] - xhat[i]);
                x[i] = z[i];
            }
            ++nprox;
        } else {
            memcpy(x, xhat, n * sizeof(double));
        }
        if (theta_trace) theta_trace[kk] = (uint8_t)th;
        if (obj_trace) obj_trace[kk] = orc_objective(A, b, x, P->alpha);
    }
    if (n_proj_out) *n_proj_out = nproj;
    free(res); free(g); free(w); free(xhat); free(v); free(z);
    return nprox;
}

/* Alg. "PDHGSkip-2" with the TV prox by orc_tv_prox_skip (as above). */
int64_t orc_pdhgskip_inner(const orc_op* A, const double* b, double* x, double* h, double* y,
                           double* q, double* h_in, double p_in, const orc_params* P,
                           uint8_t* theta_trace, double* obj_trace, int64_t* n_proj_out) {
    int H = A->H, W = A->W;
    size_t n = (size_t)H * W, m = orc_op_out_size(A);
    double sigma = P->step, tau = P->dual_step, p = P->p;
    double lam = P->alpha * sigma / p;
    double coef = sigma - sigma / p;
    double rate = p / sigma;
    double* kty = dalloc(n);
    double* w = dalloc(n);
    double* xhat = dalloc(n);
    double* v = dalloc(n);
    double* z = dalloc(n);
    double* xbar = dalloc(n);
    double* kx = dalloc(m);
    int64_t nprox = 0, nproj = 0;
    for (int64_t kk = 0; kk < P->outer_iters; ++kk) {
        int64_t k = P->k0 + kk;
        orc_op_adjoint(A, y, kty);
        for (size_t i = 0; i < n; ++i) {
            w[i] = x[i] - sigma * kty[i];
            xhat[i] = w[i] + sigma * h[i];
        }
        int th = orc_coin(P->seed, P->stream_id, k, p);
        if (th) {
            for (size_t i = 0; i < n; ++i) v[i] = w[i] + coef * h[i];
            nproj += orc_tv_prox_skip(H, W, v, lam, P->nonneg, P->inner_iters, p_in, P->seed,
                                      P->stream_id ^ ORC_INNER_STREAM, k * P->inner_iters, q,
                                      h_in, z);
            for (size_t i = 0; i < n; ++i) h[i] = h[i] + rate * (z[i] - xhat[i]);
            ++nprox;
        } else {
            memcpy(z, xhat, n * sizeof(double));
        }
        for (size_t i = 0; i < n; ++i) {
            xbar[i] = 2.0 * z[i] - x[i];
            x[i] = z[i];
        }
        orc_op_apply(A, xbar, kx);
        for (size_t i = 0; i < m; ++i) y[i] = (y[i] + tau * (kx[i] - b[i])) / (1.0 + tau);
        if (theta_trace) theta_trace[kk] = (uint8_t)th;
        if (obj_trace) obj_trace[kk] = orc_objective(A, b, x, P->alpha);
    }
    if (n_proj_out) *n_proj_out = nproj;
    free(kty); free(w); free(xhat); free(v); free(z); free(xbar); free(kx);
    return nprox;
}
