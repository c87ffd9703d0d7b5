/*
 * cnn.c -- plain CPU FP64 reference of the learned TV prox.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as oracle.c): used by the tests, the
 * smoke check and the benchmark's CPU leg, never by the product library.
 *
 * The paper's prox is an inner iterative solver of eq. (3) with R = TV
 * (Sec. 2.1, Sec. 3.1).  The learned prox replaces the inner solver by a
 * small convolutional network that predicts a dual field; the primal point
 * is then recovered exactly as the dual method recovers it:
 *
 *   input   x0 = (v, lam * 1)                 2 channels, zero outside the image
 *   layer l pre_l[co](p) = b_l[co] + sum_t sum_ci W_l[t][ci][co] x_{l-1}[ci](p + o_t)
 *           o_t = (t / 3 - 1, t % 3 - 1) (row, column offset), t = 0..8
 *           x_l = max(pre_l, 0) for l = 1, 2, 3;  qt = pre_4 (2 channels)
 *   head    q = P_lam(qt)   (the ball projection of eq. (7), strict branch)
 *           z = P_X(v + div q)                 (u = b + div q, Sec. 2.1)
 *   loss    L = sum over the batch of [(z - z_target)^2 + mu |q - q_target|^2]
 *               / (2 * pixels), the dual term optional (q_target = NULL or
 *               mu = 0); it pins the dual where z alone leaves it free (where
 *               D z = 0 any feasible dual with the same divergence fits)
 *
 * Channels 2 -> 32 -> 32 -> 32 -> 2, 3x3 kernels, zero padding.  The dual
 * output makes the duality gap of eq. (6) computable for every prediction,
 * and gives an exact warm start for the inner solver when the gap is too
 * large.  Parameter vector: for l = 1..4, W_l[9][C_in][C_out] then b_l[C_out].
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const int CIN[ORC_CNN_LAYERS] = {2, 32, 32, 32};
static const int COUT[ORC_CNN_LAYERS] = {32, 32, 32, 2};

static double* zalloc(size_t n) {
    double* p = (double*)calloc(n ? n : 1, sizeof(double));
    if (!p) abort();
    return p;
}

size_t orc_cnn_param_count(void) {
    size_t s = 0;
    for (int l = 0; l < ORC_CNN_LAYERS; ++l) s += (size_t)9 * CIN[l] * COUT[l] + COUT[l];
    return s;
}

/* offsets of layer l's weights and biases in the parameter vector */
static size_t w_off(int l) {
    size_t s = 0;
    for (int k = 0; k < l; ++k) s += (size_t)9 * CIN[k] * COUT[k] + COUT[k];
    return s;
}
static size_t b_off(int l) { return w_off(l) + (size_t)9 * CIN[l] * COUT[l]; }

/* 3x3 cross-correlation with zero padding, planar [C][H][W] tensors. */
static void conv_fwd(int H, int W, int cin, int cout, const double* w, const double* b,
                     const double* x, double* y) {
    for (int co = 0; co < cout; ++co)
        for (int i = 0; i < H; ++i)
            for (int j = 0; j < W; ++j) {
                double s = b[co];
                for (int t = 0; t < 9; ++t) {
                    int ii = i + t / 3 - 1, jj = j + t % 3 - 1;
                    if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
                    for (int ci = 0; ci < cin; ++ci)
                        s += w[((size_t)t * cin + ci) * cout + co] *
                             x[((size_t)ci * H + ii) * W + jj];
                }
                y[((size_t)co * H + i) * W + j] = s;
            }
}

/* Adjoint of conv_fwd with respect to its input and its parameters:
 *   gx[ci](p) = sum_t sum_co W[t][ci][co] gy[co](p - o_t)  (p - o_t inside),
 *   gw[t][ci][co] += sum_p x[ci](p + o_t) gy[co](p),  gb[co] += sum_p gy[co](p).
 * gx may be NULL (the first layer needs no input gradient). */
static void conv_bwd(int H, int W, int cin, int cout, const double* w, const double* x,
                     const double* gy, double* gx, double* gw, double* gb) {
    if (gx) {
        for (int ci = 0; ci < cin; ++ci)
            for (int i = 0; i < H; ++i)
                for (int j = 0; j < W; ++j) {
                    double s = 0.0;
                    for (int t = 0; t < 9; ++t) {
                        int ii = i - (t / 3 - 1), jj = j - (t % 3 - 1);
                        if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
                        for (int co = 0; co < cout; ++co)
                            s += w[((size_t)t * cin + ci) * cout + co] *
                                 gy[((size_t)co * H + ii) * W + jj];
                    }
                    gx[((size_t)ci * H + i) * W + j] = s;
                }
    }
    for (int t = 0; t < 9; ++t)
        for (int ci = 0; ci < cin; ++ci)
            for (int co = 0; co < cout; ++co) {
                double s = 0.0;
                for (int i = 0; i < H; ++i)
                    for (int j = 0; j < W; ++j) {
                        int ii = i + t / 3 - 1, jj = j + t % 3 - 1;
                        if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
                        s += x[((size_t)ci * H + ii) * W + jj] * gy[((size_t)co * H + i) * W + j];
                    }
                gw[((size_t)t * cin + ci) * cout + co] += s;
            }
    for (int co = 0; co < cout; ++co) {
        double s = 0.0;
        for (size_t p = 0; p < (size_t)H * W; ++p) s += gy[(size_t)co * H * W + p];
        gb[co] += s;
    }
}

/* Per-image activations of one forward pass. */
typedef struct {
    double* x[ORC_CNN_LAYERS];    /* x[0] = input, x[l] = output of layer l (l = 1..3) */
    double* pre[ORC_CNN_LAYERS];  /* pre-activations of every layer; pre[3] = qt */
    double* q;                    /* P_lam(qt) */
    double* u;                    /* v + div q */
    double* z;
} acts;

static void acts_alloc(acts* a, int H, int W) {
    size_t n = (size_t)H * W;
    for (int l = 0; l < ORC_CNN_LAYERS; ++l) {
        a->x[l] = zalloc((size_t)CIN[l] * n);
        a->pre[l] = zalloc((size_t)COUT[l] * n);
    }
    a->q = zalloc(2 * n);
    a->u = zalloc(n);
    a->z = zalloc(n);
}

static void acts_free(acts* a) {
    for (int l = 0; l < ORC_CNN_LAYERS; ++l) { free(a->x[l]); free(a->pre[l]); }
    free(a->q); free(a->u); free(a->z);
}

static void forward_one(int H, int W, const double* v, double lam, int nonneg,
                        const double* params, acts* a) {
    size_t n = (size_t)H * W;
    for (size_t p = 0; p < n; ++p) { a->x[0][p] = v[p]; a->x[0][n + p] = lam; }
    for (int l = 0; l < ORC_CNN_LAYERS; ++l) {
        conv_fwd(H, W, CIN[l], COUT[l], params + w_off(l), params + b_off(l), a->x[l], a->pre[l]);
        if (l + 1 < ORC_CNN_LAYERS)
            for (size_t p = 0; p < (size_t)COUT[l] * n; ++p)
                a->x[l + 1][p] = a->pre[l][p] > 0.0 ? a->pre[l][p] : 0.0;
    }
    orc_proj_ball(n, a->pre[ORC_CNN_LAYERS - 1], lam, a->q);
    orc_div(H, W, a->q, a->u);
    for (size_t p = 0; p < n; ++p) {
        a->u[p] += v[p];
        a->z[p] = (nonneg && !(a->u[p] > 0.0)) ? 0.0 : a->u[p];
    }
}

void orc_cnn_forward(int nimg, int H, int W, const double* v, const double* lam, int nonneg,
                     const double* params, double* qt_out, double* z_out) {
    size_t n = (size_t)H * W;
    acts a;
    acts_alloc(&a, H, W);
    for (int b = 0; b < nimg; ++b) {
        forward_one(H, W, v + b * n, lam[b], nonneg, params, &a);
        if (qt_out) memcpy(qt_out + 2 * b * n, a.pre[ORC_CNN_LAYERS - 1], 2 * n * sizeof(double));
        if (z_out) memcpy(z_out + b * n, a.z, n * sizeof(double));
    }
    acts_free(&a);
}

/* Loss and its gradient by reverse-mode differentiation of the forward pass
 * above (chain rule through P_X, div, P_lam, the convolutions and ReLU).
 * The derivative of max(u, 0) is taken as [u > 0]; that of P_lam at
 * |qt| > lam is (lam / |qt|)(I - n n^T) with n = qt / |qt|, else I.
 * grad (nullable) is overwritten.  Returns the loss. */
double orc_cnn_loss_grad(int nimg, int H, int W, const double* v, const double* lam,
                         int nonneg, const double* params, const double* z_target,
                         const double* q_target, double mu, double* grad) {
    size_t n = (size_t)H * W;
    double npx = (double)nimg * (double)n;
    size_t np = orc_cnn_param_count();
    if (grad) memset(grad, 0, np * sizeof(double));
    acts a;
    acts_alloc(&a, H, W);
    double* gu = zalloc(n);
    double* gq = zalloc(2 * n);
    double* gpre[ORC_CNN_LAYERS];
    double* gx = zalloc((size_t)32 * n);
    for (int l = 0; l < ORC_CNN_LAYERS; ++l) gpre[l] = zalloc((size_t)COUT[l] * n);
    double loss = 0.0;
    for (int b = 0; b < nimg; ++b) {
        const double* vb = v + b * n;
        const double* zt = z_target + b * n;
        forward_one(H, W, vb, lam[b], nonneg, params, &a);
        for (size_t p = 0; p < n; ++p) {
            double d = a.z[p] - zt[p];
            loss += d * d;
            gu[p] = (nonneg && !(a.u[p] > 0.0)) ? 0.0 : d / npx;
        }
        const double* qtg = q_target ? q_target + 2 * b * n : NULL;
        if (qtg && mu != 0.0)
            for (size_t p = 0; p < 2 * n; ++p) {
                double d = a.q[p] - qtg[p];
                loss += mu * d * d;
            }
        if (!grad) continue;
        /* z = P_X(v + div q):  dL/dq = div^T gu = -D gu, plus the dual term */
        orc_grad(H, W, gu, gq);
        for (size_t p = 0; p < 2 * n; ++p) gq[p] = -gq[p];
        if (qtg && mu != 0.0)
            for (size_t p = 0; p < 2 * n; ++p) gq[p] += mu * (a.q[p] - qtg[p]) / npx;
        /* q = P_lam(qt) */
        double* qt = a.pre[ORC_CNN_LAYERS - 1];
        double* g4 = gpre[ORC_CNN_LAYERS - 1];
        for (size_t p = 0; p < n; ++p) {
            double qy = qt[p], qx = qt[n + p];
            double nrm = sqrt(qy * qy + qx * qx);
            if (nrm > lam[b]) {
                double ny = qy / nrm, nx = qx / nrm, s = lam[b] / nrm;
                double dot = ny * gq[p] + nx * gq[n + p];
                g4[p] = s * (gq[p] - ny * dot);
                g4[n + p] = s * (gq[n + p] - nx * dot);
            } else {
                g4[p] = gq[p];
                g4[n + p] = gq[n + p];
            }
        }
        for (int l = ORC_CNN_LAYERS - 1; l >= 0; --l) {
            conv_bwd(H, W, CIN[l], COUT[l], params + w_off(l), a.x[l], gpre[l],
                     l > 0 ? gx : NULL, grad + w_off(l), grad + b_off(l));
            if (l > 0)  /* x_l = max(pre_{l-1}, 0) */
                for (size_t p = 0; p < (size_t)CIN[l] * n; ++p)
                    gpre[l - 1][p] = a.pre[l - 1][p] > 0.0 ? gx[p] : 0.0;
        }
    }
    for (int l = 0; l < ORC_CNN_LAYERS; ++l) free(gpre[l]);
    free(gx); free(gu); free(gq);
    acts_free(&a);
    return loss / (2.0 * npx);
}

/* One Adam step (Kingma and Ba, 2015) on a parameter vector; `step` is the
 * 1-based step count used in the bias corrections. */
void orc_adam_step(size_t n, double* params, const double* grad, double* m, double* v,
                   int64_t step, double lr, double beta1, double beta2, double eps) {
    double c1 = 1.0 - pow(beta1, (double)step);
    double c2 = 1.0 - pow(beta2, (double)step);
    for (size_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        params[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
