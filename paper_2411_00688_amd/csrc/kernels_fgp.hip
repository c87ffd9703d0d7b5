// FGP (the paper's AProjGD: accelerated projected gradient on the TV dual)
// for gfx950.
//
// One FGP iteration on the dual field q = (q_y, q_x) (two H x W planes):
//   r   = q_{k-1} + beta_k (q_{k-1} - q_{k-2})          FISTA momentum
//   z   = P_X(v + div r)                                 primal point
//   q_k = P_lambda(r + D z / 8)                          projected step, 1/L = 1/8
// with div = -D^T, D forward differences zero in the last row / column, and
// P_lambda the pixelwise projection onto the lambda ball (eq. (7), read as a
// ball of radius lambda).  beta_k = (t_{k-1} - 1) / t_k, t_0 = 1 (Beck and
// Teboulle's sequence; the paper's printed extrapolation is garbled).
//
// Kernel design (temporal blocking): a workgroup owns a BH x BW output tile
// and loads the tile plus a halo of TS pixels of (q_{k-1}, q_{k-2}, v) into
// registers.  Each iteration has radius 1 (z looks one pixel up/left, D z
// one pixel down/right), so after TS iterations computed entirely from LDS
// and registers the central tile is exact; it is written back together with
// the previous iterate (needed for the next momentum step).  HBM traffic per
// launch is one read of (q_{k-1}, q_{k-2}, v) plus the halo and one write of
// two dual fields, instead of TS times that.  Pixels outside the image are
// zero and never feed an in-image pixel: every neighbour access is guarded by
// the image-global boundary conditions.
//
// For images far beyond the caches the strip kernels (fgp_strip: one
// iteration per launch; fgp_strip_tb: TS per launch) instead give each
// workgroup a 256-column strip that it walks down row by row, so loads and
// stores are whole aligned row segments, rows are read once, and
// neighbours come through two LDS rows with one barrier per row.
#include "tvs_internal.hpp"

namespace tvs {

template <typename T>
__device__ __forceinline__ T ball_scale(T wy, T wx, T lam);

// float: hardware reciprocal square root (about 1 ulp).  n2 is clamped away
// from the denormal range, where the instruction flushes to zero: there
// n2 > lam^2 implies lam < 1e-18 and the clamped scale is still <= 1.
template <>
__device__ __forceinline__ float ball_scale<float>(float wy, float wx, float lam) {
    float n2 = wy * wy + wx * wx;
    return (n2 > lam * lam) ? lam * __builtin_amdgcn_rsqf(fmaxf(n2, 1e-37f)) : 1.0f;
}

template <>
__device__ __forceinline__ double ball_scale<double>(double wy, double wx, double lam) {
    double nrm = sqrt(wy * wy + wx * wx);
    return (nrm > lam) ? lam / nrm : 1.0;
}

template <typename T>
struct FgpArgs {
    const T* v;
    const T* qa;   // q_{k-1}
    const T* qb;   // q_{k-2}
    T* oa;         // out: last iterate
    T* ob;         // out: the one before (nullptr when nsteps == 1)
    const T* beta; // beta[k]: momentum coefficient used to form r of iteration k
    int k_start;
    int nsteps;    // <= TS
    T lam;
    int nonneg;
    int H, W;
    size_t plane;  // H * W
    const int* run_flag = nullptr;  // if set and *run_flag == 0 the launch does nothing
};

// bit flags of a pixel's neighbour relations, precomputed once per launch
enum : int {
    F_IN = 1,       // inside the image and the loaded region
    F_DY = 2,       // i < H-1: D_y exists at this pixel
    F_UP = 4,       // i > 0 and the upper neighbour is in the tile
    F_DX = 8,       // j < W-1
    F_LEFT = 16,    // j > 0 and the left neighbour is in the tile
    F_DOWN = 32,    // i < H-1 and the lower neighbour is in the tile
    F_RIGHT = 64,   // j < W-1 and the right neighbour is in the tile
    F_OUT = 128     // in the central tile and inside the image (stored)
};

// One output tile (tile row ty, tile column tx) of one image.  v, qa, qb, oa,
// ob point at the image's data (dual planes [2][H][W] at qa etc.).
template <typename T, int BW, int BH, int TS, int NT>
__device__ __forceinline__ void fgp_tile(const FgpArgs<T>& a, int ty, int tx) {
    constexpr int RW = BW + 2 * TS, RH = BH + 2 * TS, R = RW * RH;
    constexpr int PPT = (R + NT - 1) / NT;
    __shared__ T s_ry[R];
    __shared__ T s_rx[R];
    __shared__ T s_z[R];

    const int H = a.H, W = a.W;
    const int i0 = ty * BH - TS;
    const int j0 = tx * BW - TS;
    const int tid = (int)threadIdx.x;

    T qay[PPT], qax[PPT], qby[PPT], qbx[PPT], vv[PPT], ry[PPT], rx[PPT], zz[PPT];
    int fl[PPT];

#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int idx = tid + p * NT;
        const int li = idx / RW, lj = idx - (idx / RW) * RW;
        const int i = i0 + li, j = j0 + lj;
        const bool inr = idx < R;
        const bool in = inr && i >= 0 && i < H && j >= 0 && j < W;
        int f = 0;
        if (in) {
            f |= F_IN;
            if (i < H - 1) f |= F_DY;
            if (i > 0 && li > 0) f |= F_UP;
            if (j < W - 1) f |= F_DX;
            if (j > 0 && lj > 0) f |= F_LEFT;
            if (i < H - 1 && li < RH - 1) f |= F_DOWN;
            if (j < W - 1 && lj < RW - 1) f |= F_RIGHT;
            if (li >= TS && li < TS + BH && lj >= TS && lj < TS + BW) f |= F_OUT;
        }
        fl[p] = f;
        const size_t g = in ? (size_t)i * W + j : 0;
        qay[p] = in ? a.qa[g] : T(0);
        qax[p] = in ? a.qa[a.plane + g] : T(0);
        qby[p] = in ? a.qb[g] : T(0);
        qbx[p] = in ? a.qb[a.plane + g] : T(0);
        vv[p] = in ? a.v[g] : T(0);
    }

    const T lam = a.lam;
    const T eighth = T(0.125);
    for (int s = 0; s < a.nsteps; ++s) {
        const T beta = a.beta[a.k_start + s];
        // r = q_{k-1} + beta (q_{k-1} - q_{k-2})
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int idx = tid + p * NT;
            ry[p] = qay[p] + beta * (qay[p] - qby[p]);
            rx[p] = qax[p] + beta * (qax[p] - qbx[p]);
            if (idx < R) {
                s_ry[idx] = ry[p];
                s_rx[idx] = rx[p];
            }
        }
        __syncthreads();
        // z = P_X(v + div r)
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int idx = tid + p * NT;
            const int f = fl[p];
            T d = T(0);
            if (f & F_DY) d += ry[p];
            if (f & F_UP) d -= s_ry[idx - RW];
            if (f & F_DX) d += rx[p];
            if (f & F_LEFT) d -= s_rx[idx - 1];
            T z = vv[p] + d;
            if (a.nonneg) z = (z > T(0)) ? z : T(0);
            zz[p] = z;
            if (idx < R) s_z[idx] = z;
        }
        __syncthreads();
        // q_k = P_lambda(r + D z / 8)
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int idx = tid + p * NT;
            const int f = fl[p];
            const T gy = (f & F_DOWN) ? s_z[idx + RW] - zz[p] : T(0);
            const T gx = (f & F_RIGHT) ? s_z[idx + 1] - zz[p] : T(0);
            const T wy = ry[p] + eighth * gy;
            const T wx = rx[p] + eighth * gx;
            const T sc = ball_scale<T>(wy, wx, lam);
            qby[p] = qay[p];
            qbx[p] = qax[p];
            qay[p] = (f & F_IN) ? wy * sc : T(0);
            qax[p] = (f & F_IN) ? wx * sc : T(0);
        }
        // No barrier here: the next step's first LDS writes (s_ry, s_rx) do not
        // touch s_z, and its writes of s_z come after its first barrier.
    }

#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        if (fl[p] & F_OUT) {
            const int idx = tid + p * NT;
            const int li = idx / RW, lj = idx - (idx / RW) * RW;
            const size_t g = (size_t)(i0 + li) * W + (j0 + lj);
            a.oa[g] = qay[p];
            a.oa[a.plane + g] = qax[p];
            if (a.ob) {
                a.ob[g] = qby[p];
                a.ob[a.plane + g] = qbx[p];
            }
        }
    }
}

// One FGP iteration (nsteps == 1) on a strip of 256 columns and RC rows,
// walked down row by row: thread t owns column j0 + t, so every load and
// store is one aligned, contiguous row segment and rows are read once (no
// halo rows; the strip's side halo is one column each way, loaded by the
// edge threads).  Step i forms r at row i and z at row i (its up term is
// r_y of row i-1, kept in a register; its left term r_x of the left
// neighbour, through LDS) and then finishes q at row i-1, which needs z at
// rows i-1 and i and at the right neighbour of row i-1 (from the previous
// step's LDS row).  Double-buffered LDS rows leave one barrier per row.  The
// operands of the next row are in flight while a row is computed.  The
// per-pixel arithmetic and its order are those of fgp_tile, so results are
// bitwise identical.
template <typename T, int RC>
__device__ __forceinline__ void fgp_strip(const FgpArgs<T>& a, int ty, int tx) {
    constexpr int SW = 256;
    __shared__ T s_rx[2][SW + 1];  // [0]: left halo column, [t + 1]: thread t
    __shared__ T s_z[2][SW + 1];   // [t]: thread t, [SW]: right halo column
    const int H = a.H, W = a.W;
    const int tid = (int)threadIdx.x;
    const int j0 = tx * SW, j = j0 + tid, jr = j0 + SW;
    const int ib = ty * RC;
    const int ie = (ib + RC < H) ? ib + RC : H;  // output rows [ib, ie)
    const bool col = j < W;
    const bool hl = tid == 0 && j0 > 0;        // loads r_x of column j0 - 1
    const bool hr = tid == SW - 1 && jr < W;   // loads column jr
    const T* qay = a.qa;
    const T* qax = a.qa + a.plane;
    const T* qby = a.qb;
    const T* qbx = a.qb + a.plane;
    const T beta = a.beta[a.k_start];
    const T lam = a.lam;
    const T eighth = T(0.125);
    auto rf = [&](T qa_, T qb_) { return qa_ + beta * (qa_ - qb_); };

    // r_y of row ib - 1 (the up term of z at row ib)
    T ry_up = T(0), ryh_up = T(0);
    if (ib > 0) {
        const size_t g = (size_t)(ib - 1) * W;
        if (col) ry_up = rf(qay[g + j], qby[g + j]);
        if (hr) ryh_up = rf(qay[g + jr], qby[g + jr]);
    }
    // operands of a row: own column, right halo column (h*), left halo (l*)
    struct Row {
        T ay, ax, by, bx, v, hay, hax, hby, hbx, hv, lax, lbx;
    };
    auto load_row = [&](int i) {
        Row r{};
        if (i >= H) return r;
        const size_t g = (size_t)i * W;
        if (col) {
            r.ay = qay[g + j];
            r.ax = qax[g + j];
            r.by = qby[g + j];
            r.bx = qbx[g + j];
            r.v = a.v[g + j];
        }
        if (hr) {
            r.hay = qay[g + jr];
            r.hax = qax[g + jr];
            r.hby = qby[g + jr];
            r.hbx = qbx[g + jr];
            r.hv = a.v[g + jr];
        }
        if (hl) {
            r.lax = qax[g + j0 - 1];
            r.lbx = qbx[g + j0 - 1];
        }
        return r;
    };
    Row nx = load_row(ib);  // row i + 1 is in flight while row i is computed
    T ry_p = T(0), rx_p = T(0), z_p = T(0);  // row i - 1
    for (int i = ib; i <= ie; ++i) {
        const int b = (i - ib) & 1;
        const bool row = i < H;
        const Row c = nx;
        if (i < ie) nx = load_row(i + 1);
        const T ay = c.ay, ax = c.ax, by = c.by, bx = c.bx, vv = c.v;
        const T hay = c.hay, hax = c.hax, hby = c.hby, hbx = c.hbx, hv = c.hv;
        const T lax = c.lax, lbx = c.lbx;
        const bool in = row && col;
        const T ry = in ? rf(ay, by) : T(0);
        const T rx = in ? rf(ax, bx) : T(0);
        const bool hin = row && hr;
        const T ryh = hin ? rf(hay, hby) : T(0);
        const T rxh = hin ? rf(hax, hbx) : T(0);
        s_rx[b][tid + 1] = rx;
        if (tid == 0) s_rx[b][0] = (row && hl) ? rf(lax, lbx) : T(0);
        __syncthreads();
        // z = P_X(v + div r) at row i
        T z = T(0);
        if (in) {
            T d = T(0);
            if (i < H - 1) d += ry;
            if (i > 0) d -= ry_up;
            if (j < W - 1) d += rx;
            if (j > 0) d -= s_rx[b][tid];
            z = vv + d;
            if (a.nonneg) z = (z > T(0)) ? z : T(0);
        }
        s_z[b][tid] = z;
        if (tid == SW - 1) {
            T zh = T(0);
            if (hin) {
                T d = T(0);
                if (i < H - 1) d += ryh;
                if (i > 0) d -= ryh_up;
                if (jr < W - 1) d += rxh;
                d -= rx;  // jr > 0: the left neighbour is this thread's column
                zh = hv + d;
                if (a.nonneg) zh = (zh > T(0)) ? zh : T(0);
            }
            s_z[b][SW] = zh;
        }
        // q = P_lambda(r + D z / 8) at row i - 1
        if (i > ib && col) {
            const int o = i - 1;
            const T gy = (o < H - 1) ? z - z_p : T(0);
            const T gx = (j < W - 1) ? s_z[b ^ 1][tid + 1] - z_p : T(0);
            const T wy = ry_p + eighth * gy;
            const T wx = rx_p + eighth * gx;
            const T sc = ball_scale<T>(wy, wx, lam);
            const size_t g = (size_t)o * W + j;
            a.oa[g] = wy * sc;
            a.oa[a.plane + g] = wx * sc;
        }
        ry_up = ry;
        ryh_up = ryh;
        ry_p = ry;
        rx_p = rx;
        z_p = z;
    }
}

// TS iterations per launch on a strip of 256 columns walked down its rows
// (TS >= 2): a pipeline of TS row-walking stages, stage s computing
// iteration k + s - 1 and running two rows behind stage s - 1, whose output
// row of the previous step it consumes, so all stages share one barrier
// per row.  Momentum needs q_{k+s-3}: stage s - 2's output three steps
// earlier (register histories).  Every stage loses one valid column on each
// side, so strips overlap: a strip loads 256 columns and stores the middle
// 256 - 2 TS; a block stores RC rows and reads RC + 2 TS.  A stage skips
// (uniformly) the rows its successors do not need.  Per-pixel arithmetic
// and order are those of fgp_tile: bitwise identical results.
template <typename T, int RC, int TS>
__device__ __forceinline__ void fgp_strip_tb(const FgpArgs<T>& a, int ty, int tx) {
    constexpr int SW = 256, OW = SW - 2 * TS, NV = 2 * TS - 1;
    __shared__ T s_rx[TS][2][SW + 1];  // [t + 1]: thread t, [0]: zero
    __shared__ T s_z[TS][2][SW + 1];   // [t]: thread t, [SW]: zero
    const int H = a.H, W = a.W;
    const int tid = (int)threadIdx.x;
    const int j = tx * OW - TS + tid;
    const int ib = ty * RC;
    const int ie = (ib + RC < H) ? ib + RC : H;  // stored rows [ib, ie)
    const int i0 = ib - TS;                       // first row read
    const int ns = a.nsteps;
    const bool col = j >= 0 && j < W;
    const bool ocol = col && tid >= TS && tid < SW - TS;
    const T* qay = a.qa;
    const T* qax = a.qa + a.plane;
    const T* qby = a.qb;
    const T* qbx = a.qb + a.plane;
    const T lam = a.lam;
    const T eighth = T(0.125);
    if (tid < TS * 2) {
        s_rx[tid >> 1][tid & 1][0] = T(0);
        s_z[tid >> 1][tid & 1][SW] = T(0);
    }
    T beta[TS];
#pragma unroll
    for (int s = 0; s < TS; ++s) beta[s] = (s < ns) ? a.beta[a.k_start + s] : T(0);
    // Ey/Ex[s][d]: stage s's output row of d + 1 steps ago (s = 0: the q_{k-1}
    // row read then); qb1: the q_{k-2} row read one step ago; V[d]: v of d + 1
    // steps ago; per stage: r_y of its previous row, that row's r and z.
    T Ey[TS][3], Ex[TS][3], V[NV];
    T ryup[TS], ryp[TS], rxp[TS], zp[TS];
#pragma unroll
    for (int s = 0; s < TS; ++s) {
#pragma unroll
        for (int d = 0; d < 3; ++d) Ey[s][d] = Ex[s][d] = T(0);
        ryup[s] = ryp[s] = rxp[s] = zp[s] = T(0);
    }
#pragma unroll
    for (int d = 0; d < NV; ++d) V[d] = T(0);
    T qby1 = T(0), qbx1 = T(0);
    const int nsteps = (ie - ib) + 3 * TS;
    for (int t = 0; t < nsteps; ++t) {
        const int b = t & 1;
        // the row read in this step is consumed in the next
        T ly = T(0), lx = T(0), lby = T(0), lbx = T(0), lv = T(0);
        const int li = i0 + t;
        if (col && li >= 0 && li < H && li < ie + TS) {
            const size_t g = (size_t)li * W + j;
            ly = qay[g];
            lx = qax[g];
            lby = qby[g];
            lbx = qbx[g];
            lv = a.v[g];
        }
        T ry[TS], rx[TS];
#pragma unroll
        for (int s = 0; s < TS; ++s) {
            const int m = i0 + t - 2 * s - 1;  // row of stage s + 1
            const bool act = s < ns && m >= ib - TS + s && m < ie + TS - s;
            const bool in = act && col && m >= 0 && m < H;
            const T Ay = Ey[s][0], Ax = Ex[s][0];
            const T By = (s == 0) ? qby1 : Ey[s - 1][2];
            const T Bx = (s == 0) ? qbx1 : Ex[s - 1][2];
            ry[s] = in ? Ay + beta[s] * (Ay - By) : T(0);
            rx[s] = in ? Ax + beta[s] * (Ax - Bx) : T(0);
            if (act) s_rx[s][b][tid + 1] = rx[s];
        }
        __syncthreads();
        T ey[TS], ex[TS];
#pragma unroll
        for (int s = 0; s < TS; ++s) {
            ey[s] = ex[s] = T(0);
            const int m = i0 + t - 2 * s - 1;
            const bool act = s < ns && m >= ib - TS + s && m < ie + TS - s;
            if (!act) continue;
            // z = P_X(v + div r) at row m
            T z = T(0);
            if (col && m >= 0 && m < H) {
                T d = T(0);
                if (m < H - 1) d += ry[s];
                if (m > 0) d -= ryup[s];
                if (j < W - 1) d += rx[s];
                if (j > 0) d -= s_rx[s][b][tid];
                z = V[2 * s] + d;
                if (a.nonneg) z = (z > T(0)) ? z : T(0);
            }
            s_z[s][b][tid] = z;
            // q = P_lambda(r + D z / 8) at row m - 1
            const int o = m - 1;
            if (col && o >= 0 && o < H) {
                const T gy = (o < H - 1) ? z - zp[s] : T(0);
                const T gx = (j < W - 1) ? s_z[s][b ^ 1][tid + 1] - zp[s] : T(0);
                const T wy = ryp[s] + eighth * gy;
                const T wx = rxp[s] + eighth * gx;
                const T sc = ball_scale<T>(wy, wx, lam);
                ey[s] = wy * sc;
                ex[s] = wx * sc;
                if (ocol && o >= ib && o < ie) {
                    const size_t g = (size_t)o * W + j;
                    if (s + 1 == ns) {
                        a.oa[g] = ey[s];
                        a.oa[a.plane + g] = ex[s];
                    } else if (s + 2 == ns && a.ob) {
                        a.ob[g] = ey[s];
                        a.ob[a.plane + g] = ex[s];
                    }
                }
            }
            ryup[s] = ry[s];
            ryp[s] = ry[s];
            rxp[s] = rx[s];
            zp[s] = z;
        }
        // histories
#pragma unroll
        for (int s = 0; s < TS; ++s) {
            Ey[s][2] = Ey[s][1];
            Ex[s][2] = Ex[s][1];
            Ey[s][1] = Ey[s][0];
            Ex[s][1] = Ex[s][0];
        }
        Ey[0][0] = ly;
        Ex[0][0] = lx;
#pragma unroll
        for (int s = 1; s < TS; ++s) {
            Ey[s][0] = ey[s - 1];
            Ex[s][0] = ex[s - 1];
        }
        qby1 = lby;
        qbx1 = lbx;
#pragma unroll
        for (int d = NV - 1; d > 0; --d) V[d] = V[d - 1];
        V[0] = lv;
    }
}

// Threads per tile workgroup: 1024 when 256 threads would each hold eight or
// more region pixels, else 256.  At 512^2 (256 tiles of 32 x 32) the deep
// 32 x 32 tiles, whose halo recomputation is 2.25x instead of 4x for
// 16 x 16, then run 16 waves per CU instead of 4 and fill the chip; the
// shallow ones keep 256 threads, which are faster at HBM-bound sizes (more
// loads in flight per thread).
template <int BW, int BH, int TS>
struct FgpTileThreads {
    static constexpr int value =
        (((BW + 2 * TS) * (BH + 2 * TS) + 255) / 256 >= 8) ? 1024 : 256;
};

template <typename T, int BW, int BH, int TS>
__global__ __launch_bounds__((FgpTileThreads<BW, BH, TS>::value)) void fgp_tb_kernel(FgpArgs<T> a) {
    if (a.run_flag && *a.run_flag == 0) return;  // uniform across the grid
    const int gx = div_up(a.W, BW);
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    fgp_tile<T, BW, BH, TS, FgpTileThreads<BW, BH, TS>::value>(a, t / gx, t % gx);
}

template <typename T, int RC>
__global__ __launch_bounds__(256) void fgp_strip_kernel(FgpArgs<T> a) {
    if (a.run_flag && *a.run_flag == 0) return;  // uniform across the grid
    const int gx = div_up(a.W, 256);
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    fgp_strip<T, RC>(a, t / gx, t % gx);
}

template <typename T, int RC, int TS>
__global__ __launch_bounds__(256) void fgp_strip_tb_kernel(FgpArgs<T> a) {
    if (a.run_flag && *a.run_flag == 0) return;  // uniform across the grid
    const int gx = div_up(a.W, 256 - 2 * TS);
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    fgp_strip_tb<T, RC, TS>(a, t / gx, t % gx);
}

// Batched form: block b of the launch works on tile (b - prefix[i]) of slice
// act[i], where prefix holds the cumulative tile counts of the active
// slices (binary search).  Each slice has its own size, offset and lambda.
template <typename T>
struct FgpBatchArgs {
    FgpArgs<T> pools;     // v, qa, qb, oa, ob of the pools; beta, k_start, nsteps, nonneg
    const BSlice<T>* sl;
    const int* act;
    const int* prefix;
    int n_act;
};

__device__ __forceinline__ int find_item(const int* prefix, int n, int b) {
    int lo = 0, hi = n;  // prefix[lo] <= b < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// The slice and tile (ty, tx) of block b of a batched launch with tiles
// BW wide; returns the slice's arguments.
template <typename T, int BW>
__device__ __forceinline__ FgpArgs<T> batched_tile(const FgpBatchArgs<T>& a, int b, int& ty,
                                                   int& tx) {
    const int i = find_item(a.prefix, a.n_act, b);
    const BSlice<T> sl = a.sl[a.act[i]];
    const int t = b - a.prefix[i];
    const int tiles_x = div_up(sl.W, BW);
    FgpArgs<T> f = a.pools;
    const size_t off = (size_t)sl.off;
    f.v = a.pools.v + off;
    f.qa = a.pools.qa + 2 * off;
    f.qb = a.pools.qb + 2 * off;
    f.oa = a.pools.oa + 2 * off;
    f.ob = a.pools.ob ? a.pools.ob + 2 * off : nullptr;
    f.lam = sl.lam;
    f.H = sl.H;
    f.W = sl.W;
    f.plane = (size_t)sl.H * sl.W;
    ty = t / tiles_x;
    tx = t % tiles_x;
    return f;
}

template <typename T, int BW, int BH, int TS>
__global__ __launch_bounds__((FgpTileThreads<BW, BH, TS>::value)) void fgp_tb_batched_kernel(
    FgpBatchArgs<T> a) {
    const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);  // one block per tile
    int ty, tx;
    const FgpArgs<T> f = batched_tile<T, BW>(a, b, ty, tx);
    fgp_tile<T, BW, BH, TS, FgpTileThreads<BW, BH, TS>::value>(f, ty, tx);
}

template <typename T, int RC>
__global__ __launch_bounds__(256) void fgp_strip_batched_kernel(FgpBatchArgs<T> a) {
    const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    int ty, tx;
    const FgpArgs<T> f = batched_tile<T, 256>(a, b, ty, tx);
    fgp_strip<T, RC>(f, ty, tx);
}

template <typename T, int RC, int TS>
__global__ __launch_bounds__(256) void fgp_strip_tb_batched_kernel(FgpBatchArgs<T> a) {
    const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    int ty, tx;
    const FgpArgs<T> f = batched_tile<T, 256 - 2 * TS>(a, b, ty, tx);
    fgp_strip_tb<T, RC, TS>(f, ty, tx);
}

// ----------------------------------------------------------------- configs
// Tile shapes compiled in; the autotuner (or the default) picks one by index.
struct FgpVariant {
    int bw, bh, ts;
    int strip = 0;  // 1: row-walking strips, bw stored columns (256 - 2 ts), bh rows per block
};
static const FgpVariant kFgpVariants[] = {
    {32, 32, 1}, {32, 32, 2}, {32, 32, 4}, {32, 32, 8},
    {64, 16, 1}, {64, 16, 4}, {64, 32, 4}, {16, 16, 4}, {64, 32, 8},
    // small images (latency-bound: fewer launches per prox call; a depth
    // that divides the iteration count saves a short last launch)
    {16, 16, 8}, {32, 16, 4}, {32, 16, 8}, {16, 16, 2}, {16, 16, 5},
    // row-walking strips (HBM-bound sizes): one iteration per launch, or four
    {256, 8, 1, 1}, {248, 32, 4, 1}, {248, 64, 4, 1},
    // 1024-thread tiles at other depths (5 and 10 divide 50)
    {32, 32, 5}, {32, 32, 6}, {64, 16, 8},
};

template <typename T>
static void launch_fgp_variant(int vi, const FgpArgs<T>& a, hipStream_t st) {
    const FgpVariant& V = kFgpVariants[vi];
    dim3 grid(div_up(a.W, V.bw) * div_up(a.H, V.bh));
#define TVS_FGPV(BW_, BH_, TS_)                                                            \
    if (!V.strip && V.bw == BW_ && V.bh == BH_ && V.ts == TS_) {                                    \
        hipLaunchKernelGGL((fgp_tb_kernel<T, BW_, BH_, TS_>), grid,                       \
                           dim3(FgpTileThreads<BW_, BH_, TS_>::value), 0, st, a);               \
        return;                                                                            \
    }
    TVS_FGPV(32, 32, 1) TVS_FGPV(32, 32, 2) TVS_FGPV(32, 32, 4) TVS_FGPV(32, 32, 8)
    TVS_FGPV(64, 16, 1) TVS_FGPV(64, 16, 4) TVS_FGPV(64, 32, 4) TVS_FGPV(16, 16, 4)
    TVS_FGPV(16, 16, 8) TVS_FGPV(32, 16, 4) TVS_FGPV(32, 16, 8) TVS_FGPV(16, 16, 2)
    TVS_FGPV(16, 16, 5) TVS_FGPV(32, 32, 5) TVS_FGPV(32, 32, 6) TVS_FGPV(64, 16, 8)
    if (sizeof(T) == 4) { TVS_FGPV(64, 32, 8) }
#undef TVS_FGPV
    const dim3 sgrid(div_up(a.W, 256) * div_up(a.H, V.bh));
#define TVS_FGPS(RC_)                                                                  \
    if (V.strip && V.ts == 1 && V.bh == RC_) {                                         \
        hipLaunchKernelGGL((fgp_strip_kernel<T, RC_>), sgrid, dim3(256), 0, st, a); \
        return;                                                                        \
    }
    TVS_FGPS(8)
#undef TVS_FGPS
#define TVS_FGPT(RC_, TS_)                                                                   \
    if (V.strip && V.bh == RC_ && V.ts == TS_) {                                             \
        const dim3 tgrid(div_up(a.W, 256 - 2 * TS_) * div_up(a.H, RC_));                    \
        hipLaunchKernelGGL((fgp_strip_tb_kernel<T, RC_, TS_>), tgrid, dim3(256), 0, st, a); \
        return;                                                                              \
    }
    TVS_FGPT(32, 4) TVS_FGPT(64, 4)
#undef TVS_FGPT
    throw Error{TVS_ERR_UNSUPPORTED, "FGP tile variant not compiled for this dtype"};
}

int fgp_variant_count() { return (int)(sizeof(kFgpVariants) / sizeof(kFgpVariants[0])); }

FgpConfig fgp_variant(int index) {
    FgpConfig c;
    c.tile_w = kFgpVariants[index].bw;
    c.tile_h = kFgpVariants[index].bh;
    c.steps = kFgpVariants[index].ts;
    return c;
}

int find_variant_index(const FgpConfig& c, int dtype_bytes) {
    for (int i = 0; i < fgp_variant_count(); ++i) {
        const FgpVariant& V = kFgpVariants[i];
        if (V.bw == c.tile_w && V.bh == c.tile_h && V.ts == c.steps) {
            if (dtype_bytes == 8 && V.bw == 64 && V.bh == 32 && V.ts == 8) return -1;
            return i;
        }
    }
    return -1;
}

static int find_variant(const FgpConfig& c, int dtype_bytes) {
    const int i = find_variant_index(c, dtype_bytes);
    if (i < 0) throw Error{TVS_ERR_UNSUPPORTED, "FGP tile configuration not compiled"};
    return i;
}

// Runs `iters` FGP iterations; returns the buffer holding the final dual
// (q_inout itself or a scratch buffer).  q_inout is only read.
template <typename T>
T* run_fgp(tvs_ctx* ctx, int H, int W, const T* v, double lambda, int iters, int nonneg,
           T* q_inout, const FgpConfig& cfg, const int* run_flag) {
    const size_t plane = (size_t)H * W;
    T* work[3] = {(T*)scratch(ctx, S_Q1, 2 * plane * sizeof(T)),
                  (T*)scratch(ctx, S_Q2, 2 * plane * sizeof(T)),
                  (T*)scratch(ctx, S_Q3, 2 * plane * sizeof(T))};
    const T* beta = beta_table_dev<T>(ctx, iters + 1);
    return run_fgp_bufs<T>(ctx, H, W, v, lambda, iters, nonneg, q_inout, work, beta, cfg, run_flag);
}

// The FGP launch sequence on caller-given work buffers (three dual fields of
// 2 H W elements) and momentum table (iters + 1 entries).
template <typename T>
T* run_fgp_bufs(tvs_ctx* ctx, int H, int W, const T* v, double lambda, int iters, int nonneg,
                T* q_inout, T* const* work, const T* beta, const FgpConfig& cfg,
                const int* run_flag) {
    const size_t plane = (size_t)H * W;
    const int vi = find_variant(cfg, (int)sizeof(T));
    const int TS = kFgpVariants[vi].ts;
    T* bufs[4] = {q_inout, work[0], work[1], work[2]};
    T* qa = q_inout;
    T* qb = q_inout;  // iteration 0 forms r = q_warm whatever beta is
    int k = 0;
    while (k < iters) {
        const int ns = (iters - k) < TS ? (iters - k) : TS;
        T* outs[2];
        int n = 0;
        for (int b = 0; b < 4 && n < 2; ++b)
            if (bufs[b] != qa && bufs[b] != qb) outs[n++] = bufs[b];
        FgpArgs<T> a;
        a.v = v;
        a.qa = qa;
        a.qb = qb;
        a.oa = outs[0];
        a.ob = ns > 1 ? outs[1] : nullptr;
        a.beta = beta;
        a.k_start = k;
        a.nsteps = ns;
        a.lam = (T)lambda;
        a.nonneg = nonneg;
        a.H = H;
        a.W = W;
        a.plane = plane;
        a.run_flag = run_flag;
        launch_fgp_variant<T>(vi, a, ctx->stream);
        TVS_LAUNCH_CHECK();
        if (ns > 1) {
            qb = outs[1];
        } else {
            qb = qa;
        }
        qa = outs[0];
        k += ns;
    }
    return qa;
}

template <typename T>
static void launch_fgp_batched_variant(int vi, const FgpBatchArgs<T>& a, int blocks, hipStream_t st) {
    const FgpVariant& V = kFgpVariants[vi];
#define TVS_FGPB(BW_, BH_, TS_)                                                                  \
    if (!V.strip && V.bw == BW_ && V.bh == BH_ && V.ts == TS_) {                                          \
        hipLaunchKernelGGL((fgp_tb_batched_kernel<T, BW_, BH_, TS_>), dim3(blocks),              \
                           dim3(FgpTileThreads<BW_, BH_, TS_>::value), 0, st, a);                     \
        return;                                                                                  \
    }
    TVS_FGPB(32, 32, 1) TVS_FGPB(32, 32, 2) TVS_FGPB(32, 32, 4) TVS_FGPB(32, 32, 8)
    TVS_FGPB(64, 16, 1) TVS_FGPB(64, 16, 4) TVS_FGPB(64, 32, 4) TVS_FGPB(16, 16, 4)
    TVS_FGPB(16, 16, 8) TVS_FGPB(32, 16, 4) TVS_FGPB(32, 16, 8) TVS_FGPB(16, 16, 2)
    TVS_FGPB(16, 16, 5) TVS_FGPB(32, 32, 5) TVS_FGPB(32, 32, 6) TVS_FGPB(64, 16, 8)
    if (sizeof(T) == 4) { TVS_FGPB(64, 32, 8) }
#undef TVS_FGPB
#define TVS_FGPS(RC_)                                                                            \
    if (V.strip && V.ts == 1 && V.bh == RC_) {                                                   \
        hipLaunchKernelGGL((fgp_strip_batched_kernel<T, RC_>), dim3(blocks), dim3(256), 0, st, a); \
        return;                                                                                  \
    }
    TVS_FGPS(8)
#undef TVS_FGPS
#define TVS_FGPT(RC_, TS_)                                                                   \
    if (V.strip && V.bh == RC_ && V.ts == TS_) {                                             \
        hipLaunchKernelGGL((fgp_strip_tb_batched_kernel<T, RC_, TS_>), dim3(blocks), dim3(256), \
                           0, st, a);                                                        \
        return;                                                                              \
    }
    TVS_FGPT(32, 4) TVS_FGPT(64, 4)
#undef TVS_FGPT
    throw Error{TVS_ERR_UNSUPPORTED, "FGP tile variant not compiled for this dtype"};
}

// FGP on every active slice of one batched iteration, with the same buffer
// rotation as run_fgp; returns the pool holding the final duals.
template <typename T>
T* run_fgp_batched(tvs_ctx* ctx, const BSlice<T>* sl, const BatchLists& L, const T* v_pool,
                   T* q_pool, size_t total_px, int iters, int nonneg, const FgpConfig& cfg) {
    const int vi = find_variant(cfg, (int)sizeof(T));
    const int TS = kFgpVariants[vi].ts;
    T* bufs[4] = {q_pool, (T*)scratch(ctx, S_Q1, 2 * total_px * sizeof(T)),
                  (T*)scratch(ctx, S_Q2, 2 * total_px * sizeof(T)),
                  (T*)scratch(ctx, S_Q3, 2 * total_px * sizeof(T))};
    const T* beta = beta_table_dev<T>(ctx, iters + 1);
    T* qa = q_pool;
    T* qb = q_pool;
    int k = 0;
    while (k < iters) {
        const int ns = (iters - k) < TS ? (iters - k) : TS;
        T* outs[2];
        int n = 0;
        for (int b = 0; b < 4 && n < 2; ++b)
            if (bufs[b] != qa && bufs[b] != qb) outs[n++] = bufs[b];
        FgpBatchArgs<T> a;
        a.pools.v = v_pool;
        a.pools.qa = qa;
        a.pools.qb = qb;
        a.pools.oa = outs[0];
        a.pools.ob = ns > 1 ? outs[1] : nullptr;
        a.pools.beta = beta;
        a.pools.k_start = k;
        a.pools.nsteps = ns;
        a.pools.lam = T(0);
        a.pools.nonneg = nonneg;
        a.pools.H = a.pools.W = 0;
        a.pools.plane = 0;
        a.sl = sl;
        a.act = L.act;
        a.prefix = L.pref_fgp;
        a.n_act = L.n_act;
        launch_fgp_batched_variant<T>(vi, a, L.tiles_fgp, ctx->stream);
        TVS_LAUNCH_CHECK();
        qb = ns > 1 ? outs[1] : qa;
        qa = outs[0];
        k += ns;
    }
    return qa;
}

// -------------------------------------------------------------- finalize
// z = P_X(v + div q) and the bookkeeping that follows a prox evaluation.
// 32 x 32 tiles, 256 threads (4 pixels each); the transposed copy of xbar
// goes through LDS so that both stores are coalesced.
// finalize: one 32 x 32 tile per workgroup, one pixel per thread
constexpr int FIN_NT = 1024, FIN_PPT = 1024 / FIN_NT;

template <typename T>
__global__ __launch_bounds__(FIN_NT) void finalize_kernel(Finalize<T> f, int H, int W) {
    constexpr int TW = 32, TH = 32;
    __shared__ T s_t[TH][TW + 1];
    const size_t plane = (size_t)H * W;
    const int i0 = (int)blockIdx.y * TH, j0 = (int)blockIdx.x * TW;
    const T* qy = f.q;
    const T* qx = f.q + plane;
    // every load of the thread's pixels first, then the arithmetic and the
    // stores (loads after a store would wait for possible aliasing)
    T qc_y[FIN_PPT], qc_x[FIN_PPT], qu[FIN_PPT], ql[FIN_PPT], vv[FIN_PPT], xh[FIN_PPT],
        hh[FIN_PPT], xo[FIN_PPT];
#pragma unroll
    for (int p = 0; p < FIN_PPT; ++p) {
        const int idx = (int)threadIdx.x + p * FIN_NT;
        const int li = idx / TW, lj = idx % TW;
        const int i = i0 + li, j = j0 + lj;
        const bool ok = i < H && j < W;
        const size_t g = ok ? (size_t)i * W + j : 0;
        qc_y[p] = ok ? qy[g] : T(0);
        qc_x[p] = ok ? qx[g] : T(0);
        qu[p] = ok && i > 0 ? qy[g - W] : T(0);
        ql[p] = ok && j > 0 ? qx[g - 1] : T(0);
        vv[p] = ok ? f.v[g] : T(0);
        xh[p] = ok && f.mode != 0 && f.mode != 4 ? f.xhat[g] : T(0);
        hh[p] = ok && f.mode != 0 && f.mode != 4 ? f.h[g] : T(0);
        xo[p] = ok && (f.mode == 2 || f.mode == 4) ? f.x[g] : T(0);
    }
#pragma unroll
    for (int p = 0; p < FIN_PPT; ++p) {
        const int idx = (int)threadIdx.x + p * FIN_NT;
        const int li = idx / TW, lj = idx % TW;
        const int i = i0 + li, j = j0 + lj;
        if (i >= H || j >= W) continue;
        const size_t g = (size_t)i * W + j;
        T d = T(0);
        if (i < H - 1) d += qc_y[p];
        if (i > 0) d -= qu[p];
        if (j < W - 1) d += qc_x[p];
        if (j > 0) d -= ql[p];
        T z = vv[p] + d;
        if (f.nonneg) z = (z > T(0)) ? z : T(0);
        if (f.q_out != f.q) {
            f.q_out[g] = qc_y[p];
            f.q_out[plane + g] = qc_x[p];
        }
        if (f.mode == 0) {
            f.z[g] = z;
        } else {
            if (f.mode != 4) f.h[g] = hh[p] + f.rate * (z - xh[p]);
            if (f.mode >= 2) {
                // PDHGSkip-2 extrapolates; the stochastic-angle method
                // (mode 3) takes x+ itself; PDHGSkip-1 (mode 4) forms
                // x_{k+1} + xhat_k = c1 x+ - c2 x_k
                const T xb = f.mode == 3 ? z : (f.mode == 4 ? f.c1 * z - f.c2 * xo[p] : T(2) * z - xo[p]);
                f.xbar[(size_t)i * f.xbar_ld + j] = xb;
                s_t[li][lj] = xb;
            }
            f.x[g] = z;
        }
    }
    if (f.mode >= 2 && f.xbarT) {
        __syncthreads();
#pragma unroll
        for (int p = 0; p < FIN_PPT; ++p) {
            const int idx = (int)threadIdx.x + p * FIN_NT;
            const int jj = idx / TH, ii = idx % TH;
            const int i = i0 + ii, j = j0 + jj;
            if (i < H && j < W) f.xbarT[(size_t)j * f.xbarT_ld + i] = s_t[ii][jj];
        }
    }
}

template <typename T>
void launch_finalize(tvs_ctx* ctx, int H, int W, const Finalize<T>& f) {
    dim3 grid(div_up(W, 32), div_up(H, 32));
    hipLaunchKernelGGL((finalize_kernel<T>), grid, dim3(FIN_NT), 0, ctx->stream, f, H, W);
    TVS_LAUNCH_CHECK();
}

// Batched finalize (ProxSkip bookkeeping) over the active slices' 32 x 32 tiles.
template <typename T>
__global__ __launch_bounds__(256) void finalize_batched_kernel(const BSlice<T>* sl, BatchLists L,
                                                              const T* v, const T* q, T* q_out,
                                                              T* x, T* h, const T* xhat,
                                                              int nonneg) {
    const int b = (int)blockIdx.x;
    const int it = find_item(L.pref_fin, L.n_act, b);
    const BSlice<T> S = sl[L.act[it]];
    const int t = b - L.pref_fin[it];
    const int tiles_x = div_up(S.W, 32);
    const int i0 = (t / tiles_x) * 32, j0 = (t % tiles_x) * 32;
    const int H = S.H, W = S.W;
    const size_t off = (size_t)S.off, plane = (size_t)H * W;
    const T* qy = q + 2 * off;
    const T* qx = qy + plane;
    // all loads of the thread's four pixels before its stores
    T qc_y[4], qc_x[4], qu[4], ql[4], vv[4], xh[4], hh[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int idx = (int)threadIdx.x + p * 256;
        const int i = i0 + idx / 32, j = j0 + idx % 32;
        const bool ok = i < H && j < W;
        const size_t g = ok ? (size_t)i * W + j : 0;
        qc_y[p] = ok ? qy[g] : T(0);
        qc_x[p] = ok ? qx[g] : T(0);
        qu[p] = ok && i > 0 ? qy[g - W] : T(0);
        ql[p] = ok && j > 0 ? qx[g - 1] : T(0);
        vv[p] = ok ? v[off + g] : T(0);
        xh[p] = ok ? xhat[off + g] : T(0);
        hh[p] = ok ? h[off + g] : T(0);
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int idx = (int)threadIdx.x + p * 256;
        const int i = i0 + idx / 32, j = j0 + idx % 32;
        if (i >= H || j >= W) continue;
        const size_t g = (size_t)i * W + j;
        T d = T(0);
        if (i < H - 1) d += qc_y[p];
        if (i > 0) d -= qu[p];
        if (j < W - 1) d += qc_x[p];
        if (j > 0) d -= ql[p];
        T z = vv[p] + d;
        if (nonneg) z = (z > T(0)) ? z : T(0);
        if (q_out != q) {
            q_out[2 * off + g] = qc_y[p];
            q_out[2 * off + plane + g] = qc_x[p];
        }
        h[off + g] = hh[p] + S.rate * (z - xh[p]);
        x[off + g] = z;
    }
}

template <typename T>
void launch_finalize_batched(tvs_ctx* ctx, const BSlice<T>* sl, const BatchLists& L, const T* v,
                             const T* q, T* q_out, T* x, T* h, const T* xhat, int nonneg) {
    hipLaunchKernelGGL((finalize_batched_kernel<T>), dim3(L.tiles_fin), dim3(256), 0, ctx->stream,
                       sl, L, v, q, q_out, x, h, xhat, nonneg);
    TVS_LAUNCH_CHECK();
}

// ------------------------------------------------------------- grad / div
template <typename T>
__global__ void grad_kernel(int H, int W, const T* u, T* q) {
    const size_t n = (size_t)H * W;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(g / W), j = (int)(g % W);
        const T uc = u[g];
        q[g] = (i < H - 1) ? u[g + W] - uc : T(0);
        q[n + g] = (j < W - 1) ? u[g + 1] - uc : T(0);
    }
}

template <typename T>
__global__ void div_kernel(int H, int W, const T* q, T* out) {
    const size_t n = (size_t)H * W;
    const T* qy = q;
    const T* qx = q + n;
    for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n;
         g += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(g / W), j = (int)(g % W);
        T d = T(0);
        if (i < H - 1) d += qy[g];
        if (i > 0) d -= qy[g - W];
        if (j < W - 1) d += qx[g];
        if (j > 0) d -= qx[g - 1];
        out[g] = d;
    }
}

static int grid1d(size_t n) {
    size_t b = (n + 255) / 256;
    return (int)(b < 65536 ? (b ? b : 1) : 65536);
}

template <typename T>
void launch_grad(tvs_ctx* ctx, int H, int W, const T* u, T* q) {
    hipLaunchKernelGGL((grad_kernel<T>), dim3(grid1d((size_t)H * W)), dim3(256), 0, ctx->stream,
                       H, W, u, q);
    TVS_LAUNCH_CHECK();
}

template <typename T>
void launch_div(tvs_ctx* ctx, int H, int W, const T* q, T* u) {
    hipLaunchKernelGGL((div_kernel<T>), dim3(grid1d((size_t)H * W)), dim3(256), 0, ctx->stream,
                       H, W, q, u);
    TVS_LAUNCH_CHECK();
}

#define TVS_INST(T)                                                                          \
    template T* run_fgp<T>(tvs_ctx*, int, int, const T*, double, int, int, T*, const FgpConfig&,  \
                           const int*);                                                         \
    template T* run_fgp_bufs<T>(tvs_ctx*, int, int, const T*, double, int, int, T*, T* const*,    \
                                const T*, const FgpConfig&, const int*);                        \
    template T* run_fgp_batched<T>(tvs_ctx*, const BSlice<T>*, const BatchLists&, const T*, T*,   \
                                   size_t, int, int, const FgpConfig&);                          \
    template void launch_finalize_batched<T>(tvs_ctx*, const BSlice<T>*, const BatchLists&,      \
                                             const T*, const T*, T*, T*, T*, const T*, int);     \
    template void launch_finalize<T>(tvs_ctx*, int, int, const Finalize<T>&);                \
    template void launch_grad<T>(tvs_ctx*, int, int, const T*, T*);                          \
    template void launch_div<T>(tvs_ctx*, int, int, const T*, T*);
TVS_INST(float)
TVS_INST(double)
#undef TVS_INST

}  // namespace tvs
