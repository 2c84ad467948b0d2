// Least squares for a batch of small matrices after their batched
// factorisation: one workgroup per matrix runs the whole solve, Q^T b, the
// triangular solve and the refinement with FP64 residuals on the original
// A, up to its own stopping test, with no host round trip.  The operators
// are those of the single-matrix solver: Q^T and Q applied as the tile
// reflectors of Section 3.2.1 with the inner blocks of Section 3.2.3
// (Q^T = I - V T^T V^T per inner panel), Bjorck's augmented-system
// refinement for m > n and classical refinement for m == n (Section 3.2.4
// advises checking the backward error and refining).
//
// Vectors live in a per-matrix scratch area in device memory (small enough
// to stay in cache); every reduction has a fixed order, so results do not
// depend on timing.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "tileqr_internal.h"

namespace tq {

namespace {

constexpr int LT = 256;   // threads of the workgroup

// Sum of v over the workgroup, in a fixed order; every thread gets it.
__device__ double wg_sum(double v, double *red)
{
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
    for (int h = LT / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

__device__ double wg_max(double v, double *red)
{
    const int t = threadIdx.x;
    __syncthreads();
    red[t] = v;
    __syncthreads();
    for (int h = LT / 2; h > 0; h >>= 1) {
        if (t < h) red[t] = fmax(red[t], red[t + h]);
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

struct Mat {
    const LsDesc &D;
    __device__ const double *tile(int i, int j) const
    {
        return D.tiles + ((size_t)j * D.p + i) * (size_t)D.nb * D.nb;
    }
    __device__ const double *tblk(int k, int i) const { return D.T + ((size_t)k * D.p + i) * (size_t)D.ib * D.nb; }
    // R entry (r, c), r <= c < n.
    __device__ double R(int r, int c) const { return tile(r / D.nb, c / D.nb)[(size_t)(r % D.nb) * D.nb + c % D.nb]; }
};

// One inner panel (columns c0 .. c0 + ib of tile vt) applied to the vector
// f: with `diag` the diagonal reflectors of block k (V unit lower triangular
// from row c0), otherwise the coupled TS reflectors [e; V] acting on rows
// c0 .. c0 + ib of block k and all of block i.  trans: H^T (w <- T^T w),
// else H (w <- T w).  lds: at least (LT + 2 * 32) doubles.
__device__ void apply_panel_vec(const Mat &M, const double *vt, const double *Tl, int c0, bool diag, bool trans,
                                double *f, int k, int i, double *lds)
{
    const int nb = M.D.nb, ib = M.D.ib, t = threadIdx.x;
    const int parts = LT / ib, j = t % ib, part = t / ib;
    double *red = lds, *wv = lds + LT, *wt = lds + LT + 32;
    double *fk = f + (size_t)k * nb, *fi = f + (size_t)i * nb;
    const int rlo = diag ? c0 : 0;
    double s = 0.0;
    for (int r = rlo + part; r < nb; r += parts) {
        double v;
        if (diag) v = r == c0 + j ? 1.0 : (r > c0 + j ? vt[(size_t)r * nb + c0 + j] : 0.0);
        else v = vt[(size_t)r * nb + c0 + j];
        s += v * (diag ? fk[r] : fi[r]);
    }
    __syncthreads();
    red[part * ib + j] = s;
    __syncthreads();
    if (t < ib) {
        double w = diag ? 0.0 : fk[c0 + t];
        for (int q = 0; q < parts; ++q) w += red[q * ib + t];
        wv[t] = w;
    }
    __syncthreads();
    if (t < ib) {
        double w = 0.0;
        if (trans)
            for (int q = 0; q <= t; ++q) w += Tl[q * ib + t] * wv[q];   // (T^T w)_t
        else
            for (int q = t; q < ib; ++q) w += Tl[t * ib + q] * wv[q];   // (T w)_t
        wt[t] = w;
    }
    __syncthreads();
    if (!diag && t < ib) fk[c0 + t] -= wt[t];
    for (int r = rlo + t; r < nb; r += LT) {
        double u = 0.0;
        for (int q = 0; q < ib; ++q) {
            double v;
            if (diag) v = r == c0 + q ? 1.0 : (r > c0 + q ? vt[(size_t)r * nb + c0 + q] : 0.0);
            else v = vt[(size_t)r * nb + c0 + q];
            u += v * wt[q];
        }
        if (diag) fk[r] -= u;
        else fi[r] -= u;
    }
    __syncthreads();
}

// f <- Q^T f (trans) or Q f, f of p nb entries (row blocks).
__device__ void apply_q_vec(const Mat &M, double *f, bool trans, double *lds)
{
    const int p = M.D.p, kmax = min(M.D.p, M.D.q), np = M.D.nb / M.D.ib, ib = M.D.ib;
    for (int kk = 0; kk < kmax; ++kk) {
        const int k = trans ? kk : kmax - 1 - kk;
        // Q^T: the diagonal reflector, then the TS ones in ascending order;
        // Q: the same operators transposed, in reverse.
        for (int ii = 0; ii < p - k; ++ii) {
            const int i = trans ? k + ii : p - 1 - ii;
            const bool diag = i == k;
            const double *vt = M.tile(i, k), *Tb = M.tblk(k, i);
            for (int ll = 0; ll < np; ++ll) {
                const int l = trans ? ll : np - 1 - ll;
                apply_panel_vec(M, vt, Tb + (size_t)l * ib * ib, l * ib, diag, trans, f, k, i, lds);
            }
        }
    }
}

// y <- R^{-1} y (upper) or R^{-T} y, first n entries, by 64-row blocks: the
// diagonal block staged in LDS and solved by substitution on wave 0, then
// the rows outside it updated.  An exact zero on the diagonal sets
// STATUS_SINGULAR (and gives 0).  lds: 64 x 65 + 64 doubles.
__device__ void trsv_vec(const Mat &M, double *y, bool upper, double *lds, int *status)
{
    const int n = M.D.n, t = threadIdx.x;
    const int nrb = (n + 63) / 64;
    double *Rb = lds, *xs = lds + 64 * 65;
    for (int bb = 0; bb < nrb; ++bb) {
        const int rb = upper ? nrb - 1 - bb : bb;
        const int r0 = rb * 64, cnt = min(64, n - r0);
        __syncthreads();
        // Rb[a][c] = op(R)[r0 + a][r0 + c]
        for (int e = t; e < 64 * 64; e += LT) {
            const int a = e / 64, c = e % 64;
            double v = 0.0;
            if (a < cnt && c < cnt) v = upper ? (c >= a ? M.R(r0 + a, r0 + c) : 0.0) : (a >= c ? M.R(r0 + c, r0 + a) : 0.0);
            Rb[a * 65 + c] = v;
        }
        __syncthreads();
        if (t < 64) {
            double yv = t < cnt ? y[r0 + t] : 0.0;
            for (int s = 0; s < cnt; ++s) {
                const int c = upper ? cnt - 1 - s : s;
                double xc = 0.0;
                if (t == c) {
                    const double d = Rb[c * 65 + c];
                    if (d == 0.0) atomicOr(status, STATUS_SINGULAR);
                    xc = d != 0.0 ? yv / d : 0.0;
                }
                xc = __shfl(xc, c, 64);
                if (t == c) yv = xc;
                else if (upper ? t < c : t > c) yv -= Rb[t * 65 + c] * xc;
            }
            xs[t] = yv;
            if (t < cnt) y[r0 + t] = yv;
        }
        __syncthreads();
        // Rows outside the block that depend on it.
        if (upper) {
            for (int r = t; r < r0; r += LT) {
                double u = 0.0;
                for (int c = 0; c < cnt; ++c) u += M.R(r, r0 + c) * xs[c];
                y[r] -= u;
            }
        } else {
            for (int r = r0 + cnt + t; r < n; r += LT) {
                double u = 0.0;
                for (int c = 0; c < cnt; ++c) u += M.R(r0 + c, r) * xs[c];
                y[r] -= u;
            }
        }
    }
    __syncthreads();
}

// rr <- b - A x (rows < m); returns nothing.
__device__ void residual(const LsDesc &D, const double *x, double *rr)
{
    for (int r = threadIdx.x; r < D.m; r += LT) {
        double s = D.b[r];
        for (int c = 0; c < D.n; ++c) s -= D.A[(size_t)c * D.lda + r] * x[c];
        rr[r] = s;
    }
    __syncthreads();
}

// g <- alpha A^T v (n entries): wave w takes columns w, w + 4, .., lanes
// sum rows in a fixed order, then a fixed butterfly over the wave.
__device__ void gemv_t(const LsDesc &D, const double *v, double *g, double alpha)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int c = w; c < D.n; c += LT / 64) {
        double s = 0.0;
        for (int r = lane; r < D.m; r += 64) s += D.A[(size_t)c * D.lda + r] * v[r];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) g[c] = alpha * s;
    }
    __syncthreads();
}

// Backward errors of x with its fresh residual rr = b - A x (formed here):
//   eta_ls = ||A^T rr||_2 / (||A||_F (||A||_F ||x||_2 + ||b||_2))
//   eta_inf = ||rr||_inf / (||A||_inf ||x||_inf)      (square systems)
__device__ double measure(const LsDesc &D, const double *x, double *rr, double *g, double normA, double normb,
                          double normAinf, bool square, double *red)
{
    residual(D, x, rr);
    gemv_t(D, rr, g, 1.0);
    double sg = 0.0, sx = 0.0, mx = 0.0, mr = 0.0;
    for (int c = threadIdx.x; c < D.n; c += LT) {
        sg += g[c] * g[c];
        sx += x[c] * x[c];
        mx = fmax(mx, fabs(x[c]));
    }
    for (int r = threadIdx.x; r < D.m; r += LT) mr = fmax(mr, fabs(rr[r]));
    const double ng = sqrt(wg_sum(sg, red)), nx = sqrt(wg_sum(sx, red));
    const double den = normA * (normA * nx + normb);
    double eta = den > 0.0 ? ng / den : (ng > 0.0 ? INFINITY : 0.0);
    if (square) {
        const double xi = wg_max(mx, red), ri = wg_max(mr, red);
        const double di = normAinf * xi;
        eta = fmax(eta, di > 0.0 ? ri / di : (ri > 0.0 ? INFINITY : 0.0));
    }
    return eta;
}

}  // namespace

__global__ __launch_bounds__(LT) void k_ls_batched(const LsDesc *descs, int count, double tol, int max_iter,
                                                   LsOut *out, int *status)
{
    __shared__ double lds[64 * 65 + 64 + LT];
    __shared__ int s_status;
    const int mi = blockIdx.x;
    if (mi >= count) return;
    const LsDesc &D = descs[mi];
    const Mat M{D};
    const int t = threadIdx.x;
    const int m = D.m, n = D.n, rows = D.p * D.nb;
    const bool square = m == n;
    double *red = lds + 64 * 65 + 64;
    double *f = D.work, *r = f + rows, *rr = r + rows, *g = rr + rows, *x = g + rows, *dx = x + rows,
           *xb = dx + rows;
    if (t == 0) s_status = 0;
    // Norms fixed for the whole refinement.
    double sa = 0.0, sb = 0.0;
    for (int rw = t; rw < m; rw += LT) {
        double ar = 0.0;
        for (int c = 0; c < n; ++c) {
            const double a = D.A[(size_t)c * D.lda + rw];
            sa += a * a;
            ar += fabs(a);
        }
        sb += D.b[rw] * D.b[rw];
        dx[rw] = ar;    // row sums of |A| (dx is free until the refinement)
    }
    __syncthreads();
    double ma = 0.0;
    for (int rw = t; rw < m; rw += LT) ma = fmax(ma, dx[rw]);
    const double normA = sqrt(wg_sum(sa, red)), normb = sqrt(wg_sum(sb, red));
    const double normAinf = wg_max(ma, red);

    // x0 = R^{-1} (Q^T b)(0:n), r0 = b - A x0.
    for (int e = t; e < rows; e += LT) f[e] = e < m ? D.b[e] : 0.0;
    __syncthreads();
    apply_q_vec(M, f, true, lds);
    for (int e = t; e < rows; e += LT) x[e] = e < n ? f[e] : 0.0;
    __syncthreads();
    trsv_vec(M, x, true, lds, &s_status);
    double eta = measure(D, x, rr, g, normA, normb, normAinf, square, red);
    for (int e = t; e < rows; e += LT) {
        r[e] = e < m ? rr[e] : 0.0;
        xb[e] = x[e];
    }
    __syncthreads();
    double best = eta, prev = eta;
    int it = 0, stall = 0;
    while (eta > tol && it < max_iter && s_status == 0) {
        ++it;
        if (square) {
            // dx = R^{-1} Q^T (b - A x), with the residual measure left in rr.
            for (int e = t; e < rows; e += LT) f[e] = e < m ? rr[e] : 0.0;
            __syncthreads();
            apply_q_vec(M, f, true, lds);
            trsv_vec(M, f, true, lds, &s_status);
            for (int e = t; e < n; e += LT) x[e] += f[e];
        } else {
            // f = b - r - A x ; g = -A^T r ; [f1; f2] = Q^T f ; d1 = R^{-T} g ;
            // dx = R^{-1} (f1 - d1) ; dr = Q [d1; f2] ; x += dx ; r += dr.
            for (int e = t; e < rows; e += LT) f[e] = e < m ? rr[e] - r[e] : 0.0;   // rr = b - A x
            __syncthreads();
            gemv_t(D, r, g, -1.0);
            apply_q_vec(M, f, true, lds);
            trsv_vec(M, g, false, lds, &s_status);
            for (int e = t; e < rows; e += LT) dx[e] = e < n ? f[e] - g[e] : 0.0;
            __syncthreads();
            trsv_vec(M, dx, true, lds, &s_status);
            for (int e = t; e < n; e += LT) f[e] = g[e];
            __syncthreads();
            apply_q_vec(M, f, false, lds);
            for (int e = t; e < n; e += LT) x[e] += dx[e];
            for (int e = t; e < m; e += LT) r[e] += f[e];
        }
        __syncthreads();
        eta = measure(D, x, rr, g, normA, normb, normAinf, square, red);
        if (eta < best) {
            best = eta;
            for (int e = t; e < n; e += LT) xb[e] = x[e];
        }
        stall = eta > 0.5 * prev ? stall + 1 : 0;
        prev = eta;
        __syncthreads();
        if (stall >= 2) break;
    }
    for (int e = t; e < n; e += LT) D.x[e] = xb[e];
    if (t == 0) {
        out[mi].eta = best;
        out[mi].iterations = it;
        out[mi].status = s_status;
        if (s_status) atomicOr(status, s_status);
    }
}

hipError_t launch_ls_batched(const LsDesc *descs, int count, double tol, int max_iter, LsOut *out, int *status,
                             hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ls_batched, dim3((unsigned)count), dim3(LT), 0, st, descs, count, tol, max_iter, out, status);
    return hipGetLastError();
}

}  // namespace tq
