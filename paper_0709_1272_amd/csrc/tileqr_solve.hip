// Triangular solves with the tiled R, and the FP64 matrix-vector products and
// norms the least-squares solver and its refinement need.
//
// R lives in the factorisation's tiles (tile (i, j) at tiles + (j p + i) nb^2,
// row-major inside, R in the upper triangle of tiles i <= j).  Right-hand
// sides live in row blocks: block i holds rows [i nb, (i+1) nb) of a row-major
// array with leading dimension ldt (a multiple of 32).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "tileqr_internal.h"

namespace tq {

namespace {

constexpr int SW = 32;   // columns per strip of right-hand sides

__device__ __forceinline__ const double *tile_at(const double *tiles, int p, int nb, int i, int j)
{
    return tiles + ((size_t)j * p + i) * (size_t)nb * nb;
}

// store(e, load(e)) for e = tid, tid + nt, .. (COUNT per thread), with every
// load issued before the first store, so that the loads' latencies overlap
// (a plain copy loop waits for each load before the next one).
template <int COUNT, typename Load, typename Store>
__device__ __forceinline__ void batched_copy(int tid, int nt, Load load, Store store)
{
    double v[COUNT];
#pragma unroll
    for (int u = 0; u < COUNT; ++u) v[u] = load(tid + u * nt);
#pragma unroll
    for (int u = 0; u < COUNT; ++u) store(tid + u * nt, v[u]);
}

}  // namespace

// Triangular solve with the tiled R on a 32-wide strip of right-hand sides,
// one workgroup per row block i (and strip, blockIdx.y):
//   upper == true:  R X = C,   X_i = R_ii^{-1} (C_i - sum_{j > i} R_ij X_j)
//   upper == false: R^T X = C, X_i = R_ii^{-T} (C_i - sum_{j < i} R_ji^T X_j)
// The workgroup applies the solved blocks X_j as soon as their workgroup
// publishes them (progress flags, FLAG_STRIDE words apart), accumulating
// op(R)_ij X_j in registers (4 x 4 outputs per thread, op(R) staged in LDS by
// 32-column chunks), then solves with its diagonal tile and publishes X_i.
// Producers have the lower workgroup indices (for R the last block comes
// first), so every wait is on a workgroup that was dispatched earlier; every
// wait is bounded (STATUS_TIMEOUT).  The diagonal tile is taken in 32 x 32
// blocks: the 32 columns of op(R) holding a block are staged in LDS, the
// block is solved by half-waves (one right-hand side per half-wave, one row
// per lane, reciprocals of the diagonal computed once) and the rows that
// depend on it are updated by a register-blocked product.  Rows at or beyond
// `n` (padding) get X = 0; an exact zero on the diagonal of a real row sets
// STATUS_SINGULAR.
template <int NB>
__global__ __launch_bounds__(2 * NB) void k_trsm(const double *tiles, int p, int q, int64_t n, double *C, int ldt,
                                                 int upper, int *flags, int *status, int64_t spin_limit)
{
    constexpr int NT = 2 * NB, NBLK = NB / 32;
    __shared__ double Xs[NB][SW + 1];
    __shared__ double Rc[NB][33];
    __shared__ double dinv[32];
    __shared__ int s_abort;
    const int tid = threadIdx.x, lane = tid & 63, hw = tid >> 5;   // half-wave index
    const int strip = blockIdx.y, nstrip = gridDim.y, s0 = strip * SW;
    const int i = upper ? q - 1 - (int)blockIdx.x : (int)blockIdx.x;
    double *Ci = C + (size_t)i * NB * ldt;
    const int rgp = tid / 8, cg = tid % 8;   // rows 4 rgp .. +3, columns 4 cg .. +3
    double acc[4][4] = {};
    const int nj = upper ? q - 1 - i : i;
    for (int t = 0; t < nj; ++t) {
        const int j = upper ? q - 1 - t : t;
        if (tid == 0) {
            const int *flag = &flags[(j * nstrip + strip) * FLAG_STRIDE];
            int abort = 0, backoff = 0;
            int64_t spins = 0;
            while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & STATUS_TIMEOUT ||
                    ++spins > spin_limit) {
                    __hip_atomic_fetch_or(status, STATUS_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    abort = 1;
                    break;
                }
                backoff = backoff < 6 ? backoff + 1 : 6;
                for (int z = 0; z < (1 << backoff); ++z) __builtin_amdgcn_s_sleep(2);
            }
            s_abort = abort;
        }
        __syncthreads();
        if (s_abort) return;
        if (tid < 64) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        const double *Rt = upper ? tile_at(tiles, p, NB, i, j) : tile_at(tiles, p, NB, j, i);
        const double *Cj = C + (size_t)j * NB * ldt;
        batched_copy<NB * SW / NT>(tid, NT, [&](int e) { return Cj[(size_t)(e / SW) * ldt + s0 + e % SW]; },
                                   [&](int e, double v) { Xs[e / SW][e % SW] = v; });
        for (int kc = 0; kc < NB; kc += 32) {
            __syncthreads();
            // Rc[row][kk] = op(R)_ij[row][kc + kk]
            if (upper)
                batched_copy<NB * 32 / NT>(tid, NT, [&](int e) { return Rt[(size_t)(e / 32) * NB + kc + e % 32]; },
                                           [&](int e, double v) { Rc[e / 32][e % 32] = v; });
            else
                batched_copy<NB * 32 / NT>(tid, NT, [&](int e) { return Rt[(size_t)(kc + e / NB) * NB + e % NB]; },
                                           [&](int e, double v) { Rc[e % NB][e / NB] = v; });
            __syncthreads();
            for (int kk = 0; kk < 32; ++kk) {
                double a[4], b[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = Rc[4 * rgp + u][kk];
                    b[u] = Xs[kc + kk][4 * cg + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
            }
        }
        __syncthreads();
    }
    // X_i <- C_i - accumulated products, then the diagonal solve in place.
    batched_copy<NB * SW / NT>(tid, NT, [&](int e) { return Ci[(size_t)(e / SW) * ldt + s0 + e % SW]; },
                               [&](int e, double v) { Xs[e / SW][e % SW] = v; });
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) Xs[4 * rgp + u][4 * cg + v] -= acc[u][v];
    const double *R = tile_at(tiles, p, NB, i, i);
    for (int bb = 0; bb < NBLK; ++bb) {
        const int b = upper ? NBLK - 1 - bb : bb;
        __syncthreads();
        if (upper)
            batched_copy<NB * 32 / NT>(tid, NT, [&](int e) { return R[(size_t)(e / 32) * NB + b * 32 + e % 32]; },
                                       [&](int e, double v) { Rc[e / 32][e % 32] = v; });
        else
            batched_copy<NB * 32 / NT>(tid, NT, [&](int e) { return R[(size_t)(b * 32 + e / NB) * NB + e % NB]; },
                                       [&](int e, double v) { Rc[e % NB][e / NB] = v; });
        __syncthreads();
        if (tid < 32) {
            const double d = Rc[b * 32 + tid][tid];
            const bool real = (int64_t)i * NB + b * 32 + tid < n;
            if (real && d == 0.0) atomicOr(status, STATUS_SINGULAR);
            dinv[tid] = (real && d != 0.0) ? 1.0 / d : 0.0;
        }
        __syncthreads();
        const int r_i = lane & 31;
        const int64_t grow = (int64_t)i * NB + b * 32 + r_i;
        // The half-wave's right-hand sides (columns hw, hw + HW, ..) advance
        // together, so that their substitution chains overlap.
        constexpr int HW = NT / 32, CPH = SW / HW;
        double x[CPH];
#pragma unroll
        for (int u = 0; u < CPH; ++u) x[u] = Xs[b * 32 + r_i][hw + u * HW];
        for (int qq = 0; qq < 32; ++qq) {
            const int r = upper ? 31 - qq : qq;
            const double rv = Rc[b * 32 + r_i][r], dr = dinv[r];
#pragma unroll
            for (int u = 0; u < CPH; ++u) {
                const double xr = __shfl(x[u], r, 32) * dr;
                if (r_i == r) x[u] = xr;
                else if (upper ? r_i < r : r_i > r) x[u] -= rv * xr;
            }
        }
#pragma unroll
        for (int u = 0; u < CPH; ++u) Xs[b * 32 + r_i][hw + u * HW] = grow < n ? x[u] : 0.0;
        __syncthreads();
        // Rows outside the block that depend on it.
        const int r0 = upper ? 0 : (b + 1) * 32, r1 = upper ? b * 32 : NB;
        if (4 * rgp >= r0 && 4 * rgp < r1) {
            double d4a[4][4] = {};
            for (int jj = 0; jj < 32; ++jj) {
                double a[4], xv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = Rc[4 * rgp + u][jj];
                    xv[u] = Xs[b * 32 + jj][4 * cg + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) d4a[u][v] += a[u] * xv[v];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) Xs[4 * rgp + u][4 * cg + v] -= d4a[u][v];
        }
    }
    __syncthreads();
    for (int e = tid; e < NB * SW; e += NT) Ci[(size_t)(e / SW) * ldt + s0 + e % SW] = Xs[e / SW][e % SW];
    // Publish X_i: every wave waits for its stores, then one writes back
    // and raises the flag.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&flags[(i * nstrip + strip) * FLAG_STRIDE], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Y (row-major rows, leading dimension ldt, m x nrhs) <- alpha A X + beta Y
// for column-major A (m x n, lda) and X in row blocks (n x nrhs, ldt).  A is
// read once: each workgroup takes 256 rows and a slice of the columns; the
// per-slice partial sums are written to `part` and reduced in a second pass
// in slice order (deterministic).
__global__ __launch_bounds__(256) void k_gemv_n_part(const double *A, int64_t lda, int64_t m, int64_t n,
                                                     const double *X, int ldt, int nrhs, int64_t cols_per_slice,
                                                     double *part)
{
    __shared__ double xs[64][SW];
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * cols_per_slice, c1 = std::min<int64_t>(n, c0 + cols_per_slice);
    const int nr = std::min(nrhs, SW);
    double acc[SW];
#pragma unroll
    for (int v = 0; v < SW; ++v) acc[v] = 0.0;
    for (int64_t cb = c0; cb < c1; cb += 64) {
        __syncthreads();
        batched_copy<64 * SW / 256>((int)threadIdx.x, 256,
                                    [&](int e) {
                                        const int64_t c = cb + e / SW;
                                        return (c < c1 && e % SW < nr) ? X[c * ldt + e % SW] : 0.0;
                                    },
                                    [&](int e, double v) { xs[e / SW][e % SW] = v; });
        __syncthreads();
        if (row < m) {
            const int cn = (int)std::min<int64_t>(64, c1 - cb);
            for (int j = 0; j < cn; ++j) {
                const double a = A[(cb + j) * lda + row];
#pragma unroll
                for (int v = 0; v < SW; ++v) acc[v] += a * xs[j][v];
            }
        }
    }
    if (row < m)
        for (int v = 0; v < nr; ++v) part[((int64_t)blockIdx.y * m + row) * SW + v] = acc[v];
}

__global__ void k_gemv_n_sum(const double *part, int nslice, int64_t m, int nrhs, double alpha, double beta, double *Y,
                             int ldt)
{
    const int64_t total = m * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = e / nrhs;
        const int v = (int)(e % nrhs);
        double s = 0.0;
        for (int q = 0; q < nslice; ++q) s += part[((int64_t)q * m + row) * SW + v];
        Y[row * ldt + v] = alpha * s + (beta == 0.0 ? 0.0 : beta * Y[row * ldt + v]);
    }
}

// Y (n x nrhs rows) <- alpha A^T R + beta Y.  Workgroup (x, y) takes 64
// columns of A and a slice of its rows: per chunk of 64 rows the chunk of R
// and the 64 x 64 block of A are staged in LDS (A read once, coalesced down
// its columns), each thread keeps 8 outputs (one column, 8 right-hand
// sides); the per-slice partial sums go to `part` and a second pass adds
// them in slice order (deterministic).
__global__ __launch_bounds__(256) void k_gemv_t_part(const double *A, int64_t lda, int64_t m, int64_t n,
                                                     const double *Rv, int ldt, int nr, int64_t rows_per_slice,
                                                     double *part)
{
    __shared__ double rs[64][SW + 1];
    __shared__ double as[64][65];
    const int tid = threadIdx.x, cl = tid % 64, vg = tid / 64;
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_slice, r1 = std::min<int64_t>(m, r0 + rows_per_slice);
    double acc[8] = {};
    for (int64_t rb = r0; rb < r1; rb += 64) {
        __syncthreads();
        batched_copy<64 * SW / 256>(tid, 256,
                                    [&](int e) {
                                        const int64_t row = rb + e / SW;
                                        return (row < r1 && e % SW < nr) ? Rv[row * ldt + e % SW] : 0.0;
                                    },
                                    [&](int e, double v) { rs[e / SW][e % SW] = v; });
        batched_copy<64 * 64 / 256>(tid, 256,
                                    [&](int e) {
                                        const int64_t row = rb + e % 64, col = c0 + e / 64;
                                        return (row < r1 && col < n) ? A[col * lda + row] : 0.0;
                                    },
                                    [&](int e, double v) { as[e / 64][e % 64] = v; });
        __syncthreads();
        for (int rr = 0; rr < 64; ++rr) {
            const double a = as[cl][rr];
#pragma unroll
            for (int v = 0; v < 8; ++v) acc[v] += a * rs[rr][vg * 8 + v];
        }
    }
    const int64_t col = c0 + cl;
    if (col < n)
#pragma unroll
        for (int v = 0; v < 8; ++v)
            if (vg * 8 + v < nr) part[((int64_t)blockIdx.y * n + col) * SW + vg * 8 + v] = acc[v];
}

__global__ void k_gemv_t_sum(const double *part, int nslice, int64_t n, int nr, double alpha, double beta, double *Y,
                             int ldt)
{
    const int64_t total = n * nr;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t col = e / nr;
        const int v = (int)(e % nr);
        double s = 0.0;
        for (int q = 0; q < nslice; ++q) s += part[((int64_t)q * n + col) * SW + v];
        Y[col * ldt + v] = alpha * s + (beta == 0.0 ? 0.0 : beta * Y[col * ldt + v]);
    }
}

// out[v] = sum over rows r < m of Y[r][v]^2 (per column v < nrhs), in a
// fixed order: per-block partial sums, then one block adds them in order.
__global__ __launch_bounds__(256) void k_colsq_part(const double *Y, int ldt, int64_t m, int nrhs, double *part)
{
    __shared__ double red[256];
    for (int v = 0; v < nrhs; ++v) {
        double s = 0.0;
        for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < m; r += (int64_t)gridDim.x * 256) {
            const double y = Y[r * ldt + v];
            s += y * y;
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)v * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

__global__ void k_colsq_sum(const double *part, int nblk, int nrhs, double *out)
{
    const int v = threadIdx.x;
    if (v < nrhs) {
        double s = 0.0;
        for (int q = 0; q < nblk; ++q) s += part[(int64_t)v * nblk + q];
        out[v] = s;
    }
}

// ||A||_F^2 of a column-major matrix, same two-pass scheme (one column per
// thread block row of work).
__global__ __launch_bounds__(256) void k_frob_part(const double *A, int64_t lda, int64_t m, int64_t n, double *part)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t c = blockIdx.x; c < n; c += gridDim.x)
        for (int64_t r = threadIdx.x; r < m; r += 256) {
            const double a = A[c * lda + r];
            s += a * a;
        }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[v] = max over rows r < m of |Y[r][v]| (per column v < nrhs): per-block
// maxima, then one block takes the maximum of those (order-independent).
__global__ __launch_bounds__(256) void k_colmax_part(const double *Y, int ldt, int64_t m, int nrhs, double *part)
{
    __shared__ double red[256];
    for (int v = 0; v < nrhs; ++v) {
        double s = 0.0;
        for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < m; r += (int64_t)gridDim.x * 256)
            s = fmax(s, fabs(Y[r * ldt + v]));
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)v * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
}

__global__ void k_colmax_sum(const double *part, int nblk, int nrhs, double *out)
{
    const int v = threadIdx.x;
    if (v < nrhs) {
        double s = 0.0;
        for (int q = 0; q < nblk; ++q) s = fmax(s, part[(int64_t)v * nblk + q]);
        out[v] = s;
    }
}

// ||A||_inf = max over rows of sum_c |A[r][c]| for column-major A.  Pass 1:
// workgroup (x, y) sums rows [256 x, 256 x + 256) over the column slice y
// (consecutive threads read consecutive rows: coalesced); pass 2 adds the
// slices of each row in slice order and takes per-block maxima; pass 3 the
// maximum of those.
__global__ __launch_bounds__(256) void k_absrow_part(const double *A, int64_t lda, int64_t m, int64_t n,
                                                     int64_t cols_per_slice, double *part)
{
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.y * cols_per_slice, c1 = std::min<int64_t>(n, c0 + cols_per_slice);
    if (row >= m) return;
    double s = 0.0;
    for (int64_t c = c0; c < c1; ++c) s += fabs(A[c * lda + row]);
    part[(int64_t)blockIdx.y * m + row] = s;
}

__global__ __launch_bounds__(256) void k_absrow_max(const double *part, int nslice, int64_t m, double *out)
{
    __shared__ double red[256];
    double mx = 0.0;
    for (int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x; row < m; row += (int64_t)gridDim.x * 256) {
        double s = 0.0;
        for (int q = 0; q < nslice; ++q) s += part[(int64_t)q * m + row];
        mx = fmax(mx, s);
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Y[r][v] <- N(0, 1) for r < rows, v < cols (zero in the other columns up to
// ldt), by the Box-Muller transform of two uniforms drawn from a
// counter-based hash of (seed, r, v): probe vectors of the factorisation
// check.
__device__ __forceinline__ uint64_t hash64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

__global__ void k_fill_normal(double *Y, int ldt, int64_t rows, int cols, uint64_t seed)
{
    const int64_t total = rows * ldt;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int v = (int)(e % ldt);
        double z = 0.0;
        if (v < cols) {
            const uint64_t h1 = hash64(seed * 0x9e3779b97f4a7c15ULL + 2 * (uint64_t)e + 1);
            const uint64_t h2 = hash64(h1 ^ 0x632be59bd9b4e019ULL);
            const double u1 = ((double)(h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);   // (0, 1)
            const double u2 = (double)(h2 >> 11) * (1.0 / 9007199254740992.0);
            z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
        }
        Y[e] = z;
    }
}

// W = R Z for the tiled R (upper triangle of tiles i <= j < q, R_ii its upper
// triangle only) and Z in row blocks (rows >= n zero): workgroup (i, strip)
// forms W_i = sum_{j >= i} R_ij Z_j for one 32-wide strip, staging Z_j and
// 32-column chunks of R_ij in LDS; row blocks i >= q get W_i = 0.
template <int NB>
__global__ __launch_bounds__(2 * NB) void k_trmm(const double *tiles, int p, int q, double *W, const double *Z,
                                                 int ldt)
{
    constexpr int NT = 2 * NB;
    __shared__ double Zs[NB][SW + 1];
    __shared__ double Rc[NB][33];
    const int tid = threadIdx.x, i = (int)blockIdx.x, s0 = (int)blockIdx.y * SW;
    const int rgp = tid / 8, cg = tid % 8;   // rows 4 rgp .. +3, columns 4 cg .. +3
    double acc[4][4] = {};
    for (int j = i; j < q; ++j) {
        const double *Rt = tile_at(tiles, p, NB, i, j);
        const double *Zj = Z + (size_t)j * NB * ldt;
        __syncthreads();
        batched_copy<NB * SW / NT>(tid, NT, [&](int e) { return Zj[(size_t)(e / SW) * ldt + s0 + e % SW]; },
                                   [&](int e, double v) { Zs[e / SW][e % SW] = v; });
        for (int kc = 0; kc < NB; kc += 32) {
            __syncthreads();
            batched_copy<NB * 32 / NT>(tid, NT,
                                       [&](int e) {
                                           const int r = e / 32, c = kc + e % 32;
                                           return (j > i || c >= r) ? Rt[(size_t)r * NB + c] : 0.0;
                                       },
                                       [&](int e, double v) { Rc[e / 32][e % 32] = v; });
            __syncthreads();
            for (int kk = 0; kk < 32; ++kk) {
                double a[4], b[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = Rc[4 * rgp + u][kk];
                    b[u] = Zs[kc + kk][4 * cg + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
            }
        }
    }
    double *Wi = W + (size_t)i * NB * ldt;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) Wi[(size_t)(4 * rgp + u) * ldt + s0 + 4 * cg + v] = acc[u][v];
}

// Elementwise helpers on row blocks (rows < m, columns < nrhs).
//   op 0: Y = X - Y       op 1: Y += X      op 2: Y = X      op 3: Y = -Y
__global__ void k_axpy_rows(const double *X, double *Y, int ldt, int64_t m, int nrhs, int op)
{
    const int64_t total = m * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t off = (e / nrhs) * ldt + e % nrhs;
        if (op == 0) Y[off] = X[off] - Y[off];
        else if (op == 1) Y[off] += X[off];
        else if (op == 2) Y[off] = X[off];
        else Y[off] = -Y[off];
    }
}

// Progress flags of k_trsm <- 0 (one per FLAG_STRIDE words).
__global__ void k_fill_flags(int *flags, int count)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < count; e += gridDim.x * blockDim.x)
        flags[e * FLAG_STRIDE] = 0;
}

// ------------------------------------------------------------ launchers

template <int NB>
static hipError_t trsm_impl(const double *tiles, int p, int64_t n, double *C, int ldt, bool upper, int *flags,
                            int *status, int64_t spin_limit, hipStream_t st)
{
    const int q = (int)((n + NB - 1) / NB);
    const int nstrip = ldt / SW;
    hipLaunchKernelGGL(k_fill_flags, dim3((unsigned)std::max(1, std::min(1024, (q * nstrip + 255) / 256))), dim3(256),
                       0, st, flags, q * nstrip);
    hipLaunchKernelGGL(k_trsm<NB>, dim3(q, nstrip), dim3(2 * NB), 0, st, tiles, p, q, n, C, ldt, upper ? 1 : 0, flags,
                       status, spin_limit);
    return hipGetLastError();
}

hipError_t launch_trsm(int nb, const double *tiles, int p, int64_t n, double *C, int ldt, bool upper, int *flags,
                       int64_t flags_cap, int *status, int64_t spin_limit, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t q = (n + nb - 1) / nb;
    if (q * (ldt / SW) * FLAG_STRIDE > flags_cap) return hipErrorInvalidValue;
    if (nb == 64) return trsm_impl<64>(tiles, p, n, C, ldt, upper, flags, status, spin_limit, st);
    if (nb == 128) return trsm_impl<128>(tiles, p, n, C, ldt, upper, flags, status, spin_limit, st);
    if (nb == 256) return trsm_impl<256>(tiles, p, n, C, ldt, upper, flags, status, spin_limit, st);
    return hipErrorInvalidValue;
}

hipError_t launch_gemv_n(const double *A, int64_t lda, int64_t m, int64_t n, const double *X, int ldt, int nrhs,
                         double alpha, double beta, double *Y, double *part, int64_t part_cap, hipStream_t st)
{
    if (m <= 0 || nrhs <= 0) return hipSuccess;
    for (int v0 = 0; v0 < nrhs; v0 += SW) {
        const int nr = std::min(SW, nrhs - v0);
        const int64_t rowblk = (m + 255) / 256;
        int64_t nslice = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048 / std::max<int64_t>(1, rowblk) + 1));
        nslice = std::min<int64_t>(nslice, std::max<int64_t>(1, part_cap / (m * SW)));
        const int64_t cps = (n + nslice - 1) / nslice;
        hipLaunchKernelGGL(k_gemv_n_part, dim3((unsigned)rowblk, (unsigned)nslice), dim3(256), 0, st, A, lda, m, n,
                           X + v0, ldt, nr, cps, part);
        const int64_t blocks = std::min<int64_t>((m * nr + 255) / 256, 4096);
        hipLaunchKernelGGL(k_gemv_n_sum, dim3((unsigned)blocks), dim3(256), 0, st, part, (int)nslice, m, nr, alpha,
                           beta, Y + v0, ldt);
    }
    return hipGetLastError();
}

hipError_t launch_gemv_t(const double *A, int64_t lda, int64_t m, int64_t n, const double *R, int ldt, int nrhs,
                         double alpha, double beta, double *Y, double *part, int64_t part_cap, hipStream_t st)
{
    if (n <= 0 || nrhs <= 0) return hipSuccess;
    const int64_t colblk = (n + 63) / 64, rowchunks = std::max<int64_t>(1, (m + 63) / 64);
    int64_t nslice = std::max<int64_t>(1, std::min<int64_t>(rowchunks, (2048 + colblk - 1) / colblk));
    nslice = std::min<int64_t>(nslice, part_cap / (n * SW));
    if (nslice < 1) return hipErrorInvalidValue;
    const int64_t rps = ((m + nslice - 1) / nslice + 63) / 64 * 64;
    nslice = std::max<int64_t>(1, (m + rps - 1) / rps);
    for (int v0 = 0; v0 < nrhs; v0 += SW) {
        const int nr = std::min(SW, nrhs - v0);
        hipLaunchKernelGGL(k_gemv_t_part, dim3((unsigned)colblk, (unsigned)nslice), dim3(256), 0, st, A, lda, m, n,
                           R + v0, ldt, nr, rps, part);
        const int64_t blocks = std::min<int64_t>((n * nr + 255) / 256, 4096);
        hipLaunchKernelGGL(k_gemv_t_sum, dim3((unsigned)blocks), dim3(256), 0, st, part, (int)nslice, n, nr, alpha,
                           beta, Y + v0, ldt);
    }
    return hipGetLastError();
}

hipError_t launch_colsq(const double *Y, int ldt, int64_t m, int nrhs, double *part, int64_t part_cap, double *out,
                        hipStream_t st)
{
    const int nblk = COLSQ_BLOCKS;
    if ((int64_t)nblk * nrhs > part_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_colsq_part, dim3(nblk), dim3(256), 0, st, Y, ldt, m, nrhs, part);
    hipLaunchKernelGGL(k_colsq_sum, dim3(1), dim3(64), 0, st, part, nblk, nrhs, out);
    return hipGetLastError();
}

hipError_t launch_frob2(const double *A, int64_t lda, int64_t m, int64_t n, double *part, int64_t part_cap,
                        double *out, hipStream_t st)
{
    const int nblk = COLSQ_BLOCKS;
    if (nblk > part_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_frob_part, dim3(nblk), dim3(256), 0, st, A, lda, m, n, part);
    hipLaunchKernelGGL(k_colsq_sum, dim3(1), dim3(64), 0, st, part, nblk, 1, out);
    return hipGetLastError();
}

hipError_t launch_colmax(const double *Y, int ldt, int64_t m, int nrhs, double *part, int64_t part_cap, double *out,
                         hipStream_t st)
{
    const int nblk = COLSQ_BLOCKS;
    if ((int64_t)nblk * nrhs > part_cap) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_colmax_part, dim3(nblk), dim3(256), 0, st, Y, ldt, m, nrhs, part);
    hipLaunchKernelGGL(k_colmax_sum, dim3(1), dim3(64), 0, st, part, nblk, nrhs, out);
    return hipGetLastError();
}

hipError_t launch_norm_inf(const double *A, int64_t lda, int64_t m, int64_t n, double *part, int64_t part_cap,
                           double *out, hipStream_t st)
{
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t rowblk = (m + 255) / 256;
    int64_t nslice = std::max<int64_t>(1, std::min<int64_t>((n + 63) / 64, 4096 / rowblk + 1));
    nslice = std::min<int64_t>(nslice, (part_cap - COLSQ_BLOCKS) / m);
    if (nslice < 1) return hipErrorInvalidValue;
    const int64_t cps = (n + nslice - 1) / nslice;
    nslice = (n + cps - 1) / cps;
    double *part2 = part + nslice * m;
    hipLaunchKernelGGL(k_absrow_part, dim3((unsigned)rowblk, (unsigned)nslice), dim3(256), 0, st, A, lda, m, n,
                       cps, part);
    hipLaunchKernelGGL(k_absrow_max, dim3(COLSQ_BLOCKS), dim3(256), 0, st, part, (int)nslice, m, part2);
    hipLaunchKernelGGL(k_colmax_sum, dim3(1), dim3(64), 0, st, part2, COLSQ_BLOCKS, 1, out);
    return hipGetLastError();
}

hipError_t launch_fill_normal(double *Y, int ldt, int64_t rows, int cols, uint64_t seed, hipStream_t st)
{
    const int64_t total = rows * ldt;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill_normal, dim3((unsigned)blocks), dim3(256), 0, st, Y, ldt, rows, cols, seed);
    return hipGetLastError();
}

hipError_t launch_trmm(int nb, const double *tiles, int p, int64_t n, double *W, const double *Z, int ldt,
                       hipStream_t st)
{
    const int q = (int)((n + nb - 1) / nb);
    const dim3 grid((unsigned)p, (unsigned)(ldt / SW));
    // Row blocks i >= q (below R) hold zeros: the loop over j >= i is empty.
    if (nb == 64) hipLaunchKernelGGL(k_trmm<64>, grid, dim3(128), 0, st, tiles, p, q, W, Z, ldt);
    else if (nb == 128) hipLaunchKernelGGL(k_trmm<128>, grid, dim3(256), 0, st, tiles, p, q, W, Z, ldt);
    else if (nb == 256) hipLaunchKernelGGL(k_trmm<256>, grid, dim3(512), 0, st, tiles, p, q, W, Z, ldt);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_axpy_rows(const double *X, double *Y, int ldt, int64_t m, int nrhs, int op, hipStream_t st)
{
    const int64_t total = m * nrhs;
    if (total <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_axpy_rows, dim3((unsigned)blocks), dim3(256), 0, st, X, Y, ldt, m, nrhs, op);
    return hipGetLastError();
}

}  // namespace tq
