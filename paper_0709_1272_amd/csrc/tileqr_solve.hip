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
// by row blocks of RB = 64 rows (a tile holds nb / 64 of them), one
// workgroup of four waves per row block r (and strip, blockIdx.y):
//   upper == true:  R X = C,   X_r = R_rr^{-1} (C_r - sum_{c > r} R_rc X_c)
//   upper == false: R^T X = C, X_r = R_rr^{-T} (C_r - sum_{c < r} R_cr^T X_c)
// The workgroup applies each solved block X_c as soon as its workgroup
// publishes it (progress flags, FLAG_STRIDE words apart): op(R)_rc X_c is a
// 64 x 64 by 64 x 32 product on v_mfma_f64_16x16x4_f64, wave w owning rows
// 16 w .. 16 w + 15.  The K index of chunk kk and lane group g is 16 g + kk,
// so that a lane's A operands for the 16 chunks are 16 consecutive entries
// of one row of R (upper) and are loaded before the wait (R is final).
// The diagonal block is then solved by substitution (backward for R,
// forward for R^T), each wave taking 8 right-hand sides with 8 lanes per
// right-hand side holding 8 rows each: per block of 8 rows the owning lane
// solves its triangle locally, its 8 values go to the column's other lanes
// by shuffles, and they update their rows.  Producers have the lower
// workgroup indices (for R the last block comes first), so every wait is on
// a workgroup that was dispatched earlier; every wait is bounded
// (STATUS_TIMEOUT).  Rows at or beyond `n` (padding) get X = 0; an exact
// zero on the diagonal of a real row sets STATUS_SINGULAR.
constexpr int RB = 64;
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int NB>
__global__ __launch_bounds__(256) void k_trsm(const double *tiles, int p, int nrb, int64_t n, double *C, int ldt,
                                              int upper, int *flags, int *status, int64_t spin_limit)
{
    __shared__ double Xs[RB][SW + 1];
    __shared__ double Rd[RB][RB + 1];
    __shared__ double dinv[RB];
    __shared__ int s_abort;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, ln = lane & 15, g = lane >> 4;
    const int strip = blockIdx.y, nstrip = gridDim.y, s0 = strip * SW;
    const int r = upper ? nrb - 1 - (int)blockIdx.x : (int)blockIdx.x;
    const int rt = r * RB / NB, ro = r * RB % NB;

    // The diagonal block as the triangle solved with: Rd = op(R)_rr.
    {
        const double *Rt = tile_at(tiles, p, NB, rt, rt);
        if (upper)
            batched_copy<RB * RB / 256>(tid, 256, [&](int e) { return Rt[(size_t)(ro + e / RB) * NB + ro + e % RB]; },
                                        [&](int e, double v) { Rd[e / RB][e % RB] = v; });
        else
            batched_copy<RB * RB / 256>(tid, 256, [&](int e) { return Rt[(size_t)(ro + e / RB) * NB + ro + e % RB]; },
                                        [&](int e, double v) { Rd[e % RB][e / RB] = v; });
        __syncthreads();
        if (tid < RB) {
            const double d = Rd[tid][tid];
            const bool real = (int64_t)r * RB + tid < n;
            if (real && d == 0.0) atomicOr(status, STATUS_SINGULAR);
            dinv[tid] = (real && d != 0.0) ? 1.0 / d : 0.0;
        }
    }

    // This block's right-hand sides, read before the first wait (only this
    // workgroup writes them, with the solution, at the end).
    double *Cr = C + (size_t)r * RB * ldt;
    double crv[2][4];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) crv[cb][e] = Cr[(size_t)(16 * w + 4 * e + g) * ldt + s0 + 16 * cb + ln];

    d4 acc[2] = {};   // element e: row 16 w + 4 e + g, column 16 cb + ln
    const int nc = upper ? nrb - 1 - r : r;
    for (int u = 0; u < nc; ++u) {
        const int c = upper ? nrb - 1 - u : u;
        const int ct = c * RB / NB, co = c * RB % NB;
        double a[16];
        if (upper) {
            const double *Rb = tile_at(tiles, p, NB, rt, ct) + (size_t)(ro + 16 * w + ln) * NB + co + 16 * g;
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) a[kk] = Rb[kk];
        } else {
            const double *Rb = tile_at(tiles, p, NB, ct, rt) + (size_t)(co + 16 * g) * NB + ro + 16 * w + ln;
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) a[kk] = Rb[(size_t)kk * NB];
        }
        if (tid == 0) {
            const int *flag = &flags[(c * nstrip + strip) * FLAG_STRIDE];
            // The block solved just before this one is on the critical path:
            // poll it without backing off.
            const bool next = upper ? c == r + 1 : c == r - 1;
            int abort = 0, backoff = 0;
            int64_t spins = 0;
            while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & STATUS_TIMEOUT ||
                    ++spins > spin_limit) {
                    __hip_atomic_fetch_or(status, STATUS_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    abort = 1;
                    break;
                }
                if (next) {
                    __builtin_amdgcn_s_sleep(1);
                } else {
                    backoff = backoff < 5 ? backoff + 1 : 5;
                    for (int z = 0; z < (1 << backoff); ++z) __builtin_amdgcn_s_sleep(2);
                }
            }
            // Acquire before the barrier: the other waves read X_c after it.
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_abort = abort;
        }
        __syncthreads();
        if (s_abort) return;
        const double *Cc = C + (size_t)c * RB * ldt;
        batched_copy<RB * SW / 256>(tid, 256, [&](int e) { return Cc[(size_t)(e / SW) * ldt + s0 + e % SW]; },
                                    [&](int e, double v) { Xs[e / SW][e % SW] = v; });
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) acc[cb] = mfma_f64(a[kk], Xs[16 * g + kk][16 * cb + ln], acc[cb]);
        __syncthreads();
    }

    // Y = C_r - accumulated products, in Xs.
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) Xs[16 * w + 4 * e + g][16 * cb + ln] = crv[cb][e] - acc[cb][e];
    __syncthreads();

    // Substitution with op(R)_rr: lane (cl, part) of wave w holds rows
    // 8 part .. 8 part + 7 of right-hand side 8 w + cl.
    const int cl = lane >> 3, part = lane & 7, col = 8 * w + cl;
    double y[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) y[e] = Xs[8 * part + e][col];
#pragma unroll 1
    for (int bb = 0; bb < 8; ++bb) {
        const int pb = upper ? 7 - bb : bb;
        // The owning lane solves the 8 x 8 triangle of block pb (every lane
        // runs the same steps on its own rows; only the owner's are used).
        double z[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) z[e] = y[e];
        if (upper) {
#pragma unroll
            for (int e = 7; e >= 0; --e) {
                z[e] *= dinv[8 * pb + e];
#pragma unroll
                for (int f = 0; f < e; ++f) z[f] -= Rd[8 * pb + f][8 * pb + e] * z[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                z[e] *= dinv[8 * pb + e];
#pragma unroll
                for (int f = e + 1; f < 8; ++f) z[f] -= Rd[8 * pb + f][8 * pb + e] * z[e];
            }
        }
        double x[8];
        const int owner = (lane & ~7) | pb;
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = __shfl(z[e], owner, 64);
        if (part == pb) {
#pragma unroll
            for (int e = 0; e < 8; ++e) y[e] = x[e];
        } else if (upper ? part < pb : part > pb) {
#pragma unroll
            for (int f = 0; f < 8; ++f) {
                double s = y[f];
#pragma unroll
                for (int e = 0; e < 8; ++e) s -= Rd[8 * part + f][8 * pb + e] * x[e];
                y[f] = s;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int row = 8 * part + e;
        Cr[(size_t)row * ldt + s0 + col] = (int64_t)r * RB + row < n ? y[e] : 0.0;
    }
    // Publish X_r: every wave waits for its stores, then one writes back
    // and raises the flag.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&flags[(r * nstrip + strip) * FLAG_STRIDE], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Y (row-major rows, leading dimension ldt, m x nrhs) <- alpha A X + beta Y
// for column-major A (m x n, lda) and X in row blocks (n x nrhs, ldt): a
// product with 16 or 32 columns, on v_mfma_f64_16x16x4_f64.  Each wave
// forms one 16-row tile over a slice of the columns of A (workgroup of four
// waves: 64 rows); the K index of chunk kk and lane group g is 16 g + kk, so
// that for each chunk the 16 lanes of a group read 16 consecutive rows of
// one column of A (128 bytes).  A is read once.  The per-slice partial sums
// go to `part` and are added in slice order by a second pass
// (deterministic).
template <int NV>
__global__ __launch_bounds__(256) void k_gemv_n_part(const double *A, int64_t lda, int64_t m, int64_t n,
                                                     const double *X, int ldt, int nr, int64_t cols_per_slice,
                                                     double *part)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, ln = lane & 15, g = lane >> 4;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + w) * 16;
    if (row0 >= m) return;
    const int64_t row = row0 + ln;
    const bool rin = row < m;
    const double *Ar = A + (rin ? row : m - 1);
    const int64_t c0 = (int64_t)blockIdx.y * cols_per_slice, c1 = std::min<int64_t>(n, c0 + cols_per_slice);
    d4 acc[NV] = {};
    for (int64_t kb = c0; kb < c1; kb += 64) {
        double a[16], b[NV][16];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int64_t k = kb + 16 * g + kk;
            const bool kin = k < c1;
            a[kk] = (kin && rin) ? Ar[k * lda] : 0.0;
#pragma unroll
            for (int cb = 0; cb < NV; ++cb) b[cb][kk] = kin ? X[k * ldt + 16 * cb + ln] : 0.0;
        }
#pragma unroll
        for (int kk = 0; kk < 16; ++kk)
#pragma unroll
            for (int cb = 0; cb < NV; ++cb) acc[cb] = mfma_f64(a[kk], b[cb][kk], acc[cb]);
    }
    // Element e of acc[cb]: row row0 + 4 e + g, column 16 cb + ln.
#pragma unroll
    for (int cb = 0; cb < NV; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t rr = row0 + 4 * e + g;
            const int v = 16 * cb + ln;
            if (rr < m && v < nr) part[((int64_t)blockIdx.y * m + rr) * SW + v] = acc[cb][e];
        }
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

// Y (n x nrhs rows) <- alpha A^T R + beta Y, on v_mfma_f64_16x16x4_f64.
// Workgroup (x, y) takes 64 columns of A and a slice of its rows: per chunk
// of 64 rows the 64 x 64 block of A is staged in LDS (read once, coalesced
// down its columns) and wave w forms the 16 x (16 NV) tile of columns
// 16 w .. 16 w + 15 (A^T as the left operand from LDS, R from memory, the K
// index of chunk kk and lane group g is 16 g + kk).  The per-slice partial
// sums go to `part` and a second pass adds them in slice order
// (deterministic).
template <int NV>
__global__ __launch_bounds__(256) void k_gemv_t_part(const double *A, int64_t lda, int64_t m, int64_t n,
                                                     const double *Rv, int ldt, int nr, int64_t rows_per_slice,
                                                     double *part)
{
    __shared__ double as[64][66];   // as[column][row]
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, ln = lane & 15, g = lane >> 4;
    const int64_t c0 = (int64_t)blockIdx.x * 64;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_slice, r1 = std::min<int64_t>(m, r0 + rows_per_slice);
    d4 acc[NV] = {};
    for (int64_t rb = r0; rb < r1; rb += 64) {
        __syncthreads();
        batched_copy<64 * 64 / 256>(tid, 256,
                                    [&](int e) {
                                        const int64_t row = rb + e % 64, col = c0 + e / 64;
                                        return (row < r1 && col < n) ? A[col * lda + row] : 0.0;
                                    },
                                    [&](int e, double v) { as[e / 64][e % 64] = v; });
        double b[NV][16];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const int64_t row = rb + 16 * g + kk;
#pragma unroll
            for (int cb = 0; cb < NV; ++cb) b[cb][kk] = row < r1 ? Rv[row * ldt + 16 * cb + ln] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const double a = as[16 * w + ln][16 * g + kk];
#pragma unroll
            for (int cb = 0; cb < NV; ++cb) acc[cb] = mfma_f64(a, b[cb][kk], acc[cb]);
        }
    }
    // Element e of acc[cb]: column c0 + 16 w + 4 e + g of A, right-hand side 16 cb + ln.
#pragma unroll
    for (int cb = 0; cb < NV; ++cb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t col = c0 + 16 * w + 4 * e + g;
            const int v = 16 * cb + ln;
            if (col < n && v < nr) part[((int64_t)blockIdx.y * n + col) * SW + v] = acc[cb][e];
        }
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
    // Eight rows per thread and pass, in eight partial sums, so that eight
    // loads are in flight together; the sums are added in a fixed order.
    double s8[8] = {};
    for (int64_t c = blockIdx.x; c < n; c += gridDim.x)
        for (int64_t r0 = threadIdx.x; r0 < m; r0 += 256 * 8) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = r0 + 256 * u < m ? A[c * lda + r0 + 256 * u] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) s8[u] += a[u] * a[u];
        }
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += s8[u];
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
            // Unrolled by 8 only: fully unrolled, the compiler hoists all 32
            // steps' LDS reads ahead of the products and spills.
#pragma unroll 8
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
    const int nrb = (int)((n + RB - 1) / RB);
    const int nstrip = ldt / SW;
    hipLaunchKernelGGL(k_fill_flags, dim3((unsigned)std::max(1, std::min(1024, (nrb * nstrip + 255) / 256))),
                       dim3(256), 0, st, flags, nrb * nstrip);
    hipLaunchKernelGGL(k_trsm<NB>, dim3(nrb, nstrip), dim3(256), 0, st, tiles, p, nrb, n, C, ldt, upper ? 1 : 0,
                       flags, status, spin_limit);
    return hipGetLastError();
}

int64_t trsm_flags_needed(int64_t n, int ldt) { return (n + RB - 1) / RB * (ldt / SW) * FLAG_STRIDE; }

hipError_t launch_trsm(int nb, const double *tiles, int p, int64_t n, double *C, int ldt, bool upper, int *flags,
                       int64_t flags_cap, int *status, int64_t spin_limit, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (trsm_flags_needed(n, ldt) > flags_cap) return hipErrorInvalidValue;
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
        const int64_t rowblk = (m + 63) / 64;
        // About 8192 waves in flight: slices of the columns when the rows alone give fewer.
        int64_t nslice = std::max<int64_t>(1, std::min<int64_t>((n + 63) / 64, 2048 / rowblk));
        nslice = std::min<int64_t>(nslice, std::max<int64_t>(1, part_cap / (m * SW)));
        const int64_t cps = ((n + nslice - 1) / nslice + 63) / 64 * 64;
        nslice = std::max<int64_t>(1, (n + cps - 1) / cps);
        if (nr <= 16)
            hipLaunchKernelGGL(k_gemv_n_part<1>, dim3((unsigned)rowblk, (unsigned)nslice), dim3(256), 0, st, A, lda,
                               m, n, X + v0, ldt, nr, cps, part);
        else
            hipLaunchKernelGGL(k_gemv_n_part<2>, dim3((unsigned)rowblk, (unsigned)nslice), dim3(256), 0, st, A, lda,
                               m, n, X + v0, ldt, nr, cps, part);
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
        if (nr <= 16)
            hipLaunchKernelGGL(k_gemv_t_part<1>, dim3((unsigned)colblk, (unsigned)nslice), dim3(256), 0, st, A, lda,
                               m, n, R + v0, ldt, nr, rps, part);
        else
            hipLaunchKernelGGL(k_gemv_t_part<2>, dim3((unsigned)colblk, (unsigned)nslice), dim3(256), 0, st, A, lda,
                               m, n, R + v0, ldt, nr, rps, part);
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
