// Tiled LU factorisation with tiled pairwise pivoting (Section 3.2.2,
// Algorithm 3, inner blocking of Section 3.2.3) on gfx950: nb x nb tiles,
// row-major inside (the layout of the QR tiles), and the DAG of GETRF /
// GESSM / TSTRF / SSSSM tasks run by a persistent kernel with per-task
// dependency counters and ready queues in HBM (Section 4).
//
// One workgroup of four wave64s runs one task, with its tiles in LDS:
//   GETRF(k)      partial pivoting column by column: the pivot by a
//                 wave-wide (magnitude, index) reduction, the exchange of
//                 whole tile rows, the multipliers and the rank-1 update;
//   GESSM(k, j)   the exchanges of GETRF, then L_kk^{-1} by forward
//                 substitution, one column of A_kj per thread;
//   TSTRF(k, i)   [U_kk; A_ik] by inner panels of ib columns: per column the
//                 pivot among U_kk's diagonal entry and A_ik's column, the
//                 exchange of U's row with an A row from the column on (the
//                 A row's multipliers of the panel's earlier columns moving
//                 to L_up), the multipliers and the update of the panel's
//                 later columns; after the panel, the columns right of it:
//                 U's panel rows by L_up, then A_ik by the multipliers;
//   SSSSM(k, i, j) panel by panel: the exchanges between A_kj and A_ij rows,
//                 A_kj's panel rows by L_up, then A_ij -= L_ik A_kj[panel]
//                 on FP64 MFMA.
// Every task's arithmetic is fixed by its inputs (pivot choices included:
// the reductions take the largest magnitude and, among equal ones, the first
// candidate), so the DAG result is bitwise the one of Algorithm 3's loop
// order, whatever order the tasks run in.
#include "tileqr_host.h"
#include "../../include/tilelu.h"

#include <algorithm>
#include <climits>
#include <random>
#include <vector>

using namespace tq;

namespace tl {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NB = 64;         // tile size
constexpr int NT = 256;        // threads per workgroup
constexpr int LD = NB + 2;     // LDS row stride (MFMA operand loads conflict-free)
constexpr int NXQ = 8;         // XCDs (queues of the update levels)
constexpr int QSTRIDE = 64;    // words between queue heads / tails
constexpr int NQ = 2 + 2 * NXQ;
enum { T_GETRF = 0, T_GESSM = 1, T_TSTRF = 2, T_SSSSM = 3 };
enum { ST_NONFINITE = 1, ST_TIMEOUT = 2, ST_SINGULAR = 4 };

struct Sched {
    double *tiles;
    double *lup;               // p * p * ib * NB
    int32_t *piv;              // p * p * NB
    int32_t p, ib;
    int32_t *counters;
    int32_t *qslot;
    int64_t qoff[NQ];
    uint32_t *qctl;
    uint32_t *done;
    int64_t total_ids, total_tasks, nslot;
    int32_t *status;
    int32_t *minor;
    int64_t spin_limit;
    int32_t shuffle;
    uint64_t seed;
};

struct LTask {
    int type, k, i, j;
};

// Dense ids: GETRF(k) = k; GESSM(k, j) = p + k p + j; TSTRF(k, i) =
// p + p^2 + k p + i; SSSSM(k, i, j) = p + 2 p^2 + (k p + i) p + j.
__host__ __device__ inline int64_t id_getrf(int p, int k) { (void)p; return k; }
__host__ __device__ inline int64_t id_gessm(int p, int k, int j) { return (int64_t)p + (int64_t)k * p + j; }
__host__ __device__ inline int64_t id_tstrf(int p, int k, int i)
{
    return (int64_t)p + (int64_t)p * p + (int64_t)k * p + i;
}
__host__ __device__ inline int64_t id_ssssm(int p, int k, int i, int j)
{
    return (int64_t)p + 2 * (int64_t)p * p + ((int64_t)k * p + i) * p + j;
}

__host__ __device__ inline LTask decode(int p, int64_t id)
{
    LTask t{0, 0, 0, 0};
    const int64_t pp = (int64_t)p * p;
    if (id < p) {
        t.type = T_GETRF;
        t.k = t.i = t.j = (int)id;
    } else if (id < p + pp) {
        const int64_t r = id - p;
        t.type = T_GESSM;
        t.k = t.i = (int)(r / p);
        t.j = (int)(r % p);
    } else if (id < p + 2 * pp) {
        const int64_t r = id - p - pp;
        t.type = T_TSTRF;
        t.k = t.j = (int)(r / p);
        t.i = (int)(r % p);
    } else {
        int64_t r = id - p - 2 * pp;
        t.type = T_SSSSM;
        t.j = (int)(r % p);
        r /= p;
        t.i = (int)(r % p);
        t.k = (int)(r / p);
    }
    return t;
}

__host__ __device__ inline bool valid(int p, const LTask &t)
{
    if (t.type == T_GETRF) return t.k < p;
    if (t.type == T_GESSM) return t.k < t.j && t.j < p;
    if (t.type == T_TSTRF) return t.k < t.i && t.i < p;
    return t.k < t.i && t.i < p && t.k < t.j && t.j < p;
}

__host__ __device__ inline int indegree(const LTask &t)
{
    const int prev = t.k > 0 ? 1 : 0;   // the step k-1 update of the same tile
    if (t.type == T_GETRF) return prev;
    if (t.type == T_GESSM) return 1 + prev;   // GETRF(k)
    if (t.type == T_TSTRF) return 1 + prev;   // GETRF(k) or TSTRF(k, i-1): U_kk
    return 2 + prev;                          // TSTRF(k, i); GESSM(k, j) or SSSSM(k, i-1, j): A_kj
}

// The consumer in step k+1 of tile (i, j), i, j > k.
__host__ __device__ inline int64_t next_step(int p, int k, int i, int j)
{
    const int k1 = k + 1;
    if (i == k1 && j == k1) return id_getrf(p, k1);
    if (i == k1) return id_gessm(p, k1, j);
    if (j == k1) return id_tstrf(p, k1, i);
    return id_ssssm(p, k1, i, j);
}

__host__ __device__ inline int nsucc(int p, const LTask &t)
{
    const int more = t.i + 1 < p ? 1 : 0;
    if (t.type == T_GETRF) return (p - t.k - 1) + (t.k + 1 < p ? 1 : 0);
    if (t.type == T_GESSM) return t.k + 1 < p ? 1 : 0;
    if (t.type == T_TSTRF) return (p - t.k - 1) + more;
    return 1 + more;
}

__host__ __device__ inline int64_t succ(int p, const LTask &t, int n)
{
    if (t.type == T_GETRF) return n < p - t.k - 1 ? id_gessm(p, t.k, t.k + 1 + n) : id_tstrf(p, t.k, t.k + 1);
    if (t.type == T_GESSM) return id_ssssm(p, t.k, t.k + 1, t.j);
    if (t.type == T_TSTRF) return n < p - t.k - 1 ? id_ssssm(p, t.k, t.i, t.k + 1 + n) : id_tstrf(p, t.k, t.i + 1);
    // SSSSM(k, i, j): the next step's consumer of (i, j), then SSSSM(k, i+1, j).
    return n == 0 ? next_step(p, t.k, t.i, t.j) : id_ssssm(p, t.k, t.i + 1, t.j);
}

// Queues: GETRF and TSTRF (the panel chain), GESSM, then per XCD the SSSSM
// of column k+1 (they feed the next step's panel) and the other SSSSM.
__host__ __device__ inline int level_of(const LTask &t)
{
    if (t.type == T_GETRF || t.type == T_TSTRF) return 0;
    if (t.type == T_GESSM) return 1;
    return t.j == t.k + 1 ? 2 : 3;
}
__host__ __device__ inline int queue_of(const LTask &t)
{
    const int lv = level_of(t);
    return lv < 2 ? lv : 2 + (lv - 2) * NXQ + t.j % NXQ;
}

int64_t count_tasks(int64_t p, int64_t *c)
{
    const int64_t c0 = p, c1 = p * (p - 1) / 2, c2 = c1, c3 = (p - 1) * p * (2 * p - 1) / 6;
    if (c) {
        c[0] = c0;
        c[1] = c1;
        c[2] = c2;
        c[3] = c3;
    }
    return c0 + c1 + c2 + c3;
}

// ------------------------------------------------------------ tile kernels

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    // D = A B + C on 16 x 16 x 4 FP64 blocks: lane L (n = L % 16, g = L / 16)
    // supplies A[n][g] and B[g][n] and holds D[4 r + g][n] in element r.
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct Smem {
    double X[NB][LD];          // GETRF / GESSM: the tile; TSTRF: U_kk; SSSSM: A_kj
    double Y[NB][LD];          // GESSM: L_kk; TSTRF: A_ik; SSSSM: A_ij
    double Z[NB][LD];          // SSSSM: the multipliers L_ik
    double Lup[32][NB];        // TSTRF / SSSSM: L_up of the tile
    int32_t piv[NB];
    int32_t pick;              // the chosen pivot (-1: U's row)
    int32_t fail;
};

__device__ __forceinline__ double *tile_at(const Sched &S, int i, int j)
{
    return S.tiles + ((size_t)j * S.p + i) * (size_t)(NB * NB);
}

__device__ __forceinline__ void load_tile(double (*X)[LD], const double *T)
{
    for (int e = threadIdx.x; e < NB * NB; e += NT) X[e / NB][e % NB] = T[e];
}
__device__ __forceinline__ void store_tile(double *T, const double (*X)[LD])
{
    for (int e = threadIdx.x; e < NB * NB; e += NT) T[e] = X[e / NB][e % NB];
}

// Largest |v| and, among equal magnitudes, the smallest index, over the 64
// lanes of a wave (lanes with v < 0 take no part).  Every lane gets the
// result.
__device__ __forceinline__ void wave_argmax(double &v, int &idx)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oi = __shfl_xor(idx, off, 64);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
}

__device__ __forceinline__ void fail_column(const Sched &S, int col)
{
    __hip_atomic_fetch_or(S.status, ST_SINGULAR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_min(S.minor, col + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// GETRF(k): partial pivoting of the diagonal tile, column by column on wave
// 0 (the tile has as many rows as the wave has lanes): the pivot by a
// wave-wide reduction, the exchange with one lane per column, the
// multipliers and the rank-1 update with one lane per row.  Only wave-level
// ordering between the phases; the other waves wait at the end.
__device__ void task_getrf(Smem &sm, const Sched &S, int k)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double *T = tile_at(S, k, k);
    load_tile(sm.X, T);
    if (tid == 0) sm.fail = 0;
    __syncthreads();
    if (w == 0) {
        for (int j = 0; j < NB; ++j) {
            double v = lane >= j ? fabs(sm.X[lane][j]) : -1.0;
            int idx = lane;
            wave_argmax(v, idx);
            if (v == 0.0) {
                if (lane == 0) {
                    sm.fail = 1;
                    fail_column(S, k * NB + j);
                }
                break;
            }
            if (lane == 0) sm.piv[j] = idx;
            if (idx != j) {
                const double a = sm.X[j][lane], b = sm.X[idx][lane];
                sm.X[j][lane] = b;
                sm.X[idx][lane] = a;
            }
            wave_sync();
            if (lane > j) {
                const double l = sm.X[lane][j] / sm.X[j][j];
                sm.X[lane][j] = l;
                for (int c = j + 1; c < NB; ++c) sm.X[lane][c] = sm.X[lane][c] - l * sm.X[j][c];
            }
            wave_sync();
        }
    }
    __syncthreads();
    if (sm.fail) return;
    store_tile(T, sm.X);
    int32_t *pv = S.piv + ((size_t)k * S.p + k) * NB;
    if (tid < NB) pv[tid] = sm.piv[tid];
}

// GESSM(k, j): A_kj <- L_kk^{-1} P_kk A_kj.
__device__ void task_gessm(Smem &sm, const Sched &S, int k, int j)
{
    const int tid = threadIdx.x;
    double *T = tile_at(S, k, j);
    load_tile(sm.X, T);
    // L_kk only (the strictly lower part; the TSTRF chain may be rewriting
    // the upper triangle of the same tile meanwhile).
    const double *Tk = tile_at(S, k, k);
    for (int e = tid; e < NB * NB; e += NT) {
        const int r = e / NB, c = e % NB;
        sm.Y[r][c] = r > c ? Tk[e] : 0.0;
    }
    const int32_t *pv = S.piv + ((size_t)k * S.p + k) * NB;
    if (tid < NB) sm.piv[tid] = pv[tid];
    __syncthreads();
    if (tid < NB) {
        const int c = tid;
        for (int q = 0; q < NB; ++q) {
            const int pr = sm.piv[q];
            if (pr != q) {
                const double t = sm.X[q][c];
                sm.X[q][c] = sm.X[pr][c];
                sm.X[pr][c] = t;
            }
        }
        for (int r = 1; r < NB; ++r) {
            double s = sm.X[r][c];
            for (int q = 0; q < r; ++q) s -= sm.Y[r][q] * sm.X[q][c];
            sm.X[r][c] = s;
        }
    }
    __syncthreads();
    store_tile(T, sm.X);
}

// TSTRF(k, i): [U_kk; A_ik] by inner panels of ib columns.
__device__ void task_tstrf(Smem &sm, const Sched &S, int k, int i)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int ib = S.ib;
    double *U = tile_at(S, k, k), *A = tile_at(S, i, k);
    // U_kk's upper triangle (the strictly lower part, L_kk, stays in memory
    // untouched); A_ik whole.
    for (int e = tid; e < NB * NB; e += NT) {
        const int r = e / NB, c = e % NB;
        sm.X[r][c] = r <= c ? U[e] : 0.0;
        sm.Y[r][c] = A[e];
    }
    for (int e = tid; e < 32 * NB; e += NT) sm.Lup[e / NB][e % NB] = 0.0;
    if (tid == 0) sm.fail = 0;
    __syncthreads();
    for (int l0 = 0; l0 < NB; l0 += ib) {
        const int l1 = l0 + ib;
        // The panel's columns on wave 0: lane r owns row r of A_ik for the
        // multipliers and the updates, lane c column c for the exchange.
        if (w == 0) {
            for (int j = l0; j < l1; ++j) {
                double v = fabs(sm.Y[lane][j]);
                int idx = lane;
                wave_argmax(v, idx);
                const double u = fabs(sm.X[j][j]);
                const int pick = v > u ? idx : -1;
                if (pick < 0 && u == 0.0) {
                    if (lane == 0) {
                        sm.fail = 1;
                        fail_column(S, k * NB + j);
                    }
                    break;
                }
                if (lane == 0) sm.piv[j] = pick >= 0 ? NB + pick : j;
                if (pick >= 0) {
                    const int c = lane;
                    if (c >= j) {
                        const double t = sm.X[j][c];
                        sm.X[j][c] = sm.Y[pick][c];
                        sm.Y[pick][c] = t;
                    } else if (c >= l0) {
                        sm.Lup[j - l0][c] = sm.Y[pick][c];
                        sm.Y[pick][c] = 0.0;
                    }
                }
                wave_sync();
                const double l = sm.Y[lane][j] / sm.X[j][j];
                sm.Y[lane][j] = l;
                for (int c = j + 1; c < l1; ++c) sm.Y[lane][c] = sm.Y[lane][c] - l * sm.X[j][c];
                wave_sync();
            }
        }
        __syncthreads();
        if (sm.fail) return;
        // Columns right of the panel: U's panel rows by L_up (one column per
        // thread), then A_ik by its multipliers.
        if (tid >= l1 && tid < NB) {
            const int c = tid;
            for (int r = l0; r < l1; ++r) {
                double s = sm.X[r][c];
                for (int q = l0; q < r; ++q) s -= sm.Lup[r - l0][q] * sm.X[q][c];
                sm.X[r][c] = s;
            }
        }
        __syncthreads();
        const int mc = NB - l1;
        for (int e = tid; e < NB * mc; e += NT) {
            const int r = e / mc, c = l1 + e % mc;
            double s = sm.Y[r][c];
            for (int q = l0; q < l1; ++q) s -= sm.Y[r][q] * sm.X[q][c];
            sm.Y[r][c] = s;
        }
        __syncthreads();
    }
    for (int e = tid; e < NB * NB; e += NT) {
        const int r = e / NB, c = e % NB;
        if (r <= c) U[e] = sm.X[r][c];
        A[e] = sm.Y[r][c];
    }
    double *lup = S.lup + ((size_t)k * S.p + i) * (size_t)ib * NB;
    for (int e = tid; e < ib * NB; e += NT) lup[e] = sm.Lup[e / NB][e % NB];
    int32_t *pv = S.piv + ((size_t)k * S.p + i) * NB;
    if (tid < NB) pv[tid] = sm.piv[tid];
}

// SSSSM(k, i, j): [A_kj; A_ij] <- L_ik^{-1} P_ik [A_kj; A_ij], by panels.
__device__ void task_ssssm(Smem &sm, const Sched &S, int k, int i, int j)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, n = lane & 15, g = lane >> 4;
    const int ib = S.ib;
    double *X1 = tile_at(S, k, j), *X2 = tile_at(S, i, j);
    load_tile(sm.X, X1);
    load_tile(sm.Y, X2);
    load_tile(sm.Z, tile_at(S, i, k));
    const double *lup = S.lup + ((size_t)k * S.p + i) * (size_t)ib * NB;
    for (int e = tid; e < ib * NB; e += NT) sm.Lup[e / NB][e % NB] = lup[e];
    const int32_t *pv = S.piv + ((size_t)k * S.p + i) * NB;
    if (tid < NB) sm.piv[tid] = pv[tid];
    __syncthreads();
    for (int l0 = 0; l0 < NB; l0 += ib) {
        const int l1 = l0 + ib;
        if (tid < NB) {
            const int c = tid;
            for (int q = l0; q < l1; ++q) {
                const int pq = sm.piv[q];
                if (pq >= NB) {
                    const double t = sm.X[q][c];
                    sm.X[q][c] = sm.Y[pq - NB][c];
                    sm.Y[pq - NB][c] = t;
                }
            }
            for (int r = l0; r < l1; ++r) {
                double s = sm.X[r][c];
                for (int q = l0; q < r; ++q) s -= sm.Lup[r - l0][q] * sm.X[q][c];
                sm.X[r][c] = s;
            }
        }
        __syncthreads();
        // A_ij -= L_ik[:, panel] A_kj[panel, :]: 16 blocks of 16 x 16, four
        // per wave, K = ib in steps of 4.
        for (int blk = w; blk < 16; blk += 4) {
            const int rb = blk >> 2, cb = blk & 3;
            d4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = sm.Y[16 * rb + 4 * r + g][16 * cb + n];
            for (int ks = l0 / 4; ks < l1 / 4; ++ks)
                acc = mfma(-sm.Z[16 * rb + n][4 * ks + g], sm.X[4 * ks + g][16 * cb + n], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.Y[16 * rb + 4 * r + g][16 * cb + n] = acc[r];
        }
        __syncthreads();
    }
    store_tile(X1, sm.X);
    store_tile(X2, sm.Y);
}

__device__ __forceinline__ void run_task(Smem &sm, const Sched &S, const LTask &t)
{
    if (t.type == T_GETRF) task_getrf(sm, S, t.k);
    else if (t.type == T_GESSM) task_gessm(sm, S, t.k, t.j);
    else if (t.type == T_TSTRF) task_tstrf(sm, S, t.k, t.i);
    else task_ssssm(sm, S, t.k, t.i, t.j);
}

// ------------------------------------------------------------- scheduler

__device__ __forceinline__ uint32_t ld_rlx(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void push(const Sched &S, int q, int64_t id)
{
    const uint32_t slot = __hip_atomic_fetch_add(&S.qctl[(NQ + q) * QSTRIDE], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&S.qslot[S.qoff[q] + slot], (int32_t)(id + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t pop(const Sched &S, int q)
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        const uint32_t t = ld_rlx(&S.qctl[(NQ + q) * QSTRIDE]);
        const uint32_t h = ld_rlx(&S.qctl[q * QSTRIDE]);
        if (h >= t) return -1;
        const int32_t v = __hip_atomic_load(&S.qslot[S.qoff[q] + h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v == 0) return -1;
        uint32_t expect = h;
        if (__hip_atomic_compare_exchange_strong(&S.qctl[q * QSTRIDE], &expect, h + 1, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return (int64_t)v - 1;
    }
    return -1;
}

__device__ __forceinline__ int xcd_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (NXQ - 1); }

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}

// Queues of levels up to maxlv in priority order (with shuffle, levels 0
// and 1 swapped now and then); the update levels of this XCD, and with
// `steal` of the others after it in a rotation taken modulo before the
// conversion (never negative).
__device__ __forceinline__ int64_t pop_upto(const Sched &S, int maxlv, int xcd, bool steal, uint64_t pick)
{
    int64_t id = -1;
    if (S.shuffle && (pick & 1) && maxlv >= 1) {
        if ((id = pop(S, 1)) >= 0) return id;
        if ((id = pop(S, 0)) >= 0) return id;
    } else {
        if ((id = pop(S, 0)) >= 0) return id;
        if (maxlv >= 1 && (id = pop(S, 1)) >= 0) return id;
    }
    const int rot = (int)((pick >> 8) % NXQ);
    for (int lv = 2; lv <= maxlv; ++lv) {
        const int base = 2 + (lv - 2) * NXQ;
        if ((id = pop(S, base + xcd)) >= 0) return id;
        if (steal)
            for (int d = 1; d < NXQ; ++d)
                if ((id = pop(S, base + (xcd + d + rot) % NXQ)) >= 0) return id;
    }
    return -1;
}

__global__ void k_lu_init(Sched S)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t id = t0; id < S.total_ids; id += stride) {
        const LTask t = decode(S.p, id);
        S.counters[id] = valid(S.p, t) ? indegree(t) : -1;
    }
    for (int64_t e = t0; e < S.nslot; e += stride) S.qslot[e] = 0;
    for (int64_t e = t0; e < 2 * NQ; e += stride) S.qctl[e * QSTRIDE] = 0;
    if (t0 == 0) *S.done = 0;
}

__global__ void k_lu_seed(Sched S)
{
    if (threadIdx.x == 0) {
        S.qslot[S.qoff[0]] = 1;   // GETRF(0), id 0
        S.qctl[NQ * QSTRIDE] = 1;
    }
}

__global__ __launch_bounds__(NT) void k_lu_worker(Sched S)
{
    __shared__ Smem sm;
    __shared__ int64_t s_id, s_next;
    __shared__ int s_exit;
    const int tid = threadIdx.x;
    const int xcd = xcd_id();
    uint64_t rng = mix64(S.seed ^ (0x9e3779b97f4a7c15ULL * (blockIdx.x + 1)));
    if (tid == 0) s_next = -1;
    for (;;) {
        if (tid == 0) {
            int64_t id = s_next;
            int ex = 0;
            s_next = -1;
            if (id >= 0) {
                const int lv = level_of(decode(S.p, id));
                if (lv > 0) {
                    const int64_t hi = pop_upto(S, lv - 1, xcd, false, 0);
                    if (hi >= 0) {
                        push(S, queue_of(decode(S.p, id)), id);
                        id = hi;
                    }
                }
            }
            if (id < 0) {
                int64_t idle = 0;
                uint32_t seen = ld_rlx(S.done);
                int backoff = 0;
                for (uint32_t round = 0;; ++round) {
                    uint64_t pick = 0;
                    if (S.shuffle) {
                        rng = mix64(rng + 1);
                        for (int z = 0; z < (int)(rng & 7); ++z) __builtin_amdgcn_s_sleep(1);
                        pick = rng >> 8;
                    }
                    id = pop_upto(S, 3, xcd, (round & 7) == 7, pick);
                    if (id >= 0) break;
                    if ((round & 3) == 0) {
                        if (__hip_atomic_load(S.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            ex = 1;
                            break;
                        }
                        const uint32_t d = ld_rlx(S.done);
                        if ((int64_t)d >= S.total_tasks) {
                            ex = 1;
                            break;
                        }
                        if (d != seen) {
                            seen = d;
                            idle = 0;
                        }
                    }
                    if (++idle > S.spin_limit) {
                        __hip_atomic_fetch_or(S.status, ST_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ex = 1;
                        break;
                    }
                    backoff = backoff < 6 ? backoff + 1 : 6;
                    for (int z = 0; z < (1 << backoff); ++z) __builtin_amdgcn_s_sleep(2);
                }
            }
            s_id = id;
            s_exit = ex;
        }
        __syncthreads();
        if (s_exit) break;
        const int64_t id = s_id;
        if (tid < 64) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        const LTask t = decode(S.p, id);
        if (tid == 0) sm.fail = 0;
        __syncthreads();
        run_task(sm, S, t);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (tid < 64) {
            // A task that found no pivot releases nothing: the workers stop on
            // the status.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const bool failed = sm.fail != 0;
            const int ns = failed ? 0 : nsucc(S.p, t);
            bool kept = false;
            for (int base = 0; base < ns; base += 64) {
                const int nn = base + tid;
                bool ready = false;
                int64_t sid = -1;
                if (nn < ns) {
                    sid = succ(S.p, t, nn);
                    const int32_t old = __hip_atomic_fetch_add(&S.counters[sid], -1, __ATOMIC_ACQUIRE,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                    ready = old == 1;
                }
                const uint64_t mask = __ballot(ready);
                int keeper = -1;
                if (!kept && mask != 0) {
                    keeper = __builtin_ctzll(mask);
                    kept = true;
                }
                if (ready) {
                    if (tid == keeper) s_next = sid;
                    else push(S, queue_of(decode(S.p, sid)), sid);
                }
            }
            if (tid == 0 && !failed) __hip_atomic_fetch_add(S.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// Algorithm 3 in loop order: GETRF(k), the GESSMs of step k (independent),
// then for each i in turn TSTRF(k, i) and the SSSSMs of row i (independent).
template <int TYPE>
__global__ __launch_bounds__(NT) void k_lu_step(Sched S, int k, int i)
{
    __shared__ Smem sm;
    if (*S.status != 0) return;
    if (threadIdx.x == 0) sm.fail = 0;
    __syncthreads();
    LTask t{TYPE, k, k, k};
    if (TYPE == T_GESSM) t.j = k + 1 + (int)blockIdx.x;
    if (TYPE == T_TSTRF) t.i = i;
    if (TYPE == T_SSSSM) {
        t.i = i;
        t.j = k + 1 + (int)blockIdx.x;
    }
    run_task(sm, S, t);
}

// ---------------------------------------------------------------- layout

// Column-major n x n A -> tiles (row-major inside); beyond n the diagonal
// is one and the rest zero.  NaN or Inf sets ST_NONFINITE.  One 64 x 64 tile
// per workgroup, transposed through LDS.
__global__ __launch_bounds__(256) void k_lu_in(const double *A, int64_t lda, int64_t n, double *tiles, int p,
                                               int32_t *status)
{
    __shared__ double blk[64][65];
    const int64_t b = blockIdx.x;
    const int tj = (int)(b / p), ti = (int)(b % p);
    const int64_t R0 = (int64_t)ti * 64, C0 = (int64_t)tj * 64;
    bool bad = false;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e % 64, c = e / 64;
        const int64_t R = R0 + r, C = C0 + c;
        double v = 0.0;
        if (R < n && C < n) {
            v = A[C * lda + R];
            if (!isfinite(v)) bad = true;
        } else if (R == C) {
            v = 1.0;
        }
        blk[r][c] = v;
    }
    if (bad) __hip_atomic_fetch_or(status, ST_NONFINITE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    double *T = tiles + ((size_t)tj * p + ti) * (size_t)(64 * 64);
    for (int e = threadIdx.x; e < 64 * 64; e += 256) T[e] = blk[e / 64][e % 64];
}

__global__ __launch_bounds__(256) void k_lu_out(double *A, int64_t lda, int64_t n, const double *tiles, int p,
                                                const int32_t *status)
{
    __shared__ double blk[64][65];
    if (*status != 0) return;
    const int64_t b = blockIdx.x;
    const int tj = (int)(b / p), ti = (int)(b % p);
    const double *T = tiles + ((size_t)tj * p + ti) * (size_t)(64 * 64);
    for (int e = threadIdx.x; e < 64 * 64; e += 256) blk[e / 64][e % 64] = T[e];
    __syncthreads();
    const int64_t R0 = (int64_t)ti * 64, C0 = (int64_t)tj * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e % 64, c = e / 64;
        const int64_t R = R0 + r, C = C0 + c;
        if (R < n && C < n) A[C * lda + R] = blk[r][c];
    }
}

__global__ void k_lu_status_init(int32_t *status, int32_t *minor)
{
    if (threadIdx.x == 0) {
        *status = 0;
        *minor = INT_MAX;
    }
}

hipError_t launch_run(const Sched &S, bool serial, int workers, hipStream_t st)
{
    if (serial) {
        for (int k = 0; k < S.p; ++k) {
            const int nt = S.p - k - 1;
            hipLaunchKernelGGL((k_lu_step<T_GETRF>), dim3(1), dim3(NT), 0, st, S, k, k);
            if (nt > 0) hipLaunchKernelGGL((k_lu_step<T_GESSM>), dim3(nt), dim3(NT), 0, st, S, k, k);
            for (int i = k + 1; i < S.p; ++i) {
                hipLaunchKernelGGL((k_lu_step<T_TSTRF>), dim3(1), dim3(NT), 0, st, S, k, i);
                hipLaunchKernelGGL((k_lu_step<T_SSSSM>), dim3(nt), dim3(NT), 0, st, S, k, i);
            }
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_lu_worker, dim3(workers), dim3(NT), 0, st, S);
    return hipGetLastError();
}

}  // namespace tl

extern "C" size_t tilelu_lup_size(int64_t n, int64_t nb, int64_t ib)
{
    if (n <= 0 || nb != tl::NB || (ib != 16 && ib != 32)) return 0;
    const int64_t p = cdiv(n, nb);
    return (size_t)(p * p * ib * nb);
}

extern "C" size_t tilelu_piv_size(int64_t n, int64_t nb)
{
    if (n <= 0 || nb != tl::NB) return 0;
    const int64_t p = cdiv(n, nb);
    return (size_t)(p * p * nb);
}

extern "C" int64_t tilelu_dag_counts(int64_t p, int64_t *counts)
{
    if (p < 0) return -1;
    return tl::count_tasks(p, counts);
}

extern "C" int tilelu_dag_selfcheck(int64_t p64, int64_t trials, uint64_t seed)
{
    using namespace tl;
    if (p64 < 1 || p64 > 48 || trials < 0) return -1;
    const int p = (int)p64;
    const int64_t nid = (int64_t)p + 2 * (int64_t)p * p + (int64_t)p * p * p;
    std::vector<int> seen((size_t)nid, 0);
    int64_t nvalid = 0;
    for (int64_t id = 0; id < nid; ++id) {
        const LTask t = decode(p, id);
        if (!valid(p, t)) continue;
        ++nvalid;
        for (int s = 0; s < nsucc(p, t); ++s) {
            const int64_t sid = succ(p, t, s);
            if (sid < 0 || sid >= nid || !valid(p, decode(p, sid))) return 1;
            ++seen[(size_t)sid];
        }
    }
    if (nvalid != count_tasks(p, nullptr)) return 2;
    for (int64_t id = 0; id < nid; ++id) {
        const LTask t = decode(p, id);
        if (valid(p, t) && seen[(size_t)id] != indegree(t)) return 3;
    }
    // Algorithm 3's loop order: the version of every region a task reads or
    // writes.  A diagonal tile is two regions: its upper triangle U_kk
    // (written by GETRF and the TSTRF chain) and L_kk with GETRF's pivots
    // (written by GETRF, read by GESSM), region p^2 + k.
    struct Access {
        int tile, version;
        bool write;
    };
    std::vector<std::vector<Access>> acc((size_t)nid);
    const int lreg = p * p;
    {
        std::vector<int> ver((size_t)p * p + p, 0);
        auto touch = [&](int64_t id, int i, int j, bool wr) {
            acc[(size_t)id].push_back({i * p + j, ver[(size_t)(i * p + j)], wr});
        };
        auto commit = [&](int64_t id) {
            for (auto &a : acc[(size_t)id])
                if (a.write) ++ver[(size_t)a.tile];
        };
        auto touch_l = [&](int64_t id, int k, bool wr) {
            acc[(size_t)id].push_back({lreg + k, ver[(size_t)(lreg + k)], wr});
        };
        for (int k = 0; k < p; ++k) {
            const int64_t a = id_getrf(p, k);
            touch(a, k, k, true);
            touch_l(a, k, true);
            commit(a);
            for (int j = k + 1; j < p; ++j) {
                const int64_t b = id_gessm(p, k, j);
                touch_l(b, k, false);
                touch(b, k, j, true);
                commit(b);
            }
            for (int i = k + 1; i < p; ++i) {
                const int64_t c = id_tstrf(p, k, i);
                touch(c, k, k, true);
                touch(c, i, k, true);
                commit(c);
                for (int j = k + 1; j < p; ++j) {
                    const int64_t d = id_ssssm(p, k, i, j);
                    touch(d, i, k, false);
                    touch(d, k, j, true);
                    touch(d, i, j, true);
                    commit(d);
                }
            }
        }
    }
    std::mt19937_64 rng(seed);
    for (int64_t tr = 0; tr < trials; ++tr) {
        std::vector<int> cnt((size_t)nid);
        std::vector<int64_t> ready;
        for (int64_t id = 0; id < nid; ++id) {
            const LTask t = decode(p, id);
            cnt[(size_t)id] = valid(p, t) ? indegree(t) : -1;
            if (cnt[(size_t)id] == 0) ready.push_back(id);
        }
        std::vector<int> ver((size_t)p * p + p, 0);
        int64_t ran = 0;
        while (!ready.empty()) {
            const size_t pick = (size_t)(rng() % ready.size());
            const int64_t id = ready[pick];
            ready[pick] = ready.back();
            ready.pop_back();
            for (auto &a : acc[(size_t)id])
                if (ver[(size_t)a.tile] != a.version) return 4;
            for (auto &a : acc[(size_t)id])
                if (a.write) ++ver[(size_t)a.tile];
            ++ran;
            const LTask t = decode(p, id);
            for (int s = 0; s < nsucc(p, t); ++s) {
                const int64_t sid = succ(p, t, s);
                if (--cnt[(size_t)sid] == 0) ready.push_back(sid);
            }
        }
        if (ran != nvalid) return 5;
    }
    return 0;
}

extern "C" int tilelu_factor(int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib, double *Lup, int32_t *piv,
                             const tileqr_opts *opts, tilelu_info *info)
{
    if (n < 0 || n > (int64_t)INT_MAX / 2) return -1;
    if (n > 0 && !A) return -2;
    if (lda < std::max<int64_t>(1, n)) return -3;
    if (nb <= 0) return -4;
    if (ib <= 0 || nb % ib != 0) return -5;
    if (n > 0 && !Lup) return -6;
    if (n > 0 && !piv) return -7;
    tileqr_opts o;
    tileqr_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision < TILEQR_FP64 || o.precision > TILEQR_BF16X3) return -8;
    if (info) {
        info->minor = 0;
        info->ms_factor = info->ms_worker = 0.0;
    }
    if (nb != tl::NB || (ib != 16 && ib != 32) || o.precision != TILEQR_FP64) return TILEQR_EUNSUPPORTED;
    if (n == 0) return TILEQR_OK;

    std::lock_guard<std::mutex> lock(g_mu);
    hipStream_t st = (hipStream_t)o.stream;
    Workspace *W = workspace(st);
    if (!W) return hip_fail(hipErrorNoDevice, "workspace");
    const int p = (int)cdiv(n, nb);
    int64_t cnt[4];
    const int64_t total = tl::count_tasks(p, cnt);
    const int64_t nid = (int64_t)p + 2 * (int64_t)p * p + (int64_t)p * p * p;
    // Queue capacities: every task is queued at most once, into its level's
    // queue (and XCD for the updates, by tile column).
    int64_t cap[tl::NQ] = {};
    cap[0] = cnt[0] + cnt[2];
    cap[1] = std::max<int64_t>(1, cnt[1]);
    for (int k = 0; k < p; ++k)
        for (int j = k + 1; j < p; ++j) {
            const int lv = j == k + 1 ? 2 : 3;
            cap[2 + (lv - 2) * tl::NXQ + j % tl::NXQ] += p - k - 1;   // SSSSM(k, i, j), i = k+1 .. p-1
        }
    int64_t off[tl::NQ + 1];
    off[0] = 0;
    for (int q = 0; q < tl::NQ; ++q) off[q + 1] = off[q] + std::max<int64_t>(cap[q], 1);
    int rc;
    if ((rc = W->tiles.ensure((size_t)p * p * nb * nb * sizeof(double)))) return rc;
    if ((rc = W->status.ensure(256))) return rc;
    if ((rc = W->sched.counters.ensure((size_t)nid * sizeof(int32_t)))) return rc;
    if ((rc = W->sched.qslot.ensure((size_t)off[tl::NQ] * sizeof(int32_t)))) return rc;
    if ((rc = W->sched.qctl.ensure((size_t)(2 * tl::NQ * tl::QSTRIDE + 64) * sizeof(uint32_t)))) return rc;
    const bool timing = (o.flags & TILEQR_FLAG_TIMING) && !(o.flags & TILEQR_FLAG_ASYNC) && info;
    if (timing && !W->ev[0])
        for (auto &e : W->ev) TQ_HIP(hipEventCreate(&e));

    tl::Sched S;
    S.tiles = (double *)W->tiles.ptr;
    S.lup = Lup;
    S.piv = piv;
    S.p = p;
    S.ib = (int)ib;
    S.counters = (int32_t *)W->sched.counters.ptr;
    S.qslot = (int32_t *)W->sched.qslot.ptr;
    for (int q = 0; q < tl::NQ; ++q) S.qoff[q] = off[q];
    S.qctl = (uint32_t *)W->sched.qctl.ptr;
    S.done = S.qctl + 2 * tl::NQ * tl::QSTRIDE;
    S.total_ids = nid;
    S.total_tasks = total;
    S.nslot = off[tl::NQ];
    S.status = (int32_t *)W->status.ptr;
    S.minor = S.status + 32;
    S.spin_limit = o.spin_limit > 0 ? o.spin_limit : (int64_t)1 << 24;
    S.shuffle = (o.flags & TILEQR_FLAG_SHUFFLE) ? 1 : 0;
    S.seed = o.seed;
    int workers = (int)o.workers;
    if (workers <= 0) workers = std::max(1, W->num_cu);

    hipLaunchKernelGGL(tl::k_lu_status_init, dim3(1), dim3(64), 0, st, S.status, S.minor);
    if (timing) TQ_HIP(hipEventRecord(W->ev[0], st));
    hipLaunchKernelGGL(tl::k_lu_in, dim3((unsigned)((int64_t)p * p)), dim3(256), 0, st, A, lda, n, S.tiles, p,
                       S.status);
    const bool serial = (o.flags & TILEQR_FLAG_SERIAL) != 0;
    if (!serial) {
        const int64_t work = std::max(nid, off[tl::NQ]);
        const unsigned g = (unsigned)std::min<int64_t>(4096, (work + 255) / 256);
        hipLaunchKernelGGL(tl::k_lu_init, dim3(g), dim3(256), 0, st, S);
        hipLaunchKernelGGL(tl::k_lu_seed, dim3(1), dim3(64), 0, st, S);
    }
    TQ_HIP(hipGetLastError());
    if (timing) TQ_HIP(hipEventRecord(W->ev[1], st));
    hipError_t e = tl::launch_run(S, serial, workers, st);
    if (e != hipSuccess) return hip_fail(e, "tilelu worker");
    if (timing) TQ_HIP(hipEventRecord(W->ev[2], st));
    hipLaunchKernelGGL(tl::k_lu_out, dim3((unsigned)((int64_t)p * p)), dim3(256), 0, st, A, lda, n, S.tiles, p,
                       S.status);
    TQ_HIP(hipGetLastError());
    if (timing) TQ_HIP(hipEventRecord(W->ev[3], st));
    if (o.flags & TILEQR_FLAG_ASYNC) return TILEQR_OK;
    TQ_HIP(hipMemcpyAsync(W->host_small, S.status, 33 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TQ_HIP(hipStreamSynchronize(st));
    const int32_t *hs = (const int32_t *)W->host_small;
    const int32_t status = hs[0], minor = hs[32];
    if (timing) {
        float a = 0.f, b = 0.f;
        TQ_HIP(hipEventElapsedTime(&a, W->ev[0], W->ev[3]));
        TQ_HIP(hipEventElapsedTime(&b, W->ev[1], W->ev[2]));
        info->ms_factor = a;
        info->ms_worker = b;
    }
    if (status & tl::ST_NONFINITE) return TILEQR_ENONFINITE;
    if (status & tl::ST_SINGULAR) {
        if (info) info->minor = minor;
        return TILEQR_ESINGULAR;
    }
    if (status & tl::ST_TIMEOUT) return TILEQR_ETIMEOUT;
    return TILEQR_OK;
}
