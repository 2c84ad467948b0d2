// Tiled Cholesky factorisation A = L L^T (Section 3.1, Algorithm 1) on
// gfx950: the lower triangle in nb x nb tiles, row-major inside (the layout
// of the QR tiles), and the DAG of POTF2 / TRSM / GSMM tasks run by a
// persistent kernel with per-task dependency counters and ready queues in HBM
// (the dynamic scheduling of Section 4).
//
// One workgroup of four wave64s runs one task on one tile:
//   POTF2(k)      the diagonal tile in LDS, factored by panels of 32 columns:
//                 each panel first takes the products with the columns left
//                 of it (FP64 MFMA), then its 32 x 32 diagonal block is
//                 factored by one wave column by column, and the rows below
//                 it are solved with that block row by row (one row per
//                 thread);
//   TRSM(k, i)    A_ik in LDS, solved with L_kk^T by the same panels: the
//                 products with the solved columns on MFMA (L_kk from
//                 memory), then one row per thread through the 32 x 32 block;
//   GSMM(k, i, j) C = A_ij - L_ik L_jk^T on MFMA with C in registers (each
//                 wave a quarter of the tile) and L_ik, L_jk staged through
//                 LDS 32 columns at a time, double-buffered; on a diagonal
//                 tile only the blocks on or below the diagonal.
// The paper's DPOTF2 is the unblocked factorisation of the tile; the panels
// here compute the same factor with the inner products grouped by panel.
// Every task's arithmetic is fixed by its inputs (no atomics on data, fixed
// summation orders), so the DAG result is bitwise the one of Algorithm 1's
// loop order, whatever order the tasks run in.
#include "tileqr_host.h"
#include "../../include/tilechol.h"

#include <algorithm>
#include <climits>
#include <random>
#include <vector>

using namespace tq;

namespace tc {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;        // threads per workgroup
constexpr int PW = 32;         // panel width inside a tile
constexpr int KC = 32;         // K columns per GSMM staging step
constexpr int NXQ = 8;         // XCDs (ready queues of the GSMM levels)
constexpr int QSTRIDE = 64;    // words between queue heads / tails (256 bytes)
constexpr int NQ = 2 + 2 * NXQ;
enum { T_POTF2 = 0, T_TRSM = 1, T_GSMM = 2 };
// Status bits (the caller's word): NaN / Inf in the input, watchdog, a pivot
// that is not positive.
enum { ST_NONFINITE = 1, ST_TIMEOUT = 2, ST_NOTSPD = 8 };

struct Sched {
    double *tiles;
    int32_t p, nb;
    int32_t *counters;         // [total_ids] in-degrees still open (-1: no such task)
    int32_t *qslot;            // queue slots, queue q from qoff[q]
    int64_t qoff[NQ];
    uint32_t *qctl;            // head of queue q at q * QSTRIDE, tail at (NQ + q) * QSTRIDE
    uint32_t *done;            // tasks finished
    int64_t total_ids, total_tasks;
    int64_t nslot;             // queue slots in all
    int32_t *status;           // ST_* bits
    int32_t *minor;            // smallest failing leading-minor order (INT_MAX: none)
    int64_t spin_limit;
    int32_t shuffle;
    uint64_t seed;
};

struct CTask {
    int type, k, i, j;
};

// Dense task ids (with holes): POTF2(k) = k, TRSM(k, i) = p + k p + i,
// GSMM(k, i, j) = p + p^2 + (k p + i) p + j.
__host__ __device__ inline int64_t id_potf2(int p, int k) { (void)p; return k; }
__host__ __device__ inline int64_t id_trsm(int p, int k, int i) { return (int64_t)p + (int64_t)k * p + i; }
__host__ __device__ inline int64_t id_gsmm(int p, int k, int i, int j)
{
    return (int64_t)p + (int64_t)p * p + ((int64_t)k * p + i) * p + j;
}

__host__ __device__ inline CTask decode(int p, int64_t id)
{
    CTask t{0, 0, 0, 0};
    if (id < p) {
        t.type = T_POTF2;
        t.k = t.i = t.j = (int)id;
    } else if (id < (int64_t)p + (int64_t)p * p) {
        const int64_t r = id - p;
        t.type = T_TRSM;
        t.k = (int)(r / p);
        t.i = (int)(r % p);
        t.j = t.k;
    } else {
        int64_t r = id - p - (int64_t)p * p;
        t.type = T_GSMM;
        t.j = (int)(r % p);
        r /= p;
        t.i = (int)(r % p);
        t.k = (int)(r / p);
    }
    return t;
}

__host__ __device__ inline bool valid(int p, const CTask &t)
{
    if (t.type == T_POTF2) return t.k < p;
    if (t.type == T_TRSM) return t.k < t.i && t.i < p;
    return t.k < t.j && t.j <= t.i && t.i < p;
}

// In-degree: the tasks of Algorithm 1 whose results the task reads.
__host__ __device__ inline int indegree(const CTask &t)
{
    const int prev = t.k > 0 ? 1 : 0;   // the update of the same tile in step k-1
    if (t.type == T_POTF2) return prev;
    if (t.type == T_TRSM) return 1 + prev;   // POTF2(k)
    return (t.i == t.j ? 1 : 2) + prev;      // TRSM(k, i) [and TRSM(k, j)]
}

__host__ __device__ inline int nsucc(int p, const CTask &t)
{
    return t.type == T_GSMM ? 1 : p - t.k - 1;
}

// Successor n (0 <= n < nsucc) of a task.
__host__ __device__ inline int64_t succ(int p, const CTask &t, int n)
{
    if (t.type == T_POTF2) return id_trsm(p, t.k, t.k + 1 + n);
    if (t.type == T_TRSM) {
        // L_ik feeds the updates of row i (columns k+1 .. i) and of column i
        // (rows i+1 .. p-1).
        if (n < t.i - t.k) return id_gsmm(p, t.k, t.i, t.k + 1 + n);
        return id_gsmm(p, t.k, t.i + 1 + (n - (t.i - t.k)), t.i);
    }
    if (t.j == t.k + 1) return t.i == t.j ? id_potf2(p, t.k + 1) : id_trsm(p, t.k + 1, t.i);
    return id_gsmm(p, t.k + 1, t.i, t.j);
}

// Ready queue of a task: POTF2, TRSM, then per XCD the updates that feed the
// next step's panel (column k+1) and the other updates.
__host__ __device__ inline int level_of(const CTask &t)
{
    if (t.type == T_POTF2) return 0;
    if (t.type == T_TRSM) return 1;
    return t.j == t.k + 1 ? 2 : 3;
}
__host__ __device__ inline int queue_of(const CTask &t)
{
    const int lv = level_of(t);
    return lv < 2 ? lv : 2 + (lv - 2) * NXQ + t.j % NXQ;
}

// ------------------------------------------------------------ tile kernels

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    // D = A B + C on 16 x 16 x 4 FP64 blocks: lane L (n = L % 16, g = L / 16)
    // supplies A[n][g] and B[g][n] and holds D[4 r + g][n] in element r.
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Accesses to the tiles the tasks hand to each other: relaxed atomics at
// agent scope, i.e. loads and stores coherent across the XCDs' L2 caches on
// their own.  A task's results are published by waiting for its stores to
// complete before the dependency counters move, and its inputs are read with
// such loads after the task was taken, so no task needs the whole-cache
// write-back or invalidate of an agent-scope release or acquire fence.
__device__ __forceinline__ double gld(const double *p)
{
    return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void gst(double *p, double v)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Waits until this wave's stores have completed (are visible at agent
// scope); also a compiler barrier for memory accesses.
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The thread's index, opaque to the optimiser: addresses derived from it are
// formed inside each task instead of being hoisted out of the persistent
// loop, where the three task bodies would keep all of them live at once.
__device__ __forceinline__ int opaque_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row strides of the LDS arrays: two doubles of padding, so that the 16
// rows x 4 columns an MFMA operand load reads (lane n + 16 g: row n, column
// g) fall in distinct banks in each half-wave (bank pair 4 n + 2 g).
constexpr int LDX(int cols) { return cols + 2; }

template <int NB>
struct SmemF {
    double X[NB][LDX(NB)];     // the tile being factored or solved
    double Lb[PW][PW + 1];     // TRSM: the diagonal block of L_kk of the panel
    int fail;
};

template <int NB>
struct SmemG {
    double A[2][NB][LDX(KC)];  // L_ik, columns [kc, kc + KC)
    double B[2][NB][LDX(KC)];  // L_jk, same columns
    int chain;                 // C kept in registers for the next update of the tile
};

// The update tile of a GSMM in accumulator layout: wave w (row half w / 2,
// column half w % 2) holds a quarter of C in 16 x 16 blocks.
template <int NB>
using CAcc = d4[NB / 32][NB / 32];

template <int NB>
union Smem {
    SmemF<NB> f;
    SmemG<NB> g;
};

__device__ __forceinline__ double *tile_at(const Sched &S, int i, int j)
{
    return S.tiles + ((size_t)j * S.p + i) * (size_t)S.nb * S.nb;
}

// Rows r0 .. NB-1 of panel columns [c0, c0 + PW) of X, after the products
// with columns [0, c0) of X (POTF2) or of L (TRSM) are subtracted, divided by
// L_bb^T row by row: x_c = (x_c - sum_{c' < c} x_c' L_bb[c][c']) / L_bb[c][c],
// one row per thread.
template <int NB>
__device__ __forceinline__ void solve_rows(SmemF<NB> &sm, const double *Lbb, int ld, int r0, int c0)
{
    const int r = r0 + opaque_tid();
    if (r >= NB) return;
    double x[PW];
#pragma unroll
    for (int c = 0; c < PW; ++c) x[c] = sm.X[r][c0 + c];
#pragma unroll
    for (int c = 0; c < PW; ++c) {
        double s = x[c];
#pragma unroll
        for (int cp = 0; cp < c; ++cp) s -= x[cp] * Lbb[c * ld + cp];
        x[c] = s / Lbb[c * ld + c];
    }
#pragma unroll
    for (int c = 0; c < PW; ++c) sm.X[r][c0 + c] = x[c];
}

// POTF2(k): the diagonal tile T (row-major, NB x NB) <- its Cholesky factor
// (lower triangle; the upper triangle is neither read nor written).  On a
// pivot that is not positive: the status bit and the minor's order, and no
// store.
template <int NB>
__device__ void task_potf2(SmemF<NB> &sm, double *T, int k, int32_t *status, int32_t *minor)
{
    const int tid = opaque_tid(), w = tid >> 6, lane = tid & 63, n = lane & 15, g = lane >> 4;
    for (int e = tid; e < NB * NB; e += NT) {
        const int r = e / NB, c = e % NB;
        sm.X[r][c] = r >= c ? gld(&T[e]) : 0.0;
    }
    if (tid == 0) sm.fail = 0;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB / PW; ++b) {
        const int c0 = b * PW;
        if (b > 0) {
            // X[r][c] -= sum_{k < c0} X[r][k] X[c][k] for rows r >= c0 and
            // the panel's columns (blocks wholly above the diagonal skipped).
            const int nrb = (NB - c0) / 16;
            for (int blk = w; blk < nrb * 2; blk += 4) {
                const int rb = blk >> 1, cb = blk & 1;
                if (rb < cb) continue;
                const int r0 = c0 + 16 * rb, cc0 = c0 + 16 * cb;
                d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
                for (int ks = 0; ks < c0 / 4; ++ks) acc = mfma(sm.X[r0 + n][4 * ks + g], sm.X[cc0 + n][4 * ks + g], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) sm.X[r0 + 4 * r + g][cc0 + n] -= acc[r];
            }
            __syncthreads();
        }
        // The 32 x 32 diagonal block, column by column, on wave 0: lane r
        // owns row c0 + r.
        if (w == 0) {
            for (int c = 0; c < PW; ++c) {
                const double d = sm.X[c0 + c][c0 + c];
                if (!(d > 0.0)) {
                    if (lane == 0) {
                        sm.fail = 1;
                        __hip_atomic_fetch_or(status, ST_NOTSPD, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_fetch_min(minor, k * NB + c0 + c + 1, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                    break;
                }
                const double ljj = sqrt(d);
                wave_sync();   // every lane has read the pivot
                if (lane == c) sm.X[c0 + c][c0 + c] = ljj;
                if (lane > c && lane < PW) sm.X[c0 + lane][c0 + c] = sm.X[c0 + lane][c0 + c] / ljj;
                wave_sync();
                if (lane > c && lane < PW) {
                    const double lrc = sm.X[c0 + lane][c0 + c];
                    for (int cp = c + 1; cp <= lane; ++cp)
                        sm.X[c0 + lane][c0 + cp] = sm.X[c0 + lane][c0 + cp] - lrc * sm.X[c0 + cp][c0 + c];
                }
                wave_sync();
            }
        }
        __syncthreads();
        if (sm.fail) return;
        solve_rows<NB>(sm, &sm.X[c0][c0], LDX(NB), c0 + PW, c0);
        __syncthreads();
    }
    for (int e = tid; e < NB * NB; e += NT) {
        const int r = e / NB, c = e % NB;
        if (r >= c) gst(&T[e], sm.X[r][c]);
    }
}

// Panel B of TRSM: columns [C0, C0 + PW) of X <- (X - X[:, :C0] L[C0.., :C0]^T)
// L_bb^{-T} (the products on MFMA with L_kk's values read from memory ahead
// of them, then the 32 x 32 block row by row).
template <int NB, int C0>
__device__ __forceinline__ void trsm_panel(SmemF<NB> &sm, const double *Tk)
{
    const int tid = opaque_tid(), w = tid >> 6, lane = tid & 63, n = lane & 15, g = lane >> 4;
    if constexpr (C0 > 0) {
        constexpr int NRB = NB / 16, KS = C0 / 4;
        for (int blk = w; blk < NRB * 2; blk += 4) {
            const int rb = blk >> 1, cb = blk & 1;
            const double *lrow = Tk + (size_t)(C0 + 16 * cb + n) * NB + g;
            double lv[KS];
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) lv[ks] = gld(&lrow[4 * ks]);
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) acc = mfma(sm.X[16 * rb + n][4 * ks + g], lv[ks], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.X[16 * rb + 4 * r + g][C0 + 16 * cb + n] -= acc[r];
        }
    }
    for (int e = tid; e < PW * PW; e += NT) {
        const int r = e / PW, c = e % PW;
        sm.Lb[r][c] = r >= c ? gld(&Tk[(size_t)(C0 + r) * NB + C0 + c]) : 0.0;
    }
    __syncthreads();
    solve_rows<NB>(sm, &sm.Lb[0][0], PW + 1, 0, C0);
    __syncthreads();
}

template <int NB, int B>
__device__ __forceinline__ void trsm_panels(SmemF<NB> &sm, const double *Tk)
{
    if constexpr (B < NB / PW) {
        trsm_panel<NB, B * PW>(sm, Tk);
        trsm_panels<NB, B + 1>(sm, Tk);
    }
}

// TRSM(k, i): tile Ti (row-major) <- Ti L_kk^{-T}, L_kk the factored diagonal
// tile Tk, by panels of 32 columns.
template <int NB>
__device__ void task_trsm(SmemF<NB> &sm, double *Ti, const double *Tk)
{
    const int tid = opaque_tid();
    for (int e = tid; e < NB * NB; e += NT) sm.X[e / NB][e % NB] = gld(&Ti[e]);
    __syncthreads();
    trsm_panels<NB, 0>(sm, Tk);
    for (int e = tid; e < NB * NB; e += NT) gst(&Ti[e], sm.X[e / NB][e % NB]);
}

// GSMM(k, i, j): C <- C - Li Lj^T (C, Li, Lj row-major NB x NB tiles); with
// diag (i == j) only the blocks on or below the diagonal, and of those only
// the entries on or below it are stored.
// Chaining: with have_c, C is already in acc (the previous update of the same
// tile kept it) and is not loaded.  With next_ctr (the counter of the next
// update of the tile, GSMM(k+1, i, j)) reading 1 at the end, this task is
// the last one that update waits for: C stays in acc for it, is not stored,
// and sm.chain says so (the caller then runs that update next on this
// workgroup).  The arithmetic is the same either way.
template <int NB>
__device__ __forceinline__ void task_gsmm(SmemG<NB> &sm, CAcc<NB> &acc, double *C, const double *Li, const double *Lj,
                                          bool diag, bool have_c, const int32_t *next_ctr)
{
    constexpr int H = NB / 2, BW = H / 16, NCH = NB / KC, PER = NB * KC / NT;
    const int tid = opaque_tid(), w = tid >> 6, lane = tid & 63, n = lane & 15, g = lane >> 4;
    const int wr = w >> 1, wc = w & 1;
    const bool active = !diag || wr >= wc;
    auto live = [&](int a, int bb) { return !diag || wr > wc || a >= bb; };
    if (!have_c) {
#pragma unroll
        for (int a = 0; a < BW; ++a)
#pragma unroll
            for (int bb = 0; bb < BW; ++bb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[a][bb][r] = (active && live(a, bb))
                                        ? gld(&C[(size_t)(wr * H + 16 * a + 4 * r + g) * NB + wc * H + 16 * bb + n])
                                        : 0.0;
    }
    double ra[PER], rb[PER];
    auto load_chunk = [&](int kc) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT, row = e / KC, col = e % KC;
            ra[u] = gld(&Li[(size_t)row * NB + kc + col]);
            rb[u] = gld(&Lj[(size_t)row * NB + kc + col]);
        }
    };
    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT, row = e / KC, col = e % KC;
            sm.A[buf][row][col] = ra[u];
            sm.B[buf][row][col] = rb[u];
        }
    };
    load_chunk(0);
    store_chunk(0);
    __syncthreads();
#pragma unroll 1
    for (int ch = 0; ch < NCH; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < NCH) load_chunk((ch + 1) * KC);
        if (active) {
#pragma unroll
            for (int ks = 0; ks < KC / 4; ++ks) {
                double av[BW], bv[BW];
#pragma unroll
                for (int a = 0; a < BW; ++a) av[a] = -sm.A[buf][wr * H + 16 * a + n][4 * ks + g];
#pragma unroll
                for (int bb = 0; bb < BW; ++bb) bv[bb] = sm.B[buf][wc * H + 16 * bb + n][4 * ks + g];
#pragma unroll
                for (int a = 0; a < BW; ++a)
#pragma unroll
                    for (int bb = 0; bb < BW; ++bb)
                        if (live(a, bb)) acc[a][bb] = mfma(av[a], bv[bb], acc[a][bb]);
            }
        }
        if (ch + 1 < NCH) store_chunk(buf ^ 1);
        __syncthreads();
    }
    if (tid == 0)
        sm.chain = next_ctr != nullptr &&
                           __hip_atomic_load(next_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1
                       ? 1
                       : 0;
    __syncthreads();
    if (sm.chain || !active) return;
#pragma unroll
    for (int a = 0; a < BW; ++a)
#pragma unroll
        for (int bb = 0; bb < BW; ++bb) {
            if (!live(a, bb)) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wr * H + 16 * a + 4 * r + g, col = wc * H + 16 * bb + n;
                if (!diag || row >= col) gst(&C[(size_t)row * NB + col], acc[a][bb][r]);
            }
        }
}

// With may_chain, a GSMM whose next update of the same tile is another GSMM
// may keep C in acc for it (task_gsmm); have_c says acc holds C already.
template <int NB>
__device__ __forceinline__ void run_task(Smem<NB> &sm, const Sched &S, const CTask &t, CAcc<NB> &acc, bool have_c,
                                         bool may_chain)
{
    if (t.type == T_POTF2) {
        task_potf2<NB>(sm.f, tile_at(S, t.k, t.k), t.k, S.status, S.minor);
    } else if (t.type == T_TRSM) {
        task_trsm<NB>(sm.f, tile_at(S, t.i, t.k), tile_at(S, t.k, t.k));
    } else {
        const int32_t *next = may_chain && t.j > t.k + 1 ? &S.counters[id_gsmm(S.p, t.k + 1, t.i, t.j)] : nullptr;
        task_gsmm<NB>(sm.g, acc, tile_at(S, t.i, t.j), tile_at(S, t.i, t.k), tile_at(S, t.j, t.k), t.i == t.j, have_c,
                      next);
    }
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
    __hip_atomic_store(&S.qslot[S.qoff[q] + slot], (int32_t)(id + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Non-blocking pop: -1 when the queue holds nothing claimable now.
__device__ __forceinline__ int64_t pop(const Sched &S, int q)
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        const uint32_t t = ld_rlx(&S.qctl[(NQ + q) * QSTRIDE]);
        const uint32_t h = ld_rlx(&S.qctl[q * QSTRIDE]);
        if (h >= t) return -1;
        const int32_t v = __hip_atomic_load(&S.qslot[S.qoff[q] + h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v == 0) return -1;   // claimed slot not written yet
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

// Queues of levels up to `maxlv` (inclusive), in priority order; the GSMM
// levels of this XCD, and with `steal` of the others after it.
__device__ __forceinline__ int64_t pop_upto(const Sched &S, int maxlv, int xcd, bool steal, uint64_t pick)
{
    int64_t id = -1;
    if (S.shuffle && (pick & 1) && maxlv >= 1) {
        // Randomised order (testing): TRSM before POTF2.
        if ((id = pop(S, 1)) >= 0) return id;
        if ((id = pop(S, 0)) >= 0) return id;
    } else {
        if ((id = pop(S, 0)) >= 0) return id;
        if (maxlv >= 1 && (id = pop(S, 1)) >= 0) return id;
    }
    // Other XCDs' queues from a rotation the pick chooses (taken modulo
    // before the conversion, so that it is never negative).
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

__global__ void k_chol_init(Sched S)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t id = t0; id < S.total_ids; id += stride) {
        const CTask t = decode(S.p, id);
        S.counters[id] = valid(S.p, t) ? indegree(t) : -1;
    }
    for (int64_t e = t0; e < S.nslot; e += stride) S.qslot[e] = 0;
    for (int64_t e = t0; e < 2 * NQ; e += stride) S.qctl[e * QSTRIDE] = 0;
    if (t0 == 0) *S.done = 0;
}

// Queues POTF2(0) (after k_chol_init, in stream order).
__global__ void k_chol_seed(Sched S)
{
    if (threadIdx.x == 0) {
        S.qslot[S.qoff[0]] = 1;   // POTF2(0), id 0
        S.qctl[NQ * QSTRIDE] = 1;
    }
}

template <int NB>
__global__ __launch_bounds__(NT) void k_chol_worker(Sched S)
{
    __shared__ Smem<NB> sm;
    __shared__ int64_t s_id, s_next, s_chain;
    __shared__ int s_exit;
    const int tid = threadIdx.x;
    const int xcd = xcd_id();
    uint64_t rng = mix64(S.seed ^ (0x9e3779b97f4a7c15ULL * (blockIdx.x + 1)));
    // The update tile a chained GSMM hands to the next update of its tile.
    CAcc<NB> acc;
    if (tid == 0) {
        s_next = -1;
        s_chain = -1;
    }
    for (;;) {
        if (tid == 0) {
            int64_t id = s_next;
            int ex = 0;
            s_next = -1;
            if (id >= 0 && id != s_chain) {
                // A kept successor yields to a queued task of a higher level
                // (not a chained update: its tile is in this workgroup's
                // registers only).
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
        // The task's inputs are read with agent-coherent loads (gld): no
        // acquire fence (it would invalidate the whole L2 of this XCD).
        const int64_t id = s_id;
        const CTask t = decode(S.p, id);
        run_task<NB>(sm, S, t, acc, id == s_chain, true);
        // Every wave's agent-coherent stores complete before any counter of
        // a successor moves (in place of a release fence, which would write
        // back the whole L2 of this XCD).
        stores_done();
        __syncthreads();
        if (tid < 64) {
            // A failed POTF2 releases nothing: the workers stop on the status.
            const bool failed = t.type == T_POTF2 && sm.f.fail;
            const bool chained = t.type == T_GSMM && sm.g.chain;
            const int ns = failed ? 0 : nsucc(S.p, t);
            bool kept = false;
            for (int base = 0; base < ns; base += 64) {
                const int nn = base + tid;
                bool ready = false;
                int64_t sid = -1;
                if (nn < ns) {
                    sid = succ(S.p, t, nn);
                    const int32_t old = __hip_atomic_fetch_add(&S.counters[sid], -1, __ATOMIC_RELAXED,
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
            // A chained GSMM's one successor read 1 before this task's
            // decrement, so it is ready now and kept (it is the next update
            // of the same tile, whose C is in acc).
            if (tid == 0) s_chain = chained ? s_next : -1;
            if (tid == 0 && !failed) __hip_atomic_fetch_add(S.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// Algorithm 1 in loop order, one kernel per step and task type (the tasks of
// one launch are independent): the reference order of the tests.
template <int NB, int TYPE>
__global__ __launch_bounds__(NT) void k_chol_step(Sched S, int k)
{
    __shared__ Smem<NB> sm;
    if (*S.status != 0) return;
    CTask t{TYPE, k, k, k};
    if (TYPE == T_TRSM) t.i = k + 1 + (int)blockIdx.x;
    if (TYPE == T_GSMM) {
        // blockIdx -> (i, j), k < j <= i, rows of the lower triangle in turn.
        int64_t r = blockIdx.x;
        int i = k + 1;
        while (r >= i - k) {
            r -= i - k;
            ++i;
        }
        t.i = i;
        t.j = k + 1 + (int)r;
    }
    CAcc<NB> acc;
    run_task<NB>(sm, S, t, acc, false, false);
}

// ---------------------------------------------------------------- layout

// Lower triangle of the column-major n x n matrix A -> tiles (row-major
// inside, p x p grid; only tiles i >= j are written).  Entries above the
// diagonal and outside the matrix read as zero, except that the diagonal
// beyond n is one (the last diagonal tile completed with the identity).
// NaN or Inf in the lower triangle sets ST_NONFINITE.  One 64 x 64 block per
// workgroup, transposed through LDS so that both sides are read and written
// in runs.
__global__ __launch_bounds__(256) void k_chol_in(const double *A, int64_t lda, int64_t n, double *tiles, int nb,
                                                 int p, int32_t *status)
{
    __shared__ double blk[64][65];
    const int bpt = nb / 64;                        // 64-blocks per tile side
    const int64_t nbk = (int64_t)p * bpt;           // 64-blocks per matrix side
    const int64_t b = blockIdx.x;
    const int64_t bj = b / nbk, bi = b % nbk;       // block row bi, block column bj
    const int ti = (int)(bi / bpt), tj = (int)(bj / bpt), ro = (int)(bi % bpt) * 64, co = (int)(bj % bpt) * 64;
    if (ti < tj) return;                            // tiles above the diagonal are not used
    const int tid = threadIdx.x;
    const int64_t R0 = bi * 64, C0 = bj * 64;
    bool bad = false;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e % 64, c = e / 64;           // runs down the columns of A
        const int64_t R = R0 + r, C = C0 + c;
        double v = 0.0;
        if (R < n && C < n) {
            if (R >= C) {
                v = A[C * lda + R];
                if (!isfinite(v)) bad = true;
            }
        } else if (R == C) {
            v = 1.0;
        }
        blk[r][c] = v;
    }
    if (bad) __hip_atomic_fetch_or(status, ST_NONFINITE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    double *T = tiles + ((size_t)tj * p + ti) * (size_t)nb * nb;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e / 64, c = e % 64;           // runs along the tile's rows
        T[(size_t)(ro + r) * nb + co + c] = blk[r][c];
    }
}

// Tiles -> the lower triangle of A (entries R >= C, R, C < n); nothing when
// the status word is set.
__global__ __launch_bounds__(256) void k_chol_out(double *A, int64_t lda, int64_t n, const double *tiles, int nb,
                                                  int p, const int32_t *status)
{
    __shared__ double blk[64][65];
    if (*status != 0) return;
    const int bpt = nb / 64;
    const int64_t nbk = (int64_t)p * bpt;
    const int64_t b = blockIdx.x;
    const int64_t bj = b / nbk, bi = b % nbk;
    if (bi < bj) return;                            // no entry on or below the diagonal
    const int tid = threadIdx.x;
    const int ti = (int)(bi / bpt), tj = (int)(bj / bpt), ro = (int)(bi % bpt) * 64, co = (int)(bj % bpt) * 64;
    const double *T = tiles + ((size_t)tj * p + ti) * (size_t)nb * nb;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e / 64, c = e % 64;
        blk[r][c] = T[(size_t)(ro + r) * nb + co + c];
    }
    __syncthreads();
    const int64_t R0 = bi * 64, C0 = bj * 64;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e % 64, c = e / 64;
        const int64_t R = R0 + r, C = C0 + c;
        if (R < n && C < n && R >= C) A[C * lda + R] = blk[r][c];
    }
}

__global__ void k_chol_status_init(int32_t *status, int32_t *minor)
{
    if (threadIdx.x == 0) {
        *status = 0;
        *minor = INT_MAX;
    }
}

// R = L^T in the tile layout of the QR's triangular solves (row-major nb x nb
// tiles, tile (i, j) at tiles + (j p + i) nb^2), tiles i <= j only:
// R[r][c] = L[c][r] for r <= c < n, else 0.  L is the column-major factor,
// its lower triangle read; consecutive threads read consecutive rows of one
// column of L.
__global__ __launch_bounds__(256) void k_chol_lt(const double *L, int64_t ldl, int64_t n, double *tiles, int nb, int p)
{
    const int64_t nb2 = (int64_t)nb * nb, total = (int64_t)p * p * nb2;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = e / nb2, w = e % nb2;
        const int i = (int)(t % p), j = (int)(t / p);
        if (i > j) continue;
        const int64_t r = (int64_t)i * nb + w / nb, c = (int64_t)j * nb + w % nb;
        tiles[e] = (r <= c && c < n) ? L[c + r * ldl] : 0.0;
    }
}

// ------------------------------------------------------------------ host

int64_t count_tasks(int64_t p, int64_t *counts)
{
    const int64_t c0 = p, c1 = p * (p - 1) / 2, c2 = (p - 1) * p * (p + 1) / 6;
    if (counts) {
        counts[0] = c0;
        counts[1] = c1;
        counts[2] = c2;
    }
    return c0 + c1 + c2;
}

template <int NB>
hipError_t launch_run(const Sched &S, bool serial, int workers, hipStream_t st)
{
    if (serial) {
        for (int k = 0; k < S.p; ++k) {
            hipLaunchKernelGGL((k_chol_step<NB, T_POTF2>), dim3(1), dim3(NT), 0, st, S, k);
            const int nt = S.p - k - 1;
            if (nt > 0) {
                hipLaunchKernelGGL((k_chol_step<NB, T_TRSM>), dim3(nt), dim3(NT), 0, st, S, k);
                hipLaunchKernelGGL((k_chol_step<NB, T_GSMM>), dim3((unsigned)((int64_t)nt * (nt + 1) / 2)), dim3(NT),
                                   0, st, S, k);
            }
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_chol_worker<NB>), dim3(workers), dim3(NT), 0, st, S);
    return hipGetLastError();
}

}  // namespace tc

using namespace tc;

extern "C" int64_t tilechol_dag_counts(int64_t p, int64_t *counts)
{
    if (p < 0) return -1;
    return count_tasks(p, counts);
}

extern "C" int tilechol_dag_selfcheck(int64_t p64, int64_t trials, uint64_t seed)
{
    if (p64 < 1 || p64 > 64 || trials < 0) return -1;
    const int p = (int)p64;
    const int64_t nid = (int64_t)p + (int64_t)p * p + (int64_t)p * p * p;
    // 1. In-degrees against the successor lists.
    std::vector<int> indeg_seen((size_t)nid, 0);
    int64_t nvalid = 0;
    for (int64_t id = 0; id < nid; ++id) {
        const CTask t = decode(p, id);
        if (!valid(p, t)) continue;
        ++nvalid;
        for (int s = 0; s < nsucc(p, t); ++s) {
            const int64_t sid = succ(p, t, s);
            if (sid < 0 || sid >= nid || !valid(p, decode(p, sid))) return 1;
            ++indeg_seen[(size_t)sid];
        }
    }
    if (nvalid != count_tasks(p, nullptr)) return 2;
    for (int64_t id = 0; id < nid; ++id) {
        const CTask t = decode(p, id);
        if (valid(p, t) && indeg_seen[(size_t)id] != indegree(t)) return 3;
    }
    // 2. Algorithm 1's loop order fixes, for every task, how many times each
    // tile it touches has been written before it; every random topological
    // order must present the same versions.
    struct Access {
        int tile;
        int version;
        bool write;
    };
    std::vector<std::vector<Access>> acc((size_t)nid);
    {
        std::vector<int> ver((size_t)p * p, 0);
        auto touch = [&](int64_t id, int i, int j, bool wr) {
            acc[(size_t)id].push_back({i * p + j, ver[(size_t)(i * p + j)], wr});
        };
        auto done_writes = [&](int64_t id) {
            for (auto &a : acc[(size_t)id])
                if (a.write) ++ver[(size_t)a.tile];
        };
        for (int k = 0; k < p; ++k) {
            const int64_t a = id_potf2(p, k);
            touch(a, k, k, true);
            done_writes(a);
            for (int i = k + 1; i < p; ++i) {
                const int64_t b = id_trsm(p, k, i);
                touch(b, k, k, false);
                touch(b, i, k, true);
                done_writes(b);
            }
            for (int i = k + 1; i < p; ++i)
                for (int j = k + 1; j <= i; ++j) {
                    const int64_t c = id_gsmm(p, k, i, j);
                    touch(c, i, k, false);
                    if (j != i) touch(c, j, k, false);
                    touch(c, i, j, true);
                    done_writes(c);
                }
        }
    }
    std::mt19937_64 rng(seed);
    for (int64_t tr = 0; tr < trials; ++tr) {
        std::vector<int> cnt((size_t)nid);
        std::vector<int64_t> ready;
        for (int64_t id = 0; id < nid; ++id) {
            const CTask t = decode(p, id);
            cnt[(size_t)id] = valid(p, t) ? indegree(t) : -1;
            if (cnt[(size_t)id] == 0) ready.push_back(id);
        }
        std::vector<int> ver((size_t)p * p, 0);
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
            const CTask t = decode(p, id);
            for (int s = 0; s < nsucc(p, t); ++s) {
                const int64_t sid = succ(p, t, s);
                if (--cnt[(size_t)sid] == 0) ready.push_back(sid);
            }
        }
        if (ran != nvalid) return 5;
    }
    return 0;
}

extern "C" int tilechol_factor(int64_t n, double *A, int64_t lda, int64_t nb, const tileqr_opts *opts,
                               tilechol_info *info)
{
    if (n < 0 || n > (int64_t)INT_MAX / 2) return -1;
    if (n > 0 && !A) return -2;
    if (lda < std::max<int64_t>(1, n)) return -3;
    if (nb != 0 && nb != 64 && nb != 128) return -4;
    tileqr_opts o;
    tileqr_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision < TILEQR_FP64 || o.precision > TILEQR_BF16X3) return -5;
    if (info) {
        info->minor = 0;
        info->nb = 0;
        info->ms_factor = info->ms_worker = 0.0;
    }
    if (o.precision != TILEQR_FP64) return TILEQR_EUNSUPPORTED;
    if (nb == 0) nb = n <= 512 ? 64 : 128;
    if (info) info->nb = nb;
    if (n == 0) return TILEQR_OK;

    std::lock_guard<std::mutex> lock(g_mu);
    hipStream_t st = (hipStream_t)o.stream;
    Workspace *W = workspace(st);
    if (!W) return hip_fail(hipErrorNoDevice, "workspace");
    const int p = (int)cdiv(n, nb);
    int64_t cnt[3];
    const int64_t total = count_tasks(p, cnt);
    const int64_t nid = (int64_t)p + (int64_t)p * p + (int64_t)p * p * p;
    // Queue capacities: every task is queued at most once, into the queue
    // of its level (and XCD for the updates, by tile column).
    int64_t cap[tc::NQ] = {};
    cap[0] = p;
    cap[1] = std::max<int64_t>(1, cnt[1]);
    for (int k = 0; k < p; ++k)
        for (int j = k + 1; j < p; ++j) {
            const int lv = j == k + 1 ? 2 : 3;
            cap[2 + (lv - 2) * tc::NXQ + j % tc::NXQ] += p - j;   // GSMM(k, i, j), i = j .. p-1
        }
    int64_t off[tc::NQ + 1];
    off[0] = 0;
    for (int q = 0; q < tc::NQ; ++q) off[q + 1] = off[q] + std::max<int64_t>(cap[q], 1);
    int rc;
    if ((rc = W->tiles.ensure((size_t)p * p * nb * nb * sizeof(double)))) return rc;
    if ((rc = W->status.ensure(256))) return rc;
    if ((rc = W->sched.counters.ensure((size_t)nid * sizeof(int32_t)))) return rc;
    if ((rc = W->sched.qslot.ensure((size_t)off[tc::NQ] * sizeof(int32_t)))) return rc;
    if ((rc = W->sched.qctl.ensure((size_t)(2 * tc::NQ * tc::QSTRIDE + 64) * sizeof(uint32_t)))) return rc;
    const bool timing = (o.flags & TILEQR_FLAG_TIMING) && !(o.flags & TILEQR_FLAG_ASYNC) && info;
    if (timing && !W->ev[0])
        for (auto &e : W->ev) TQ_HIP(hipEventCreate(&e));

    Sched S;
    S.tiles = (double *)W->tiles.ptr;
    S.p = p;
    S.nb = (int)nb;
    S.counters = (int32_t *)W->sched.counters.ptr;
    S.qslot = (int32_t *)W->sched.qslot.ptr;
    for (int q = 0; q < tc::NQ; ++q) S.qoff[q] = off[q];
    S.qctl = (uint32_t *)W->sched.qctl.ptr;
    S.done = S.qctl + 2 * tc::NQ * tc::QSTRIDE;
    S.total_ids = nid;
    S.total_tasks = total;
    S.nslot = off[tc::NQ];
    S.status = (int32_t *)W->status.ptr;
    S.minor = S.status + 32;
    S.spin_limit = o.spin_limit > 0 ? o.spin_limit : (int64_t)1 << 24;
    S.shuffle = (o.flags & TILEQR_FLAG_SHUFFLE) ? 1 : 0;
    S.seed = o.seed;
    int workers = (int)o.workers;
    if (workers <= 0) workers = std::max(1, W->num_cu);

    hipLaunchKernelGGL(k_chol_status_init, dim3(1), dim3(64), 0, st, S.status, S.minor);
    if (timing) TQ_HIP(hipEventRecord(W->ev[0], st));
    const int64_t blocks = (int64_t)p * (nb / 64) * p * (nb / 64);
    hipLaunchKernelGGL(k_chol_in, dim3((unsigned)blocks), dim3(256), 0, st, A, lda, n, S.tiles, (int)nb, p, S.status);
    const bool serial = (o.flags & TILEQR_FLAG_SERIAL) != 0;
    if (!serial) {
        const int64_t work = std::max(nid, off[tc::NQ]);
        const unsigned g = (unsigned)std::min<int64_t>(4096, (work + 255) / 256);
        hipLaunchKernelGGL(k_chol_init, dim3(g), dim3(256), 0, st, S);
        hipLaunchKernelGGL(k_chol_seed, dim3(1), dim3(64), 0, st, S);
    }
    TQ_HIP(hipGetLastError());
    if (timing) TQ_HIP(hipEventRecord(W->ev[1], st));
    hipError_t e = nb == 64 ? launch_run<64>(S, serial, workers, st) : launch_run<128>(S, serial, workers, st);
    if (e != hipSuccess) return hip_fail(e, "tilechol worker");
    if (timing) TQ_HIP(hipEventRecord(W->ev[2], st));
    hipLaunchKernelGGL(k_chol_out, dim3((unsigned)blocks), dim3(256), 0, st, A, lda, n, S.tiles, (int)nb, p,
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
    if (status & ST_NONFINITE) return TILEQR_ENONFINITE;
    if (status & ST_NOTSPD) {
        if (info) info->minor = minor;
        return TILEQR_ENOTSPD;
    }
    if (status & ST_TIMEOUT) return TILEQR_ETIMEOUT;
    return TILEQR_OK;
}

extern "C" int tilechol_solve(int64_t n, int64_t nrhs, const double *L, int64_t ldl, double *B, int64_t ldb,
                              int64_t nb, const tileqr_opts *opts)
{
    if (n < 0 || n > (int64_t)INT_MAX / 2) return -1;
    if (nrhs < 0 || nrhs > (int64_t)INT_MAX / 2) return -2;
    if (n > 0 && !L) return -3;
    if (ldl < std::max<int64_t>(1, n)) return -4;
    if (n > 0 && nrhs > 0 && !B) return -5;
    if (ldb < std::max<int64_t>(1, n)) return -6;
    if (nb != 0 && nb != 64 && nb != 128) return -7;
    tileqr_opts o;
    tileqr_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision < TILEQR_FP64 || o.precision > TILEQR_BF16X3) return -8;
    if (o.precision != TILEQR_FP64) return TILEQR_EUNSUPPORTED;
    if (nb == 0) nb = n <= 512 ? 64 : 128;
    if (n == 0 || nrhs == 0) return TILEQR_OK;

    std::lock_guard<std::mutex> lock(g_mu);
    hipStream_t st = (hipStream_t)o.stream;
    Workspace *W = workspace(st);
    if (!W) return hip_fail(hipErrorNoDevice, "workspace");
    const int p = (int)cdiv(n, nb);
    const int ldt = (int)cdiv(nrhs, 32) * 32;
    const int64_t rows = (int64_t)p * nb;
    const int64_t flags_cap = trsm_flags_needed(n, ldt);
    int rc;
    if ((rc = W->tiles.ensure((size_t)p * p * nb * nb * sizeof(double)))) return rc;
    if ((rc = W->rows.ensure((size_t)rows * ldt * sizeof(double)))) return rc;
    if ((rc = W->tflags.ensure((size_t)flags_cap * sizeof(int32_t)))) return rc;
    if ((rc = W->status.ensure(256))) return rc;
    double *tiles = (double *)W->tiles.ptr, *Bt = (double *)W->rows.ptr;
    int32_t *status = (int32_t *)W->status.ptr;
    const int64_t spin = o.spin_limit > 0 ? o.spin_limit : (int64_t)1 << 24;

    hipLaunchKernelGGL(k_chol_status_init, dim3(1), dim3(64), 0, st, status, status + 32);
    const int64_t total = (int64_t)p * p * nb * nb;
    hipLaunchKernelGGL(k_chol_lt, dim3((unsigned)std::min<int64_t>(8192, (total + 255) / 256)), dim3(256), 0, st, L,
                       ldl, n, tiles, (int)nb, p);
    TQ_HIP(hipGetLastError());
    TQ_HIP(launch_cm2rows(B, ldb, n, nrhs, Bt, rows, ldt, st));
    // L Y = B is R^T Y = B, then L^T X = Y is R X = Y.
    TQ_HIP(launch_trsm((int)nb, tiles, p, n, Bt, ldt, false, (int *)W->tflags.ptr, flags_cap, status, spin, st));
    TQ_HIP(launch_trsm((int)nb, tiles, p, n, Bt, ldt, true, (int *)W->tflags.ptr, flags_cap, status, spin, st));
    TQ_HIP(launch_rows2cm(B, ldb, n, nrhs, Bt, ldt, st));
    if (o.flags & TILEQR_FLAG_ASYNC) return TILEQR_OK;
    TQ_HIP(hipMemcpyAsync(W->host_small, status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TQ_HIP(hipStreamSynchronize(st));
    const int32_t s0 = *(const int32_t *)W->host_small;
    if (s0 & STATUS_SINGULAR) return TILEQR_ESINGULAR;
    if (s0 & STATUS_TIMEOUT) return TILEQR_ETIMEOUT;
    return TILEQR_OK;
}
