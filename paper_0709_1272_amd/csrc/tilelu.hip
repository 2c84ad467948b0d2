// Tiled LU factorisation with tiled pairwise pivoting (Section 3.2.2,
// Algorithm 3, inner blocking of Section 3.2.3) on gfx950: nb x nb tiles,
// row-major inside (the layout of the QR tiles), and the DAG of GETRF /
// GESSM / TSTRF / SSSSM tasks run by a persistent kernel with per-task
// dependency counters and ready queues in HBM (Section 4).
//
// One workgroup of four wave64s runs one task, with its tiles in LDS (about
// 74 KiB with ib = 16, so two workgroups share a CU):
//   GETRF(k)      partial pivoting on one wave, lane r holding tile row r in
//                 registers: the pivot by a wave-wide maximum, the exchange
//                 of rows as an exchange of row indices, the pivot row
//                 broadcast through LDS, the multipliers and rank-1 update;
//   GESSM(k, j)   one wave, lane c holding column c of A_kj: GETRF's
//                 exchanges composed into one gather, then L_kk^{-1} by
//                 forward substitution in registers;
//   TSTRF(k, i)   [U_kk; A_ik] by inner panels of ib columns: the panel's
//                 columns on one wave (A's panel rows in registers, U in
//                 LDS): per column the pivot among U_kk's diagonal entry and
//                 A_ik's column, the exchange of U's row with an A row (the
//                 A row's multipliers of the panel's earlier columns moving
//                 to L_up), the multipliers and the update of the panel;
//                 then the columns right of it: the exchanges, U's panel
//                 rows by L_up, and A_ik by its multipliers on FP64 MFMA;
//   SSSSM(k, i, j) every wave owns 16 columns of A_kj and A_ij: per panel
//                 the exchanges and L_up on A_kj's panel rows (one lane per
//                 column), then A_ij -= L_ik A_kj[panel] on FP64 MFMA.
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
    double *linv;              // p * p * ib * NB: per tile (i, k), the inverse of each panel's L_up triangle
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

// LDS of one task (about 74 KiB with ib = 16: two workgroups fit a CU).
template <int IB>
struct Smem {
    double X[NB][LD];          // GETRF: the tile; GESSM: A_kj; TSTRF: U_kk; SSSSM: A_kj
    double Y[NB][LD];          // GETRF: the pivot row; GESSM: L_kk; TSTRF: A_ik; SSSSM: A_ij
    double Lup[IB][NB];        // TSTRF / SSSSM: L_up of the tile
    int32_t piv[NB];
    int32_t fail;
    int32_t chain;             // SSSSM: A_kj stays here for SSSSM(k, i+1, j), run next by this workgroup
};

__device__ __forceinline__ double *tile_at(const Sched &S, int i, int j)
{
    return S.tiles + ((size_t)j * S.p + i) * (size_t)(NB * NB);
}

// Accesses to the data the tasks hand to each other (tiles, L_up, pivots):
// relaxed atomics at agent scope, i.e. loads and stores coherent across the
// XCDs' L2 caches on their own.  A task's results are published by waiting
// for its stores to complete before the dependency counters are touched, and
// its inputs are read with such loads after the task was taken, so no
// task needs a whole-cache write-back or invalidate (which an agent-scope
// release or acquire fence performs).
__device__ __forceinline__ double gld(const double *p)
{
    return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ double2 gld2(const double *p) { return make_double2(gld(p), gld(p + 1)); }
__device__ __forceinline__ int gldi(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gst(double *p, double v)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gst2(double *p, double2 v)
{
    gst(p, v.x);
    gst(p + 1, v.y);
}
__device__ __forceinline__ void gsti(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Waits until this wave's stores have completed (are visible at agent
// scope); also a compiler barrier for memory accesses.
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The thread's index, opaque to the optimiser: addresses derived from it are
// formed inside each task instead of being hoisted out of the persistent
// loop, where the four task bodies would keep all of them live at once.
__device__ __forceinline__ int opaque_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Whole-tile moves between HBM and LDS, 16-byte accesses: element pair e of
// the tile is row e / 32, columns 2 (e % 32) and the next.
__device__ __forceinline__ void load_regs(double2 (&v)[8], const double *T)
{
    const int tid = opaque_tid();
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = gld2(&T[2 * (tid + s * NT)]);
}
__device__ __forceinline__ void regs_to_lds(double (*X)[LD], const double2 (&v)[8])
{
    const int tid = opaque_tid();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int e = tid + s * NT;
        *reinterpret_cast<double2 *>(&X[e >> 5][2 * (e & 31)]) = v[s];
    }
}
__device__ __forceinline__ void load_tile(double (*X)[LD], const double *T)
{
    double2 v[8];
    load_regs(v, T);
    regs_to_lds(X, v);
}
__device__ __forceinline__ void store_tile(double *T, const double (*X)[LD])
{
    const int tid = opaque_tid();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int e = tid + s * NT;
        gst2(&T[2 * e], *reinterpret_cast<const double2 *>(&X[e >> 5][2 * (e & 31)]));
    }
}

__device__ __forceinline__ double2 ld2(const double *p) { return *reinterpret_cast<const double2 *>(p); }

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// v of lane l (l wave-uniform).
__device__ __forceinline__ double readlane(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// The largest v over the 64 lanes, in every lane: the maximum over each row
// of 16 lanes by DPP (xor 1, xor 2, mirror in 8, mirror in 16), then over
// the four rows.  Exact: a maximum only selects.
__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp<0xB1>(v));
    v = fmax(v, dpp<0x4E>(v));
    v = fmax(v, dpp<0x141>(v));
    v = fmax(v, dpp<0x140>(v));
    return fmax(fmax(readlane(v, 0), readlane(v, 16)), fmax(readlane(v, 32), readlane(v, 48)));
}

__device__ __forceinline__ bool uniform(bool b) { return __builtin_amdgcn_readfirstlane(b ? 1 : 0) != 0; }

__device__ __forceinline__ void fail_column(const Sched &S, int col)
{
    __hip_atomic_fetch_or(S.status, ST_SINGULAR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_min(S.minor, col + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Orders one wavefront's LDS accesses (its lanes exchange data through LDS).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Left-looking forward substitution with a unit lower triangle of PB rows
// (PB even), in registers: x_r -= sum_{q < r} l_rq x_q, the terms in
// increasing q.  lrow(r) points at row r of the triangle in LDS (columns
// 0 .. r-1 are read, two at a time).
template <int PB, typename LRow>
__device__ __forceinline__ void unit_lower_solve(double (&x)[PB], LRow lrow)
{
#pragma unroll
    for (int r = 1; r < PB; ++r) {
        const double *L = lrow(r);
#pragma unroll
        for (int q = 0; q < r; q += 2) {
            const double2 l = ld2(&L[q]);
            x[r] = x[r] - l.x * x[q];
            if (q + 1 < r) x[r] = x[r] - l.y * x[q + 1];
        }
    }
}

// The largest |v| over the wave with its lane (lanes whose candidate index
// `idx` is smallest among equal magnitudes win; v < 0 takes no part).
// Returns the magnitude; pl gets the lane, best its index.
__device__ __forceinline__ double wave_pick(double v, int idx, int &pl, int &best)
{
    const double m = wave_max(v);
    uint64_t mask = __ballot(v == m);
    pl = mask ? (int)__builtin_ctzll(mask) : 0;
    best = __builtin_amdgcn_readlane(idx, pl);
    for (mask &= mask - 1; mask; mask &= mask - 1) {
        const int L = __builtin_ctzll(mask);
        const int r = __builtin_amdgcn_readlane(idx, L);
        if (r < best) {
            best = r;
            pl = L;
        }
    }
    return m;
}

// GETRF(k): partial pivoting of the diagonal tile by panels of 16 columns.
// Per panel, on wave 0, lane r holding the panel part of tile row r in
// registers: rows are not moved while the panel is factored (each lane
// carries the index of the row it currently stands for, so an exchange of
// rows is an exchange of indices); per column j the pivot is the largest
// magnitude among rows j.. (on ties the smallest current row index, as a
// sequential search finds it), the pivot row is broadcast through LDS, rows
// below it take l = a_rj / u_jj and a_rc - l u_jc over the panel (rows on or
// above it use l = 0, which leaves them exactly as they are).  Then the panel
// rows go to their rows, the panel's exchanges are applied to the other
// columns in order (one lane per column), U12 = L11^{-1} A12 (one lane per
// column), and A22 -= L21 U12 on FP64 MFMA by the four waves.
template <int IB>
__device__ __forceinline__ void task_getrf(Smem<IB> &sm, const Sched &S, int k)
{
    constexpr int PB = 16;
    const int tid = opaque_tid(), lane = tid & 63, w = tid >> 6, n = lane & 15, g = lane >> 4;
    double *T = tile_at(S, k, k);
    load_tile(sm.X, T);
    __syncthreads();
    double *urow = &sm.Y[0][0];
#pragma unroll 1
    for (int l0 = 0; l0 < NB; l0 += PB) {
        const int l1 = l0 + PB;
        if (w == 0) {
            double y[PB];
#pragma unroll
            for (int t = 0; t < PB; t += 2) {
                const double2 v = ld2(&sm.X[lane][l0 + t]);
                y[t] = v.x;
                y[t + 1] = v.y;
            }
            int row = lane;
            int pj[PB];
            bool ok = true;     // wave-uniform
#pragma unroll
            for (int t = 0; t < PB; ++t) {
                pj[t] = l0 + t;
                if (!ok) continue;
                const int j = l0 + t;
                int pl, best;
                const double m = wave_pick(row >= j ? fabs(y[t]) : -1.0, row, pl, best);
                if (!uniform(m > 0.0)) {
                    if (lane == 0) {
                        sm.fail = 1;
                        fail_column(S, k * NB + j);
                    }
                    ok = false;
                    continue;
                }
                pj[t] = best;
                if (lane == 0) sm.piv[j] = best;
                if (row == j) row = best;
                else if (lane == pl) row = j;
                if (lane == pl)
#pragma unroll
                    for (int q = t & ~1; q < PB; q += 2) *reinterpret_cast<double2 *>(&urow[q]) = make_double2(y[q], y[q + 1]);
                wave_sync();
                const double u = readlane(y[t], pl);
                const double l = row > j ? y[t] / u : 0.0;
                if (row > j) y[t] = l;
#pragma unroll
                for (int q = (t + 1) & ~1; q < PB; q += 2) {
                    const double2 uq = ld2(&urow[q]);
                    if (q > t) y[q] = y[q] - l * uq.x;
                    y[q + 1] = y[q + 1] - l * uq.y;
                }
                wave_sync();
            }
            if (ok) {
#pragma unroll
                for (int t = 0; t < PB; t += 2) *reinterpret_cast<double2 *>(&sm.X[row][l0 + t]) = make_double2(y[t], y[t + 1]);
                wave_sync();
                if (lane < l0 || lane >= l1) {
#pragma unroll
                    for (int t = 0; t < PB; ++t) {
                        const int pr = pj[t];
                        if (pr != l0 + t) {
                            const double a = sm.X[l0 + t][lane], b = sm.X[pr][lane];
                            sm.X[l0 + t][lane] = b;
                            sm.X[pr][lane] = a;
                        }
                    }
                }
                wave_sync();
                if (lane >= l1) {
                    double xr[PB];
#pragma unroll
                    for (int t = 0; t < PB; ++t) xr[t] = sm.X[l0 + t][lane];
                    unit_lower_solve<PB>(xr, [&](int r) { return &sm.X[l0 + r][l0]; });
#pragma unroll
                    for (int t = 1; t < PB; ++t) sm.X[l0 + t][lane] = xr[t];
                }
            }
        }
        __syncthreads();
        if (sm.fail) break;
        if (l1 < NB) {
            const int nbk = (NB - l1) / 16, b0 = l1 / 16;
            for (int blk = w; blk < nbk * nbk; blk += 4) {
                const int rb = b0 + blk / nbk, cb = b0 + blk % nbk;
                d4 acc;
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = sm.X[16 * rb + 4 * r + g][16 * cb + n];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc = mfma(-sm.X[16 * rb + n][l0 + 4 * g + t], sm.X[l0 + 4 * g + t][16 * cb + n], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) sm.X[16 * rb + 4 * r + g][16 * cb + n] = acc[r];
            }
            __syncthreads();
        }
    }
    if (sm.fail) return;
    store_tile(T, sm.X);
    int32_t *pv = S.piv + ((size_t)k * S.p + k) * NB;
    if (tid < NB) gsti(&pv[tid], sm.piv[tid]);
}

// GESSM(k, j): A_kj <- L_kk^{-1} P_kk A_kj.  Every column is transformed on
// its own, so wave w owns columns 16 w .. 16 w + 15: GETRF's exchanges
// composed into one gather (lane r of every wave learns which row ends in
// row r), then forward substitution with the unit lower L_kk by blocks of
// 16 rows: the diagonal block's triangle in registers (one lane per column,
// left-looking), the rows below it on FP64 MFMA.
template <int IB>
__device__ __forceinline__ void task_gessm(Smem<IB> &sm, const Sched &S, int k, int j)
{
    const int tid = opaque_tid(), lane = tid & 63, w = tid >> 6, n = lane & 15, g = lane >> 4;
    double *T = tile_at(S, k, j);
    const double *Tk = tile_at(S, k, k);
    const int pvl = gldi(&S.piv[((size_t)k * S.p + k) * NB + lane]);
    {
        double2 a[8], b[8];
        load_regs(a, T);
        load_regs(b, Tk);
        regs_to_lds(sm.X, a);
        // L_kk only (the strictly lower part; the TSTRF chain may be
        // rewriting the upper triangle of the same tile meanwhile).
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int e = tid + s * NT, r = e >> 5, c = 2 * (e & 31);
            b[s].x = r > c ? b[s].x : 0.0;
            b[s].y = r > c + 1 ? b[s].y : 0.0;
        }
        regs_to_lds(sm.Y, b);
    }
    int src = lane;
    for (int q = 0; q < NB; ++q) {
        const int pr = __builtin_amdgcn_readlane(pvl, q);
        if (pr != q) {
            const int a = __builtin_amdgcn_readlane(src, q), b = __builtin_amdgcn_readlane(src, pr & (NB - 1));
            if (lane == q) src = b;
            if (lane == pr) src = a;
        }
    }
    __syncthreads();
    const int col = 16 * w + n;
    {
        double v[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) v[m] = sm.X[__shfl(src, g + 4 * m, 64) & (NB - 1)][col];
#pragma unroll
        for (int m = 0; m < 16; ++m) sm.X[g + 4 * m][col] = v[m];
    }
    wave_sync();
#pragma unroll 1
    for (int r0 = 0; r0 < NB; r0 += 16) {
        if (g == 0) {
            double xr[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) xr[t] = sm.X[r0 + t][col];
            unit_lower_solve<16>(xr, [&](int r) { return &sm.Y[r0 + r][r0]; });
#pragma unroll
            for (int t = 1; t < 16; ++t) sm.X[r0 + t][col] = xr[t];
        }
        wave_sync();
        double xb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) xb[t] = sm.X[r0 + 4 * g + t][col];
        for (int rb = r0 / 16 + 1; rb < 4; ++rb) {
            d4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = sm.X[16 * rb + 4 * r + g][col];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = mfma(-sm.Y[16 * rb + n][r0 + 4 * g + t], xb[t], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.X[16 * rb + 4 * r + g][col] = acc[r];
        }
        wave_sync();
    }
    // This wave's 16 columns: lane -> row lane / 8 + 8 s, columns
    // 16 w + 2 (lane % 8) and the next.
    const int rr = lane >> 3, cc = 16 * w + 2 * (lane & 7);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int r = rr + 8 * s;
        gst2(&T[r * NB + cc], ld2(&sm.X[r][cc]));
    }
}

// TSTRF(k, i): [U_kk; A_ik] by inner panels of IB columns.  The panel's
// columns on wave 0, lane r holding row r of A_ik's panel in registers and
// U_kk in LDS: per column j, the largest |a_rj| against |u_jj| (U's row on
// ties, then the first A row); a pivot in A row r exchanges the panel part
// of U's row j and A's row r from column j on and moves A row r's
// multipliers of the panel's earlier columns to L_up (U's row holds zeros
// there); then every A row's multiplier a_rj / u_jj and the update of the
// panel's later columns.  After the panel, the columns right of it: the
// panel's exchanges (one lane per column; they only move data, so deferring
// them past the panel's own columns changes nothing), U's panel rows by the
// unit lower L_up, then A -= A[:, panel] U[panel, :] on FP64 MFMA by all
// four waves.
template <int IB>
__device__ __forceinline__ void task_tstrf(Smem<IB> &sm, const Sched &S, int k, int i)
{
    constexpr int KP = IB / 4;
    const int tid = opaque_tid(), lane = tid & 63, w = tid >> 6, n = lane & 15, g = lane >> 4;
    double *U = tile_at(S, k, k), *A = tile_at(S, i, k);
    {
        double2 a[8], b[8];
        load_regs(a, U);
        load_regs(b, A);
        // U_kk's upper triangle (the strictly lower part, L_kk, stays in
        // memory untouched); A_ik whole.
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int e = tid + s * NT, r = e >> 5, c = 2 * (e & 31);
            a[s].x = r <= c ? a[s].x : 0.0;
            a[s].y = r <= c + 1 ? a[s].y : 0.0;
        }
        regs_to_lds(sm.X, a);
        regs_to_lds(sm.Y, b);
        for (int e = tid; e < IB * NB; e += NT) sm.Lup[e / NB][e % NB] = 0.0;
    }
    __syncthreads();
#pragma unroll 1
    for (int l0 = 0; l0 < NB; l0 += IB) {
        const int l1 = l0 + IB;
        if (w == 0) {
            double y[IB];
#pragma unroll
            for (int t = 0; t < IB; t += 2) {
                const double2 v = ld2(&sm.Y[lane][l0 + t]);
                y[t] = v.x;
                y[t + 1] = v.y;
            }
            int pj[IB];
            bool ok = true;     // wave-uniform
#pragma unroll
            for (int t = 0; t < IB; ++t) {
                pj[t] = l0 + t;
                if (!ok) continue;
                const int j = l0 + t;
                int pl, best;
                const double m = wave_pick(fabs(y[t]), lane, pl, best);
                const double d = fabs(sm.X[j][j]);
                const bool pick = uniform(m > d);
                if (!pick && !uniform(d > 0.0)) {
                    if (lane == 0) {
                        sm.fail = 1;
                        fail_column(S, k * NB + j);
                    }
                    ok = false;
                    continue;
                }
                if (!pick) pl = -1;
                pj[t] = pick ? NB + pl : j;
                if (lane == 0) sm.piv[j] = pj[t];
                if (lane == pl) {
#pragma unroll
                    for (int q = t; q < IB; ++q) {
                        const double u = sm.X[j][l0 + q];
                        sm.X[j][l0 + q] = y[q];
                        y[q] = u;
                    }
#pragma unroll
                    for (int q = 0; q < t; ++q) {
                        sm.Lup[t][l0 + q] = y[q];
                        y[q] = 0.0;
                    }
                }
                wave_sync();
                const double l = y[t] / sm.X[j][j];
                y[t] = l;
#pragma unroll
                for (int q = t + 1; q < IB; ++q) y[q] = y[q] - l * sm.X[j][l0 + q];
            }
#pragma unroll
            for (int t = 0; t < IB; t += 2) *reinterpret_cast<double2 *>(&sm.Y[lane][l0 + t]) = make_double2(y[t], y[t + 1]);
            wave_sync();
            // Columns right of the panel, one lane each: the panel's
            // exchanges in order, then U's panel rows by L_up.
            if (ok && lane >= l1) {
                const int c = lane;
#pragma unroll
                for (int t = 0; t < IB; ++t) {
                    const int pq = pj[t];
                    if (pq >= NB) {
                        const double u = sm.X[l0 + t][c];
                        sm.X[l0 + t][c] = sm.Y[pq - NB][c];
                        sm.Y[pq - NB][c] = u;
                    }
                }
                double xr[IB];
#pragma unroll
                for (int t = 0; t < IB; ++t) xr[t] = sm.X[l0 + t][c];
                unit_lower_solve<IB>(xr, [&](int r) { return &sm.Lup[r][l0]; });
#pragma unroll
                for (int t = 1; t < IB; ++t) sm.X[l0 + t][c] = xr[t];
            }
        }
        __syncthreads();
        if (sm.fail) break;
        if (w == 1 && lane < IB) {
            // Column `lane` of the inverse of the panel's unit lower L_up
            // (for SSSSM, which applies it as a product on MFMA).
            double x[IB];
#pragma unroll
            for (int r = 0; r < IB; ++r) x[r] = r == lane ? 1.0 : 0.0;
            unit_lower_solve<IB>(x, [&](int r) { return &sm.Lup[r][l0]; });
            double *li = S.linv + ((size_t)k * S.p + i) * (size_t)IB * NB + (size_t)l0 * IB;
#pragma unroll
            for (int r = 0; r < IB; ++r) gst(&li[r * IB + lane], x[r]);
        }
        if (l1 < NB) {
            // A[:, l1:] -= A[:, panel] U[panel, l1:], 16 x 16 blocks over the
            // waves; k-slot g of step t is panel column KP g + t.
            const int nblk = 4 * ((NB - l1) / 16);
            for (int blk = w; blk < nblk; blk += 4) {
                const int rb = blk & 3, cb = l1 / 16 + (blk >> 2);
                d4 acc;
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = sm.Y[16 * rb + 4 * r + g][16 * cb + n];
#pragma unroll
                for (int t = 0; t < KP; ++t)
                    acc = mfma(-sm.Y[16 * rb + n][l0 + KP * g + t], sm.X[l0 + KP * g + t][16 * cb + n], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) sm.Y[16 * rb + 4 * r + g][16 * cb + n] = acc[r];
            }
            __syncthreads();
        }
    }
    if (sm.fail) return;
    for (int e = tid; e < NB * NB; e += NT) {
        const int r = e / NB, c = e % NB;
        if (r <= c) gst(&U[e], sm.X[r][c]);
    }
    store_tile(A, sm.Y);
    double *lup = S.lup + ((size_t)k * S.p + i) * (size_t)IB * NB;
    for (int e = tid; e < IB * NB; e += NT) gst(&lup[e], sm.Lup[e / NB][e % NB]);
    int32_t *pv = S.piv + ((size_t)k * S.p + i) * NB;
    if (tid < NB) gsti(&pv[tid], sm.piv[tid]);
}

// SSSSM(k, i, j): [A_kj; A_ij] <- L_ik^{-1} P_ik [A_kj; A_ij], panel by
// panel, in two phases with a workgroup barrier after each:
//   by columns (wave w owns columns 16 w .. 16 w + 15): lanes 0..15 exchange
//     the panel's rows of A_kj with the chosen rows of A_ij (the pivots read
//     once, one per lane; all reads then all writes when the panel's rows of
//     A_ij are distinct, else one exchange after the other); then
//     A_kj[panel] <- L_up^{-1} A_kj[panel] on FP64 MFMA (the inverse TSTRF
//     formed);
//   by rows (wave w owns rows 16 w .. 16 w + 15 of A_ij):
//     A_ij -= L_ik[:, panel] A_kj[panel] on FP64 MFMA, each wave reading
//     only its 16 rows of L_ik from HBM, into registers, one panel ahead.
// Chaining: A_kj passes down the column, SSSSM(k, i, j) to SSSSM(k, i+1, j).
// When the latter waits only for this task (its counter reads 1: TSTRF(k, i+1)
// and the previous step's update of tile (i+1, j) are done, and no other task
// can make it ready), this workgroup runs it next with A_kj still in LDS
// (have_x), so A_kj is neither stored nor loaded in between.
template <int IB>
__device__ __forceinline__ void task_ssssm(Smem<IB> &sm, const Sched &S, int k, int i, int j, bool have_x,
                                           bool may_chain)
{
    constexpr int NH = IB / 16;        // 16-row blocks of a panel
    constexpr int KS = IB / 4;         // MFMA steps over a panel
    const int tid = opaque_tid(), lane = tid & 63, w = tid >> 6, n = lane & 15, g = lane >> 4;
    double *X1 = tile_at(S, k, j), *X2 = tile_at(S, i, j);
    const double *Z = tile_at(S, i, k);
    const double *LI = S.linv + ((size_t)k * S.p + i) * (size_t)IB * NB;
    const int pvl = gldi(&S.piv[((size_t)k * S.p + i) * NB + lane]);
    // A_ij stays in registers for the whole task: wave w holds rows
    // 16 w .. 16 w + 15 in the MFMA accumulator layout, yv[cb][r] = row
    // 16 w + 4 r + g, column 16 cb + n.  A_kj is in LDS (sm.X).
    d4 yv[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) yv[cb][r] = gld(&X2[(size_t)(16 * w + 4 * r + g) * NB + 16 * cb + n]);
    if (!have_x) load_tile(sm.X, X1);
    // Panel operands: li[h][t] = L_up^{-1}[16 h + n][KS g + t] and
    // zw[t] = L_ik[16 w + n][l0 + KS g + t] (k-slot g of step t is panel row
    // KS g + t in both products).
    double li[NH][KS], zw[KS];
    auto fetch = [&](int l0, double (&li_)[NH][KS], double (&zw_)[KS]) {
        const double *L = LI + (size_t)l0 * IB;
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int t = 0; t < KS; ++t) li_[h][t] = gld(&L[(16 * h + n) * IB + KS * g + t]);
#pragma unroll
        for (int t = 0; t < KS; ++t) zw_[t] = gld(&Z[(16 * w + n) * NB + l0 + KS * g + t]);
    };
    fetch(0, li, zw);
    __syncthreads();
    const int col = 16 * w + n;
#pragma unroll 1
    for (int l0 = 0; l0 < NB; l0 += IB) {
        const bool more = l0 + IB < NB;
        double lin[NH][KS], zwn[KS];
        if (more) fetch(l0 + IB, lin, zwn);
        // TSTRF's row exchanges, in their order: row l0 + t of A_kj with row
        // rt of A_ij.  The wave holding row rt swaps it with the LDS row; each
        // A_kj row is touched by one step only, and the steps that touch one
        // A_ij row run in order on the wave that holds it.
#pragma unroll
        for (int t = 0; t < IB; ++t) {
            const int pq = __builtin_amdgcn_readlane(pvl, l0 + t);
            if (pq < NB) continue;
            const int rt = (pq - NB) & (NB - 1);
            if (w != rt >> 4 || g != (rt & 3)) continue;
            const int r = (rt & 15) >> 2;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const double x = sm.X[l0 + t][16 * cb + n];
                double y;
                if (r == 0) { y = yv[cb][0]; yv[cb][0] = x; }
                else if (r == 1) { y = yv[cb][1]; yv[cb][1] = x; }
                else if (r == 2) { y = yv[cb][2]; yv[cb][2] = x; }
                else { y = yv[cb][3]; yv[cb][3] = x; }
                sm.X[l0 + t][16 * cb + n] = y;
            }
        }
        __syncthreads();
        {
            double xb[KS];
#pragma unroll
            for (int t = 0; t < KS; ++t) xb[t] = sm.X[l0 + KS * g + t][col];
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                d4 ax = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int t = 0; t < KS; ++t) ax = mfma(li[h][t], xb[t], ax);
#pragma unroll
                for (int r = 0; r < 4; ++r) sm.X[l0 + 16 * h + 4 * r + g][col] = ax[r];
            }
        }
        __syncthreads();
        // A_ij -= L_ik[:, panel] X_P.  The next panel's exchanges and product
        // touch other rows of A_kj, so no barrier follows.
        {
            double xb[4][KS];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int t = 0; t < KS; ++t) xb[cb][t] = sm.X[l0 + KS * g + t][16 * cb + n];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
#pragma unroll
                for (int t = 0; t < KS; ++t) yv[cb] = mfma(-zw[t], xb[cb][t], yv[cb]);
        }
        if (more) {
#pragma unroll
            for (int h = 0; h < NH; ++h)
#pragma unroll
                for (int t = 0; t < KS; ++t) li[h][t] = lin[h][t];
#pragma unroll
            for (int t = 0; t < KS; ++t) zw[t] = zwn[t];
        }
    }
    if (tid == 0)
        sm.chain = may_chain && i + 1 < S.p && gldi(&S.counters[id_ssssm(S.p, k, i + 1, j)]) == 1 ? 1 : 0;
    __syncthreads();
    if (!sm.chain) store_tile(X1, sm.X);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) gst(&X2[(size_t)(16 * w + 4 * r + g) * NB + 16 * cb + n], yv[cb][r]);
}

template <int IB>
__device__ __forceinline__ void run_task(Smem<IB> &sm, const Sched &S, const LTask &t, bool have_x = false,
                                         bool may_chain = false)
{
    if (t.type == T_GETRF) task_getrf(sm, S, t.k);
    else if (t.type == T_GESSM) task_gessm(sm, S, t.k, t.j);
    else if (t.type == T_TSTRF) task_tstrf(sm, S, t.k, t.i);
    else task_ssssm(sm, S, t.k, t.i, t.j, have_x, may_chain);
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

template <int IB>
__global__ __launch_bounds__(NT, IB == 16 ? 2 : 1) void k_lu_worker(Sched S)
{
    __shared__ Smem<IB> sm;
    __shared__ int64_t s_id, s_next, s_chain;   // s_chain: the chained SSSSM's id, else -1
    __shared__ int s_exit;
    const int tid = threadIdx.x;
    const int xcd = xcd_id();
    uint64_t rng = mix64(S.seed ^ (0x9e3779b97f4a7c15ULL * (blockIdx.x + 1)));
    if (tid == 0) {
        s_next = -1;
        s_chain = -1;
    }
    for (;;) {
        if (tid == 0) {
            int64_t id = s_next;
            int ex = 0;
            s_next = -1;
            // A chained SSSSM (its A_kj in LDS) runs now, whatever else is
            // ready; any other kept task yields to a ready one of a higher
            // level.
            if (id >= 0 && id != s_chain) {
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
        const LTask t = decode(S.p, id);
        const bool have_x = id == s_chain;
        __syncthreads();
        if (tid == 0) {
            sm.fail = 0;
            sm.chain = 0;
            s_chain = -1;
        }
        __syncthreads();
        run_task(sm, S, t, have_x, true);
        // Every wave's agent-coherent stores complete before any counter of
        // a successor moves (in place of a release fence, which would write
        // back the whole L2 of this XCD).
        stores_done();
        __syncthreads();
        if (tid < 64) {
            // A task that found no pivot releases nothing: the workers stop on
            // the status.
            const bool failed = sm.fail != 0;
            const bool chain = t.type == T_SSSSM && sm.chain != 0;
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
                    // A chain keeps SSSSM(k, i+1, j), successor 1 of an
                    // SSSSM, which this task's decrement made ready.
                    keeper = chain ? 1 : __builtin_ctzll(mask);
                    kept = true;
                }
                if (ready) {
                    if (tid == keeper) s_next = sid;
                    else push(S, queue_of(decode(S.p, sid)), sid);
                }
            }
            if (tid == 0) {
                s_chain = chain ? id_ssssm(S.p, t.k, t.i + 1, t.j) : -1;
                if (!failed) __hip_atomic_fetch_add(S.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}

// Algorithm 3 in loop order: GETRF(k), the GESSMs of step k (independent),
// then for each i in turn TSTRF(k, i) and the SSSSMs of row i (independent).
template <int TYPE, int IB>
__global__ __launch_bounds__(NT, IB == 16 ? 2 : 1) void k_lu_step(Sched S, int k, int i)
{
    __shared__ Smem<IB> sm;
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

// Algorithm 3's transformations of a finished factor applied to tile column
// j (right-hand sides, j = p: the tile array has that extra column), in the
// factorisation's order: GESSM(k, j), then SSSSM(k, i, j) for i = k+1 ..
// p-1, step after step, on one workgroup.  Each task stores its tiles and
// the next reads them back once those stores have completed.
template <int IB>
__global__ __launch_bounds__(NT, 1) void k_lu_forward(Sched S, int j)
{
    __shared__ Smem<IB> sm;
    for (int k = 0; k < S.p; ++k) {
        task_gessm<IB>(sm, S, k, j);
        stores_done();
        __syncthreads();
        for (int i = k + 1; i < S.p; ++i) {
            task_ssssm<IB>(sm, S, k, i, j, false, false);
            stores_done();
            __syncthreads();
        }
    }
}

// The same tasks as a (step, row) wavefront: workgroup k runs step k --
// GESSM(k, j), then SSSSM(k, i, j) for i = k+1 .. p-1 -- and publishes in
// prog[k] the last row it has finished (after its stores have completed).
// Before touching row i (row k for GESSM) it waits for step k-1 to have
// finished that row, the last writer of that tile before it.  A workgroup
// waits only for lower-numbered ones, which are dispatched first, and every
// wait is bounded (ST_TIMEOUT).  Each tile sees the same operations in the
// same order as under k_lu_forward, so the result is bitwise the same.
constexpr int PSTRIDE = 64;   // ints between progress words

template <int IB>
__global__ __launch_bounds__(NT, IB == 16 ? 2 : 1) void k_lu_forward_wave(Sched S, int j, int *prog)
{
    __shared__ Smem<IB> sm;
    __shared__ int s_abort;
    const int k = (int)blockIdx.x;
    auto wait_row = [&](int i) -> bool {
        if (k == 0) return true;
        if (threadIdx.x == 0) {
            int abort = 0;
            int64_t spins = 0;
            while (__hip_atomic_load(&prog[(k - 1) * PSTRIDE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < i) {
                if ((__hip_atomic_load(S.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ST_TIMEOUT) ||
                    ++spins > S.spin_limit) {
                    __hip_atomic_fetch_or(S.status, ST_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    abort = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            s_abort = abort;
        }
        __syncthreads();
        return s_abort == 0;
    };
    auto publish = [&](int i) {
        stores_done();
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(&prog[k * PSTRIDE], i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    if (!wait_row(k)) return;
    task_gessm<IB>(sm, S, k, j);
    publish(k);
    for (int i = k + 1; i < S.p; ++i) {
        if (!wait_row(i)) return;
        task_ssssm<IB>(sm, S, k, i, j, false, false);
        publish(i);
    }
}

// The factor's transformations on tile column j: the wavefront (prog holds
// p * PSTRIDE ints), or with `serial` the one-workgroup order.
hipError_t launch_forward(const Sched &S, int j, int *prog, bool serial, hipStream_t st)
{
    if (serial) {
        if (S.ib == 16) hipLaunchKernelGGL((k_lu_forward<16>), dim3(1), dim3(NT), 0, st, S, j);
        else hipLaunchKernelGGL((k_lu_forward<32>), dim3(1), dim3(NT), 0, st, S, j);
        return hipGetLastError();
    }
    hipError_t e = hipMemsetAsync(prog, 0xff, (size_t)S.p * PSTRIDE * sizeof(int), st);   // every word -1
    if (e != hipSuccess) return e;
    if (S.ib == 16) hipLaunchKernelGGL((k_lu_forward_wave<16>), dim3(S.p), dim3(NT), 0, st, S, j, prog);
    else hipLaunchKernelGGL((k_lu_forward_wave<32>), dim3(S.p), dim3(NT), 0, st, S, j, prog);
    return hipGetLastError();
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

template <int IB>
hipError_t launch_run(const Sched &S, bool serial, int workers, hipStream_t st)
{
    if (serial) {
        for (int k = 0; k < S.p; ++k) {
            const int nt = S.p - k - 1;
            hipLaunchKernelGGL((k_lu_step<T_GETRF, IB>), dim3(1), dim3(NT), 0, st, S, k, k);
            if (nt > 0) hipLaunchKernelGGL((k_lu_step<T_GESSM, IB>), dim3(nt), dim3(NT), 0, st, S, k, k);
            for (int i = k + 1; i < S.p; ++i) {
                hipLaunchKernelGGL((k_lu_step<T_TSTRF, IB>), dim3(1), dim3(NT), 0, st, S, k, i);
                hipLaunchKernelGGL((k_lu_step<T_SSSSM, IB>), dim3(nt), dim3(NT), 0, st, S, k, i);
            }
        }
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_lu_worker<IB>), dim3(workers), dim3(NT), 0, st, S);
    return hipGetLastError();
}

// Workgroups of the persistent kernel that fit the device at once.
template <int IB>
int resident_workers(int num_cu)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_lu_worker<IB>, NT, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return std::max(1, num_cu) * per_cu;
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

namespace {

// The factorisation of the column-major n x n matrix A into W's tiles (with
// `extra` further tile columns allocated after the p x p grid, which the
// factorisation does not touch): scheduler set-up, layout in, workers.  On
// return S describes the factor; the status words are not read back.  With
// `timing`, W->ev[0..2] are recorded around the layout and the workers.
int lu_run(Workspace *W, const double *A, int64_t lda, int64_t n, int64_t nb, int64_t ib, int extra, double *Lup,
           int32_t *piv, const tileqr_opts &o, bool timing, hipStream_t st, tl::Sched &S)
{
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
    if ((rc = W->tiles.ensure((size_t)p * (p + extra) * nb * nb * sizeof(double)))) return rc;
    if ((rc = W->luinv.ensure((size_t)p * p * ib * nb * sizeof(double)))) return rc;
    if ((rc = W->status.ensure(256))) return rc;
    if ((rc = W->sched.counters.ensure((size_t)nid * sizeof(int32_t)))) return rc;
    if ((rc = W->sched.qslot.ensure((size_t)off[tl::NQ] * sizeof(int32_t)))) return rc;
    if ((rc = W->sched.qctl.ensure((size_t)(2 * tl::NQ * tl::QSTRIDE + 64) * sizeof(uint32_t)))) return rc;
    if (timing && !W->ev[0])
        for (auto &e : W->ev) TQ_HIP(hipEventCreate(&e));

    S.tiles = (double *)W->tiles.ptr;
    S.lup = Lup;
    S.linv = (double *)W->luinv.ptr;
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
    if (workers <= 0) workers = ib == 16 ? tl::resident_workers<16>(W->num_cu) : tl::resident_workers<32>(W->num_cu);

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
    const hipError_t e = ib == 16 ? tl::launch_run<16>(S, serial, workers, st) : tl::launch_run<32>(S, serial, workers, st);
    if (e != hipSuccess) return hip_fail(e, "tilelu worker");
    return 0;
}

}  // namespace

extern "C" int tilelu_factor(int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib, double *Lup, int32_t *piv,
                             const tileqr_opts *opts, tilelu_info *info)
{
    if (n < 0 || n > (int64_t)INT_MAX / 2) return -1;
    if (n > 0 && !A) return -2;
    if (lda < std::max<int64_t>(1, n)) return -3;
    if (nb <= 0) return -4;
    if (ib <= 0 || nb % ib != 0) return -5;
    if (n > 0 && (!Lup || ((uintptr_t)Lup & 15))) return -6;
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
    const bool timing = (o.flags & TILEQR_FLAG_TIMING) && !(o.flags & TILEQR_FLAG_ASYNC) && info;
    tl::Sched S;
    int rc;
    if ((rc = lu_run(W, A, lda, n, nb, ib, 0, Lup, piv, o, timing, st, S))) return rc;
    const int p = S.p;
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

extern "C" int tilelu_solve(int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B, int64_t ldb,
                            double *X, int64_t ldx, int64_t ib, const tileqr_opts *opts, tilelu_solve_info *info)
{
    if (n < 0 || n > (int64_t)INT_MAX / 2) return -1;
    if (nrhs < 0 || nrhs > (int64_t)INT_MAX / 2) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    if (n > 0 && nrhs > 0 && !B) return -5;
    if (ldb < std::max<int64_t>(1, n)) return -6;
    if (n > 0 && nrhs > 0 && !X) return -7;
    if (ldx < std::max<int64_t>(1, n)) return -8;
    if (ib != 0 && ib != 16 && ib != 32) return -9;
    tileqr_opts o;
    tileqr_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision < TILEQR_FP64 || o.precision > TILEQR_BF16X3 || o.max_iter < 0 || o.max_iter > 64) return -10;
    if (info) {
        info->iterations = 0;
        info->converged = 0;
        info->eta = 0.0;
        info->minor = 0;
    }
    if (o.precision != TILEQR_FP64 || (o.flags & TILEQR_FLAG_ASYNC)) return TILEQR_EUNSUPPORTED;
    if (ib == 0) ib = 16;
    if (n == 0 || nrhs == 0) {
        if (info) info->converged = 1;
        return TILEQR_OK;
    }
    const double tol = o.tol > 0.0 ? o.tol : 1e-14;

    std::lock_guard<std::mutex> lock(g_mu);
    hipStream_t st = (hipStream_t)o.stream;
    Workspace *W = workspace(st);
    if (!W) return hip_fail(hipErrorNoDevice, "workspace");
    const int64_t nb = tl::NB;
    const int p = (int)cdiv(n, nb);
    const int ldt = (int)nb;   // the right-hand sides' tile column: row blocks of nb rows, nb wide
    const size_t slot = (size_t)p * nb * nb;
    const int64_t part_cap = std::max<int64_t>(n * 32 * 16, 1 << 20);
    constexpr int64_t SMALL = 1024, SMALL_CAP = (int64_t)COLSQ_BLOCKS * 64;
    const int64_t flags_cap = trsm_flags_needed(n, ldt);
    int rc;
    if ((rc = W->lulup.ensure(tilelu_lup_size(n, nb, ib) * sizeof(double)))) return rc;
    if ((rc = W->lupiv.ensure(tilelu_piv_size(n, nb) * sizeof(int32_t)))) return rc;
    if ((rc = W->solve.ensure(3 * slot * sizeof(double)))) return rc;
    if ((rc = W->part.ensure((size_t)part_cap * sizeof(double)))) return rc;
    if ((rc = W->misc.ensure((size_t)(SMALL + SMALL_CAP) * sizeof(double)))) return rc;
    if ((rc = W->tflags.ensure((size_t)flags_cap * sizeof(int32_t)))) return rc;
    if ((rc = W->prog.ensure((size_t)p * tl::PSTRIDE * sizeof(int32_t)))) return rc;
    const bool serial = (o.flags & TILEQR_FLAG_SERIAL) != 0;

    tl::Sched S;
    if ((rc = lu_run(W, A, lda, n, nb, ib, 1, (double *)W->lulup.ptr, (int32_t *)W->lupiv.ptr, o, false, st, S)))
        return rc;
    int32_t *tst = S.status + 48;   // the triangular solves' status word (STATUS_* bits)
    TQ_HIP(hipMemsetAsync(tst, 0, sizeof(int32_t), st));
    TQ_HIP(hipMemcpyAsync(W->host_small, S.status, 33 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    TQ_HIP(hipStreamSynchronize(st));
    {
        const int32_t *hs = (const int32_t *)W->host_small;
        if (hs[0] & tl::ST_NONFINITE) return TILEQR_ENONFINITE;
        if (hs[0] & tl::ST_SINGULAR) {
            if (info) info->minor = hs[32];
            return TILEQR_ESINGULAR;
        }
        if (hs[0] & tl::ST_TIMEOUT) return TILEQR_ETIMEOUT;
    }
    double *Bc = S.tiles + (size_t)p * p * nb * nb;   // tile column p
    double *Xr = (double *)W->solve.ptr, *Rr = Xr + slot, *Xb = Rr + slot;
    double *small = (double *)W->misc.ptr, *part = (double *)W->part.ptr;
    // Bc <- A^{-1} Bc: the factor's transformations, then U.
    auto solve_bc = [&]() -> hipError_t {
        hipError_t e = tl::launch_forward(S, p, (int *)W->prog.ptr, serial, st);
        if (e != hipSuccess) return e;
        return launch_trsm((int)nb, S.tiles, p, n, Bc, ldt, true, (int *)W->tflags.ptr, flags_cap, tst, S.spin_limit,
                           st);
    };
    TQ_HIP(launch_norm_inf(A, lda, n, n, part, part_cap, small, st));
    int max_it = 0;
    double max_eta = 0.0;
    bool all_conv = true;
    // One block of at most 64 right-hand sides (columns Bb of B, Xo of X).
    auto solve_block = [&](const double *Bb, double *Xo, int nr) -> int {
        TQ_HIP(launch_cm2rows(Bb, ldb, n, nr, Bc, (int64_t)p * nb, ldt, st));
        TQ_HIP(solve_bc());
        TQ_HIP(hipMemcpyAsync(Xr, Bc, slot * sizeof(double), hipMemcpyDeviceToDevice, st));
        // Classical refinement in FP64 (Section 3.2.4's check of the backward
        // error, then corrections through the factor) until the largest
        // ||b - A x||_inf / (||A||_inf ||x||_inf) over the columns is <= tol,
        // max_iter corrections, or two corrections that fail to halve it; the
        // best iterate is returned.
        double best = INFINITY, prev = INFINITY;
        int it = 0, stall = 0;
        bool conv = false;
        for (;;) {
            TQ_HIP(launch_cm2rows(Bb, ldb, n, nr, Rr, (int64_t)p * nb, ldt, st));
            TQ_HIP(launch_gemv_n(A, lda, n, n, Xr, ldt, nr, -1.0, 1.0, Rr, part, part_cap, st));
            TQ_HIP(launch_colmax(Rr, ldt, n, nr, small + SMALL, SMALL_CAP, small + 256, st));
            TQ_HIP(launch_colmax(Xr, ldt, n, nr, small + SMALL, SMALL_CAP, small + 320, st));
            TQ_HIP(hipMemcpyAsync(W->host_small, small, 384 * sizeof(double), hipMemcpyDeviceToHost, st));
            TQ_HIP(hipMemcpyAsync(W->host_status, tst, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            TQ_HIP(hipMemcpyAsync(W->host_status + 1, S.status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            TQ_HIP(hipStreamSynchronize(st));
            if (*W->host_status & STATUS_SINGULAR) return TILEQR_ESINGULAR;
            if ((*W->host_status & STATUS_TIMEOUT) || (W->host_status[1] & tl::ST_TIMEOUT)) return TILEQR_ETIMEOUT;
            const double *hs = W->host_small, normA = hs[0];
            double eta = 0.0;
            for (int c = 0; c < nr; ++c) {
                const double r = hs[256 + c], d = normA * hs[320 + c];
                eta = std::max(eta, d > 0.0 ? r / d : (r > 0.0 ? INFINITY : 0.0));
            }
            if (eta < best) {
                best = eta;
                TQ_HIP(hipMemcpyAsync(Xb, Xr, slot * sizeof(double), hipMemcpyDeviceToDevice, st));
            }
            if (eta <= tol) {
                conv = true;
                break;
            }
            stall = eta > 0.5 * prev ? stall + 1 : 0;
            prev = eta;
            if (it >= o.max_iter || stall >= 2) break;
            ++it;
            TQ_HIP(hipMemcpyAsync(Bc, Rr, slot * sizeof(double), hipMemcpyDeviceToDevice, st));
            TQ_HIP(solve_bc());
            TQ_HIP(launch_axpy_rows(Bc, Xr, ldt, n, nr, 1, st));
        }
        TQ_HIP(launch_rows2cm(Xo, ldx, n, nr, Xb, ldt, st));
        max_it = std::max(max_it, it);
        max_eta = std::max(max_eta, best);
        all_conv = all_conv && conv;
        return TILEQR_OK;
    };
    for (int64_t c0 = 0; c0 < nrhs; c0 += nb) {
        const int nr = (int)std::min<int64_t>(nb, nrhs - c0);
        if ((rc = solve_block(B + (size_t)c0 * ldb, X + (size_t)c0 * ldx, nr)) != TILEQR_OK) return rc;
    }
    TQ_HIP(hipStreamSynchronize(st));
    if (info) {
        info->iterations = max_it;
        info->converged = all_conv ? 1 : 0;
        info->eta = max_eta;
    }
    return all_conv ? TILEQR_OK : TILEQR_ENOCONV;
}
