// Task graph of the tiled QR (Algorithm 2, Section 3.2.1) as the scheduler
// sees it (Section 4): task ids, in-degrees and successors, shared by the
// persistent GPU scheduler and by the host-side self-check.
//
// Tasks of one p x q tile grid with kmax = min(p, q) steps and NS column
// strips per tile (the GEMM-shaped kernels are column-separable: column c of
// their output depends on column c of their inputs only, so LARFB and SSRFB
// are split into NS strip tasks; GEQRT and TSQRT stay whole):
//   GEQRT(k)            k < kmax
//   TSQRT(k, i)         k < i < p
//   LARFB(k, j, s)      k < j < q, s < NS
//   SSRFB(k, i, j, s)   k < i < p, k < j < q, s < NS
//
// Data each task touches and the task that last wrote it (Algorithm 2 order):
//   GEQRT(k)       tile (k,k)                <- SSRFB(k-1, k, k, *)
//   LARFB(k,j,s)   V_kk, T_kk                <- GEQRT(k)
//                  tile (k,j) strip s        <- SSRFB(k-1, k, j, s)
//   TSQRT(k,i)     R_kk (upper triangle)     <- TSQRT(k, i-1) or GEQRT(k)
//                  tile (i,k)                <- SSRFB(k-1, i, k, *)
//   SSRFB(k,i,j,s) V_ik, T_ik                <- TSQRT(k, i)
//                  tile (k,j) strip s        <- SSRFB(k, i-1, j, s) or LARFB(k, j, s)
//                  tile (i,j) strip s        <- SSRFB(k-1, i, j, s)
// V_kk (strict lower triangle of the diagonal tile) and R_kk (its upper
// triangle) are separate regions: LARFB(k, .) reads the first while the
// TSQRT(k, .) chain rewrites the second, so they do not wait for each other.
// Every earlier reader of a region is itself a predecessor of its next
// writer, so these read-after-write edges also cover write-after-read.
//
// The paper gives four priority levels, GEQRT > TSQRT > LARFB > SSRFB
// (Section 4): the nodes with more outgoing edges come first.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define TQ_HD __host__ __device__ inline
#else
#define TQ_HD inline
#endif

namespace tq {

enum TaskType { GEQRT = 0, TSQRT = 1, LARFB = 2, SSRFB = 3 };

struct Grid {
    int32_t p, q, kmax, ns;   // tile rows, tile columns, steps, strips per tile
    int64_t baseT, baseL, baseS, total;  // id ranges of the four types
};

struct Task {
    int32_t type, k, i, j, s;
};

TQ_HD Grid make_grid(int32_t p, int32_t q, int32_t ns)
{
    Grid g;
    g.p = p;
    g.q = q;
    g.kmax = p < q ? p : q;
    g.ns = ns;
    g.baseT = g.kmax;
    g.baseL = g.baseT + (int64_t)g.kmax * p;
    g.baseS = g.baseL + (int64_t)g.kmax * q * ns;
    g.total = g.baseS + (int64_t)g.kmax * p * q * ns;
    return g;
}

// Dense id space with holes (ids of impossible index combinations, e.g.
// i <= k, are never used); decoding is plain division.
TQ_HD int64_t id_geqrt(const Grid &g, int k) { return k; }
TQ_HD int64_t id_tsqrt(const Grid &g, int k, int i) { return g.baseT + (int64_t)k * g.p + i; }
TQ_HD int64_t id_larfb(const Grid &g, int k, int j, int s)
{
    return g.baseL + ((int64_t)k * g.q + j) * g.ns + s;
}
TQ_HD int64_t id_ssrfb(const Grid &g, int k, int i, int j, int s)
{
    return g.baseS + (((int64_t)k * g.p + i) * g.q + j) * g.ns + s;
}

TQ_HD Task decode(const Grid &g, int64_t id)
{
    Task t;
    t.i = t.j = t.s = 0;
    if (id < g.baseT) {
        t.type = GEQRT;
        t.k = (int32_t)id;
        t.i = t.j = t.k;
    } else if (id < g.baseL) {
        int64_t r = id - g.baseT;
        t.type = TSQRT;
        t.k = (int32_t)(r / g.p);
        t.i = (int32_t)(r % g.p);
        t.j = t.k;
    } else if (id < g.baseS) {
        int64_t r = id - g.baseL;
        t.type = LARFB;
        t.s = (int32_t)(r % g.ns);
        r /= g.ns;
        t.j = (int32_t)(r % g.q);
        t.k = (int32_t)(r / g.q);
        t.i = t.k;
    } else {
        int64_t r = id - g.baseS;
        t.type = SSRFB;
        t.s = (int32_t)(r % g.ns);
        r /= g.ns;
        t.j = (int32_t)(r % g.q);
        r /= g.q;
        t.i = (int32_t)(r % g.p);
        t.k = (int32_t)(r / g.p);
    }
    return t;
}

// True when the id names a task of the grid (not a hole).
TQ_HD bool valid(const Grid &g, const Task &t)
{
    if (t.k < 0 || t.k >= g.kmax) return false;
    switch (t.type) {
    case GEQRT: return true;
    case TSQRT: return t.i > t.k && t.i < g.p;
    case LARFB: return t.j > t.k && t.j < g.q && t.s < g.ns;
    default: return t.i > t.k && t.i < g.p && t.j > t.k && t.j < g.q && t.s < g.ns;
    }
}

// Number of predecessors that release the task (see the table above).
TQ_HD int32_t indegree(const Grid &g, const Task &t)
{
    const int prev = t.k > 0 ? 1 : 0;
    switch (t.type) {
    case GEQRT: return prev * g.ns;
    case TSQRT: return 1 + prev * g.ns;
    case LARFB: return 1 + prev;
    default: return 2 + prev;
    }
}

// Consumer at step k+1 of tile (i, j) strip s once SSRFB(k, i, j, s) has
// written it; -1 when step k+1 does not exist.
TQ_HD int64_t next_step_consumer(const Grid &g, int k, int i, int j, int s)
{
    const int k1 = k + 1;
    if (k1 >= g.kmax) return -1;
    if (i == k1 && j == k1) return id_geqrt(g, k1);
    if (i == k1) return id_larfb(g, k1, j, s);
    if (j == k1) return id_tsqrt(g, k1, i);
    return id_ssrfb(g, k1, i, j, s);
}

// Successors of a task.  GEQRT and TSQRT fan out to a whole tile row of strip
// tasks; `nsucc` tells how many, `succ(n)` gives the n-th.  Pure functions
// of the task, so the threads of a workgroup can release successors in
// parallel.
TQ_HD int32_t nsucc(const Grid &g, const Task &t)
{
    switch (t.type) {
    case GEQRT: return (g.q - t.k - 1) * g.ns + (t.k + 1 < g.p ? 1 : 0);
    case TSQRT: return (g.q - t.k - 1) * g.ns + (t.i + 1 < g.p ? 1 : 0);
    case LARFB: return t.k + 1 < g.p ? 1 : 0;
    default: {
        int n = t.i + 1 < g.p ? 1 : 0;
        return n + (next_step_consumer(g, t.k, t.i, t.j, t.s) >= 0 ? 1 : 0);
    }
    }
}

TQ_HD int64_t succ(const Grid &g, const Task &t, int32_t n)
{
    const int row = (g.q - t.k - 1) * g.ns;   // strip tasks of the tile row
    switch (t.type) {
    case GEQRT:
        if (n < row) return id_larfb(g, t.k, t.k + 1 + n / g.ns, n % g.ns);
        return id_tsqrt(g, t.k, t.k + 1);
    case TSQRT:
        if (n < row) return id_ssrfb(g, t.k, t.i, t.k + 1 + n / g.ns, n % g.ns);
        return id_tsqrt(g, t.k, t.i + 1);
    case LARFB:
        return id_ssrfb(g, t.k, t.k + 1, t.j, t.s);
    default:
        if (n == 0 && t.i + 1 < g.p) return id_ssrfb(g, t.k, t.i + 1, t.j, t.s);
        return next_step_consumer(g, t.k, t.i, t.j, t.s);
    }
}

// Ready-queue level of a task (0 is served first).  The paper ranks GEQRT >
// TSQRT > LARFB > SSRFB because nodes with more outgoing edges put more
// tasks in the ready state (Section 4).  Inside the LARFB/SSRFB levels the
// same criterion singles out the updates of tile column k+1: they feed the
// next step's GEQRT and TSQRT chain, whose fan-out is the widest of the
// graph, so they form their own level ahead of the other updates.
constexpr int NLEVEL = 5;

TQ_HD int priority_level(const Task &t)
{
    switch (t.type) {
    case GEQRT: return 0;
    case TSQRT: return 1;
    case LARFB: return t.j == t.k + 1 ? 2 : 3;
    default: return t.j == t.k + 1 ? 2 : 4;
    }
}

// Ready queues.  The two panel levels have one queue each; each update
// level has one queue per XCD (8 on MI355X), and a strip task always goes to
// the queue of XCD (matrix + 8 j ns + s)-hash of its tile-column strip, so
// successive updates of one strip run where its data already sits in L2 and
// the workers of one XCD only contend among themselves.
constexpr int NXQ = 8;
constexpr int NQUEUE = 2 + (NLEVEL - 2) * NXQ;

TQ_HD int queue_index(int level, int x) { return level < 2 ? level : 2 + (level - 2) * NXQ + x; }

TQ_HD int queue_of(const Task &t, int ns, int mat)
{
    const int level = priority_level(t);
    const int x = (int)(((unsigned)mat * 5u + (unsigned)t.j * (unsigned)ns + (unsigned)t.s) % NXQ);
    return queue_index(level, x);
}

// Tasks of each ready queue for one matrix (number `mat` of a batch),
// counted by index ranges rather than by decoding every id: the capacities
// the scheduler gives the queues.  Adds to counts[0 .. NQUEUE-1].
inline void count_queue_tasks(const Grid &g, int mat, int64_t *counts)
{
    for (int k = 0; k < g.kmax; ++k) {
        const int64_t rows = g.p - k - 1;   // TSQRT(k, .), and SSRFB(k, ., j, s) per (j, s)
        counts[queue_index(0, 0)] += 1;
        counts[queue_index(1, 0)] += rows;
        for (int j = k + 1; j < g.q; ++j)
            for (int s = 0; s < g.ns; ++s) {
                Task t;
                t.k = k;
                t.j = j;
                t.s = s;
                t.i = k;
                t.type = LARFB;
                counts[queue_of(t, g.ns, mat)] += 1;
                t.type = SSRFB;
                t.i = k + 1;
                counts[queue_of(t, g.ns, mat)] += rows;   // the queue does not depend on i
            }
    }
}

// Leading-order flops of one task (Section 3.2.3: SSRFB costs 4b^3 + sb^2;
// GEQRT 4b^3/3, TSQRT and LARFB 2b^3), for a strip task its share.
TQ_HD double task_flops(const Task &t, int nb, int ib, int ns)
{
    const double b = nb, s = ib;
    switch (t.type) {
    case GEQRT: return 4.0 * b * b * b / 3.0;
    case TSQRT: return 2.0 * b * b * b;
    case LARFB: return 2.0 * b * b * b / ns;
    default: return (4.0 * b * b * b + s * b * b) / ns;
    }
}

}  // namespace tq
