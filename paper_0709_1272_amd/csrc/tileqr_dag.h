// Task graph of the tiled QR (Algorithm 2, Section 3.2.1) as the scheduler
// sees it (Section 4): task ids, in-degrees and successors, shared by the
// persistent GPU scheduler and by the host-side self-check.
//
// Tasks of one p x q tile grid with kmax = min(p, q) steps, NS column
// strips per tile and NP inner panels per tile (ib-column blocks, Section
// 3.2.3).  The GEMM-shaped kernels are column-separable (column c of their
// output depends on column c of their inputs only), so LARFB and SSRFB are
// split into NS strip tasks.  GEQRT and TSQRT are split into their NP inner
// panels: panel l factors columns [l ib, (l+1) ib) of its tile and applies
// its block reflector to the columns right of it, which is exactly the l-th
// pass of the tile kernel's own loop.
//   GEQRT(k, l)         k < kmax, l < NP
//   TSQRT(k, i, l)      k < i < p, l < NP
//   LARFB(k, j, s)      k < j < q, s < NS
//   SSRFB(k, i, j, s)   k < i < p, k < j < q, s < NS
//   PUPD(k, i, l, s)    k <= i < p, l < s < NP   (only when NP == NS > 1)
// With one panel per strip (ib equal to the strip width), a panel task only
// factors its panel and forms its T, and the application of that panel's
// reflector to each later strip s of the same tile (GEQRT, i == k) or tile
// pair (TSQRT, i > k: the panel's R rows and strip s of A_ik) is a task of
// its own, PUPD.  The chain of panels of one tile then carries one
// factorisation and one strip update per link instead of a whole trailing
// update, and TSQRT(k, i+1, l) waits only for the R triangle of panel l.
//
// Data each task touches and the task that last wrote it (Algorithm 2 order):
//   GEQRT(k,l)     tile (k,k) rows >= l ib  <- GEQRT(k, l-1), or SSRFB(k-1, k, k, *) for l = 0
//   LARFB(k,j,s)   V_kk, T_kk                <- GEQRT(k, NP-1) (and so every panel)
//                  tile (k,j) strip s        <- SSRFB(k-1, k, j, s)
//   TSQRT(k,i,l)   R_kk rows of panel l      <- TSQRT(k, i-1, l) or GEQRT(k, l)
//                  tile (i,k) columns >= l ib <- TSQRT(k, i, l-1), or SSRFB(k-1, i, k, *) for l = 0
//   SSRFB(k,i,j,s) V_ik, T_ik                <- TSQRT(k, i, NP-1)
//                  tile (k,j) strip s        <- SSRFB(k, i-1, j, s) or LARFB(k, j, s)
//                  tile (i,j) strip s        <- SSRFB(k-1, i, j, s)
// With PUPD tasks (strip s = panel s):
//   GEQRT(k,l)     tile (k,k) strip l rows >= l ib <- PUPD(k, k, l-1, l), or SSRFB(k-1, k, k, 0) for l = 0
//   TSQRT(k,i,l)   R_kk triangle of panel l  <- TSQRT(k, i-1, l) or GEQRT(k, l)
//                  tile (i,k) strip l        <- PUPD(k, i, l-1, l), or SSRFB(k-1, i, k, 0) for l = 0
//   PUPD(k,i,l,s)  V and T of panel l of tile (i,k) <- GEQRT(k, l) / TSQRT(k, i, l)
//                  strip s of tile (i,k) (rows >= l ib for i = k) <- PUPD(k, i, l-1, s), or
//                                          SSRFB(k-1, i, k, s) for l = 0
//                  R rows of panel l in strip s (i > k) <- PUPD(k, i-1, l, s)
// R rows of panel l are final for GEQRT(k, .) once its panel l is done: the
// later panels touch only rows below them.  The TSQRT(k, ., l) tasks rewrite
// only those rows of R_kk, so the panel chains of one step form a wavefront
// over (i, l): TSQRT(k, i, l) may run beside TSQRT(k, i+1, l-1) and
// GEQRT(k, l+1).  V_kk (strict lower triangle of the diagonal tile) and R_kk
// (its upper triangle) are separate regions: LARFB(k, .) reads the first
// while the TSQRT(k, .) chain rewrites the second, so they do not wait for
// each other.  Every earlier reader of a region is itself a predecessor of
// its next writer, so these read-after-write edges also cover
// write-after-read.
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

enum TaskType { GEQRT = 0, TSQRT = 1, LARFB = 2, SSRFB = 3, PUPD = 4 };
constexpr int NTYPE = 5;

struct Grid {
    int32_t p, q, kmax, ns, np;   // tile rows, tile columns, steps, strips and panels per tile
    int32_t pu;                   // 1: panel updates are PUPD tasks (np == ns > 1)
    int64_t baseT, baseL, baseS, baseU, total;  // id ranges of the five types
};

// One task; l is the inner panel of GEQRT, TSQRT and PUPD (0 for the strip
// tasks), s the strip of LARFB, SSRFB and PUPD; PUPD has j = k.
struct Task {
    int32_t type, k, i, j, s, l;
};

TQ_HD Grid make_grid(int32_t p, int32_t q, int32_t ns, int32_t np)
{
    Grid g;
    g.p = p;
    g.q = q;
    g.kmax = p < q ? p : q;
    g.ns = ns;
    g.np = np;
    g.pu = (np > 1 && np == ns) ? 1 : 0;
    g.baseT = (int64_t)g.kmax * np;
    g.baseL = g.baseT + (int64_t)g.kmax * p * np;
    g.baseS = g.baseL + (int64_t)g.kmax * q * ns;
    g.baseU = g.baseS + (int64_t)g.kmax * p * q * ns;
    g.total = g.baseU + (g.pu ? (int64_t)g.kmax * p * np * np : 0);
    return g;
}

// Dense id space with holes (ids of impossible index combinations, e.g.
// i <= k, are never used); decoding is plain division.
TQ_HD int64_t id_geqrt(const Grid &g, int k, int l) { return (int64_t)k * g.np + l; }
TQ_HD int64_t id_tsqrt(const Grid &g, int k, int i, int l) { return g.baseT + ((int64_t)k * g.p + i) * g.np + l; }
TQ_HD int64_t id_larfb(const Grid &g, int k, int j, int s)
{
    return g.baseL + ((int64_t)k * g.q + j) * g.ns + s;
}
TQ_HD int64_t id_ssrfb(const Grid &g, int k, int i, int j, int s)
{
    return g.baseS + (((int64_t)k * g.p + i) * g.q + j) * g.ns + s;
}
TQ_HD int64_t id_pupd(const Grid &g, int k, int i, int l, int s)
{
    return g.baseU + (((int64_t)k * g.p + i) * g.np + l) * g.np + s;
}
// The panel task of panel l of tile (i, k): GEQRT on the diagonal tile.
TQ_HD int64_t id_panel(const Grid &g, int k, int i, int l)
{
    return i == k ? id_geqrt(g, k, l) : id_tsqrt(g, k, i, l);
}

TQ_HD Task decode(const Grid &g, int64_t id)
{
    Task t;
    t.i = t.j = t.s = t.l = 0;
    if (id < g.baseT) {
        t.type = GEQRT;
        t.k = (int32_t)(id / g.np);
        t.l = (int32_t)(id % g.np);
        t.i = t.j = t.k;
    } else if (id < g.baseL) {
        int64_t r = id - g.baseT;
        t.type = TSQRT;
        t.l = (int32_t)(r % g.np);
        r /= g.np;
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
    } else if (id < g.baseU) {
        int64_t r = id - g.baseS;
        t.type = SSRFB;
        t.s = (int32_t)(r % g.ns);
        r /= g.ns;
        t.j = (int32_t)(r % g.q);
        r /= g.q;
        t.i = (int32_t)(r % g.p);
        t.k = (int32_t)(r / g.p);
    } else {
        int64_t r = id - g.baseU;
        t.type = PUPD;
        t.s = (int32_t)(r % g.np);
        r /= g.np;
        t.l = (int32_t)(r % g.np);
        r /= g.np;
        t.i = (int32_t)(r % g.p);
        t.k = (int32_t)(r / g.p);
        t.j = t.k;
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
    case SSRFB: return t.i > t.k && t.i < g.p && t.j > t.k && t.j < g.q && t.s < g.ns;
    default: return g.pu && t.i >= t.k && t.i < g.p && t.l < t.s && t.s < g.np;
    }
}

// Number of predecessors that release the task (see the table above).
TQ_HD int32_t indegree(const Grid &g, const Task &t)
{
    const int prev = t.k > 0 ? 1 : 0;
    // Without PUPD the first panel waits for every strip of its tile, with
    // them for strip 0 only.
    const int first = g.pu ? prev : prev * g.ns;
    switch (t.type) {
    case GEQRT: return t.l > 0 ? 1 : first;
    case TSQRT: return 1 + (t.l > 0 ? 1 : first);
    case LARFB: return 1 + prev;
    case SSRFB: return 2 + prev;
    default: return 1 + (t.i > t.k ? 1 : 0) + (t.l > 0 ? 1 : prev);
    }
}

// Consumer at step k+1 of tile (i, j) strip s once SSRFB(k, i, j, s) has
// written it; -1 when step k+1 does not exist.
TQ_HD int64_t next_step_consumer(const Grid &g, int k, int i, int j, int s)
{
    const int k1 = k + 1;
    if (k1 >= g.kmax) return -1;
    if (j == k1) return (g.pu && s > 0) ? id_pupd(g, k1, i, 0, s) : id_panel(g, k1, i, 0);
    if (i == k1) return id_larfb(g, k1, j, s);
    return id_ssrfb(g, k1, i, j, s);
}

// Successors of a task.  The last panel of a GEQRT or TSQRT fans out to a
// whole tile row of strip tasks; `nsucc` tells how many, `succ(n)` gives the
// n-th.  Pure functions of the task, so the threads of a workgroup can
// release successors in parallel.  A panel task lists the next panel of its
// own tile first, then the same panel of the next tile, then the strips.
// With PUPD tasks a panel task lists the same panel of the next tile, then
// its strip updates, then (last panel) the strips; a PUPD lists the next
// panel task of its strip (or the strip's update by the next panel), then
// the same update of the next tile.
TQ_HD int32_t nsucc(const Grid &g, const Task &t)
{
    const int strips = (g.q - t.k - 1) * g.ns;
    const int more = t.l + 1 < g.np ? 1 : 0;
    if (g.pu) {
        const int last = more ? 0 : strips;
        switch (t.type) {
        case GEQRT: return (t.k + 1 < g.p ? 1 : 0) + (g.np - 1 - t.l) + last;
        case TSQRT: return (t.i + 1 < g.p ? 1 : 0) + (g.np - 1 - t.l) + last;
        case PUPD: return 1 + (t.i + 1 < g.p ? 1 : 0);
        default: break;
        }
    }
    switch (t.type) {
    case GEQRT: return more + (t.k + 1 < g.p ? 1 : 0) + (more ? 0 : strips);
    case TSQRT: return more + (t.i + 1 < g.p ? 1 : 0) + (more ? 0 : strips);
    case LARFB: return t.k + 1 < g.p ? 1 : 0;
    default: {
        int n = t.i + 1 < g.p ? 1 : 0;
        return n + (next_step_consumer(g, t.k, t.i, t.j, t.s) >= 0 ? 1 : 0);
    }
    }
}

TQ_HD int64_t succ(const Grid &g, const Task &t, int32_t n)
{
    const bool more = t.l + 1 < g.np;
    if (g.pu && t.type != LARFB && t.type != SSRFB) {
        if (t.type == PUPD) {
            if (n == 0) return t.s == t.l + 1 ? id_panel(g, t.k, t.i, t.l + 1) : id_pupd(g, t.k, t.i, t.l + 1, t.s);
            return id_pupd(g, t.k, t.i + 1, t.l, t.s);
        }
        if (t.i + 1 < g.p) {
            if (n == 0) return id_tsqrt(g, t.k, t.i + 1, t.l);
            --n;
        }
        if (n < g.np - 1 - t.l) return id_pupd(g, t.k, t.i, t.l, t.l + 1 + n);
        n -= g.np - 1 - t.l;
        return t.type == GEQRT ? id_larfb(g, t.k, t.k + 1 + n / g.ns, n % g.ns)
                               : id_ssrfb(g, t.k, t.i, t.k + 1 + n / g.ns, n % g.ns);
    }
    switch (t.type) {
    case GEQRT:
        if (more) {
            if (n == 0) return id_geqrt(g, t.k, t.l + 1);
            --n;
        }
        if (t.k + 1 < g.p) {
            if (n == 0) return id_tsqrt(g, t.k, t.k + 1, t.l);
            --n;
        }
        return id_larfb(g, t.k, t.k + 1 + n / g.ns, n % g.ns);
    case TSQRT:
        if (more) {
            if (n == 0) return id_tsqrt(g, t.k, t.i, t.l + 1);
            --n;
        }
        if (t.i + 1 < g.p) {
            if (n == 0) return id_tsqrt(g, t.k, t.i + 1, t.l);
            --n;
        }
        return id_ssrfb(g, t.k, t.i, t.k + 1 + n / g.ns, n % g.ns);
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
    case SSRFB: return t.j == t.k + 1 ? 2 : 4;
    default: return 2;   // PUPD: on the panel chain
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
        const int64_t rows = g.p - k - 1;   // TSQRT(k, ., l) per l, and SSRFB(k, ., j, s) per (j, s)
        counts[queue_index(0, 0)] += g.np;
        counts[queue_index(1, 0)] += rows * g.np;
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
        if (g.pu) {
            // PUPD(k, i, l, s) for k <= i < p, l < s: s (i, l) pairs per row
            for (int s = 1; s < g.np; ++s) {
                Task t;
                t.type = PUPD;
                t.k = t.j = t.i = k;
                t.l = 0;
                t.s = s;
                counts[queue_of(t, g.ns, mat)] += (rows + 1) * s;
            }
        }
    }
}

// Leading-order flops of one task (Section 3.2.3: SSRFB costs 4b^3 + sb^2;
// GEQRT 4b^3/3, TSQRT and LARFB 2b^3), for a strip or panel task an equal
// share of its tile kernel's.
TQ_HD double task_flops(const Task &t, int nb, int ib, int ns, int np)
{
    const double b = nb, s = ib;
    switch (t.type) {
    case GEQRT: return 4.0 * b * b * b / 3.0 / np;
    case TSQRT: return 2.0 * b * b * b / np;
    case LARFB: return 2.0 * b * b * b / ns;
    case SSRFB: return (4.0 * b * b * b + s * b * b) / ns;
    default: return 4.0 * b * s * s;   // PUPD: one ib-wide panel on one strip (ib = strip width)
    }
}

}  // namespace tq
