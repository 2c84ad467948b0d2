// Tree reduction of the panel for tall matrices, an extension beyond the
// paper: Algorithm 2 (Section 3.2.1) reduces every panel with a flat chain of
// TSQRT, one tile below the other, so a matrix of p tile rows has a chain of
// p tasks per step.  Here the rows are cut into L leaves; each leaf is
// factored by Algorithm 2 on its own (all leaves in one persistent launch of
// the batched scheduler, one task per inner panel, so the chains of the
// leaves run side by side), and the leaves' R triangles are then merged in a
// tree of fan-in up to four (the merges of a level in one batched launch): a
// merge factors the stack [R_1; ...; R_k] (kn x n) of its children's upper
// triangles with the same tile kernels (the zeros below each triangle's
// diagonal stay exactly zero through TSQRT and SSRFB, whose reflectors are
// zero there), and its R is the node's R.  Q^T is applied in the same order:
// each leaf's Q^T on its rows, then every merge's Q^T on the first n rows of
// its children (a node's rows are the first n rows of its leftmost leaf).
#include "tileqr_host.h"

#include <algorithm>
#include <vector>

using namespace tq;

namespace tq {

namespace {

struct TreeLeaf {
    int64_t r0, rows;
    size_t toff;   // T of the leaf in F
};
constexpr int kFanIn = 4;   // children per merge
struct TreeMerge {
    std::vector<int> kids;   // nodes (leftmost leaves) merged; the result is node kids[0]
    int level;
    size_t soff;   // the kn x n stacked matrix in F (leading dimension kn)
    size_t toff;   // its T in F
};
struct TreePlan {
    std::vector<TreeLeaf> leaves;
    std::vector<TreeMerge> merges;
    int levels = 0;
    size_t total = 0;
};

// Leaves of h rows (h the largest multiple of nb with L h <= m; the last
// leaf takes the rest), merged level by level in groups of up to kFanIn (a
// group of one passes up unchanged).  False if a leaf would have fewer than
// max(n, nb) rows.
bool make_plan(int64_t m, int64_t n, int64_t nb, int64_t ib, int64_t L, TreePlan &P)
{
    if (L < 1 || m < n || n < 1) return false;
    const int64_t h = (m / L) / nb * nb;
    if (h < std::max(n, nb)) return false;
    P = TreePlan();
    for (int64_t i = 0; i < L; ++i) {
        TreeLeaf f;
        f.r0 = i * h;
        f.rows = i + 1 < L ? h : m - i * h;
        f.toff = P.total;
        P.total += tileqr_t_size(f.rows, n, nb, ib);
        P.leaves.push_back(f);
    }
    std::vector<int> nodes;
    for (int i = 0; i < (int)L; ++i) nodes.push_back(i);
    int level = 0;
    while (nodes.size() > 1) {
        ++level;
        std::vector<int> next;
        for (size_t j = 0; j < nodes.size(); j += kFanIn) {
            const size_t k = std::min<size_t>(kFanIn, nodes.size() - j);
            if (k > 1) {
                TreeMerge g;
                g.kids.assign(nodes.begin() + (long)j, nodes.begin() + (long)(j + k));
                g.level = level;
                g.soff = P.total;
                P.total += (size_t)k * n * n;
                g.toff = P.total;
                P.total += tileqr_t_size((int64_t)k * n, n, nb, ib);
                P.merges.push_back(g);
            }
            next.push_back(nodes[j]);
        }
        nodes.swap(next);
    }
    P.levels = level;
    return true;
}

// dst (n x n) <- the upper triangle of src; below the diagonal zeros
// (zero_lower) or left as it is.  Column-major, one thread per entry.
__global__ void k_copy_upper(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t n, int zero_lower)
{
    for (int64_t c = blockIdx.y; c < n; c += gridDim.y)
        for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
            if (r <= c) dst[c * ldd + r] = src[c * lds + r];
            else if (zero_lower) dst[c * ldd + r] = 0.0;
        }
}

hipError_t copy_upper(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t n, bool zero_lower,
                      hipStream_t st)
{
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(n, 256), 64);
    const unsigned gy = (unsigned)std::min<int64_t>(n, 4096);
    hipLaunchKernelGGL(k_copy_upper, dim3(gx, gy), dim3(256), 0, st, src, lds, dst, ldd, n, zero_lower ? 1 : 0);
    return hipGetLastError();
}

DevBuf g_tree_y;                 // gathered rows of the merges' Q^T
DevBuf g_tree_a, g_tree_b, g_tree_f;   // tileqr_solve_ls_tree's copies and factor

// One batched factorisation of `cnt` matrices (rows[i] x n at A[i], leading
// dimension ld[i], T at T[i]), one task per inner panel.
int factor_group(const std::vector<int64_t> &rows, int64_t n, const std::vector<double *> &A,
                 const std::vector<int64_t> &ld, int64_t nb, int64_t ib, const std::vector<double *> &T,
                 const tileqr_opts &o)
{
    const int64_t cnt = (int64_t)rows.size();
    std::vector<int64_t> nv((size_t)cnt, n), nbv((size_t)cnt, nb), ibv((size_t)cnt, ib);
    tileqr_opts ob = o;
    ob.flags &= ~(unsigned)TILEQR_FLAG_ASYNC;
    if (ob.panel_tasks == 0) ob.panel_tasks = nb / ib;
    if (ob.panel_workers == 0) {
        // A quarter of the CUs for the panel chains of these tall matrices
        // (the batched default gives them more, which starves the updates).
        int dev = 0, cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu >= 8)
            ob.panel_workers = cu / 4;
    }
    return tileqr_factor_batched(cnt, rows.data(), nv.data(), A.data(), ld.data(), nbv.data(), ibv.data(), T.data(),
                                 &ob);
}

}  // namespace

}  // namespace tq

extern "C" size_t tileqr_tree_size(int64_t m, int64_t n, int64_t nb, int64_t ib, int64_t leaves)
{
    TreePlan P;
    if (nb <= 0 || ib <= 0 || nb % ib != 0 || !make_plan(m, n, nb, ib, leaves, P)) return 0;
    return P.total;
}

extern "C" int tileqr_factor_tree(int64_t m, int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib,
                                  int64_t leaves, double *F, const tileqr_opts *opts)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (A == nullptr && n > 0) return -3;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (nb <= 0) return -5;
    if (ib <= 0 || ib > nb || nb % ib != 0) return -6;
    if (n == 0) return TILEQR_OK;
    TreePlan P;
    if (!make_plan(m, n, nb, ib, leaves, P)) return -7;
    if (F == nullptr) return -8;
    tileqr_opts o;
    tileqr_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision != TILEQR_FP64 || (o.flags & (TILEQR_FLAG_SERIAL | TILEQR_FLAG_TRACE)))
        return TILEQR_EUNSUPPORTED;
    if (!tileqr_blocking_supported(nb, ib)) return TILEQR_EUNSUPPORTED;
    hipStream_t us = (hipStream_t)o.stream;
    if (P.leaves.size() == 1) {
        tileqr_opts o1 = o;
        o1.flags &= ~(unsigned)TILEQR_FLAG_ASYNC;
        return tileqr_factor_ex(m, n, A, lda, nb, ib, F + P.leaves[0].toff, &o1);
    }
    int rc;
    // The leaves, in one launch.
    const int L = (int)P.leaves.size();
    {
        std::vector<int64_t> rows, ld;
        std::vector<double *> As, Ts;
        for (const auto &f : P.leaves) {
            rows.push_back(f.rows);
            ld.push_back(lda);
            As.push_back(A + f.r0);
            Ts.push_back(F + f.toff);
        }
        if ((rc = factor_group(rows, n, As, ld, nb, ib, Ts, o))) return rc;
    }
    // The merges, level by level; a node's R is in its leaf's first n rows
    // (leaves) or in the stacked matrix of the merge that made it.
    std::vector<const double *> rsrc((size_t)L);
    std::vector<int64_t> rld((size_t)L, lda);
    for (int i = 0; i < L; ++i) rsrc[(size_t)i] = A + P.leaves[(size_t)i].r0;
    for (int lev = 1; lev <= P.levels; ++lev) {
        std::vector<int64_t> rows, ld;
        std::vector<double *> Ss, Ts;
        for (const auto &g : P.merges) {
            if (g.level != lev) continue;
            double *Sg = F + g.soff;
            const int64_t kn = (int64_t)g.kids.size() * n;
            for (size_t t = 0; t < g.kids.size(); ++t) {
                const int c = g.kids[t];
                TQ_HIP(copy_upper(rsrc[(size_t)c], rld[(size_t)c], Sg + (int64_t)t * n, kn, n, true, us));
            }
            rows.push_back(kn);
            ld.push_back(kn);
            Ss.push_back(Sg);
            Ts.push_back(F + g.toff);
            rsrc[(size_t)g.kids[0]] = Sg;
            rld[(size_t)g.kids[0]] = kn;
        }
        if ((rc = factor_group(rows, n, Ss, ld, nb, ib, Ts, o))) return rc;
    }
    // The root's R into the first n rows of A (leaf 0's reflectors below the
    // diagonal stay).
    TQ_HIP(copy_upper(rsrc[0], rld[0], A, lda, n, false, us));
    TQ_HIP(hipStreamSynchronize(us));
    return TILEQR_OK;
}

namespace {

int apply_tree(bool trans, int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, int64_t nb, int64_t ib,
               int64_t leaves, const double *F, double *B, int64_t ldb)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nrhs < 0) return -3;
    if (A == nullptr && n > 0) return -4;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (nb <= 0) return -6;
    if (ib <= 0 || ib > nb || nb % ib != 0) return -7;
    if (n == 0 || nrhs == 0) return TILEQR_OK;
    TreePlan P;
    if (!make_plan(m, n, nb, ib, leaves, P)) return -8;
    if (F == nullptr) return -9;
    if (B == nullptr) return -10;
    if (ldb < std::max<int64_t>(1, m)) return -11;
    int rc;
    auto leaf_step = [&](const TreeLeaf &f) {
        return trans ? tileqr_apply_qt(f.rows, n, nrhs, A + f.r0, lda, nb, ib, F + f.toff, B + f.r0, ldb)
                     : tileqr_apply_q(f.rows, n, nrhs, A + f.r0, lda, nb, ib, F + f.toff, B + f.r0, ldb);
    };
    if (P.leaves.size() == 1) return leaf_step(P.leaves[0]);
    double *Y;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if ((rc = g_tree_y.ensure((size_t)kFanIn * n * nrhs * sizeof(double)))) return rc;
        Y = (double *)g_tree_y.ptr;
    }
    auto merge_step = [&](const TreeMerge &g) {
        const int64_t k = (int64_t)g.kids.size(), kn = k * n;
        const size_t w = (size_t)n * sizeof(double), sp = (size_t)ldb * sizeof(double);
        const size_t yp = (size_t)kn * sizeof(double);
        for (int64_t t = 0; t < k; ++t)
            TQ_HIP(hipMemcpy2DAsync(Y + t * n, yp, B + P.leaves[(size_t)g.kids[(size_t)t]].r0, sp, w, (size_t)nrhs,
                                    hipMemcpyDeviceToDevice, nullptr));
        const double *Sg = F + g.soff, *Tg = F + g.toff;
        const int r = trans ? tileqr_apply_qt(kn, n, nrhs, Sg, kn, nb, ib, Tg, Y, kn)
                            : tileqr_apply_q(kn, n, nrhs, Sg, kn, nb, ib, Tg, Y, kn);
        if (r) return r;
        for (int64_t t = 0; t < k; ++t)
            TQ_HIP(hipMemcpy2DAsync(B + P.leaves[(size_t)g.kids[(size_t)t]].r0, sp, Y + t * n, yp, w, (size_t)nrhs,
                                    hipMemcpyDeviceToDevice, nullptr));
        TQ_HIP(hipStreamSynchronize(nullptr));
        return 0;
    };
    if (trans) {
        for (const auto &f : P.leaves)
            if ((rc = leaf_step(f))) return rc;
        for (const auto &g : P.merges)
            if ((rc = merge_step(g))) return rc;
    } else {
        for (auto it = P.merges.rbegin(); it != P.merges.rend(); ++it)
            if ((rc = merge_step(*it))) return rc;
        for (const auto &f : P.leaves)
            if ((rc = leaf_step(f))) return rc;
    }
    return TILEQR_OK;
}

}  // namespace

extern "C" int tileqr_apply_qt_tree(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, int64_t nb,
                                    int64_t ib, int64_t leaves, const double *F, double *B, int64_t ldb)
{
    return apply_tree(true, m, n, nrhs, A, lda, nb, ib, leaves, F, B, ldb);
}

extern "C" int tileqr_apply_q_tree(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, int64_t nb,
                                   int64_t ib, int64_t leaves, const double *F, double *B, int64_t ldb)
{
    return apply_tree(false, m, n, nrhs, A, lda, nb, ib, leaves, F, B, ldb);
}

extern "C" int tileqr_solve_ls_tree(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                    const double *B, int64_t ldb, double *X, int64_t ldx, int64_t nb, int64_t ib,
                                    int64_t leaves, const tileqr_opts *opts, double *ms)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nrhs < 0) return -3;
    if (A == nullptr && n > 0) return -4;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (B == nullptr && nrhs > 0) return -6;
    if (ldb < std::max<int64_t>(1, m)) return -7;
    if (X == nullptr && nrhs > 0 && n > 0) return -8;
    if (ldx < std::max<int64_t>(1, n)) return -9;
    if (nb <= 0) return -10;
    if (ib <= 0 || ib > nb || nb % ib != 0) return -11;
    if (ms) *ms = 0.0;
    if (n == 0 || nrhs == 0) return TILEQR_OK;
    const size_t fsz = tileqr_tree_size(m, n, nb, ib, leaves);
    if (fsz == 0) return -12;
    tileqr_opts o;
    tileqr_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision != TILEQR_FP64) return TILEQR_EUNSUPPORTED;
    if (!tileqr_blocking_supported(nb, ib)) return TILEQR_EUNSUPPORTED;
    hipStream_t us = (hipStream_t)o.stream;
    double *Ac, *Bc, *Fc;
    int rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if ((rc = g_tree_a.ensure((size_t)m * n * sizeof(double)))) return rc;
        if ((rc = g_tree_b.ensure((size_t)m * nrhs * sizeof(double)))) return rc;
        if ((rc = g_tree_f.ensure(fsz * sizeof(double)))) return rc;
        Ac = (double *)g_tree_a.ptr;
        Bc = (double *)g_tree_b.ptr;
        Fc = (double *)g_tree_f.ptr;
    }
    if (ms) {
        TQ_HIP(hipEventCreate(&e0));
        TQ_HIP(hipEventCreate(&e1));
        TQ_HIP(hipEventRecord(e0, us));
    }
    TQ_HIP(hipMemcpy2DAsync(Ac, (size_t)m * sizeof(double), A, (size_t)lda * sizeof(double), (size_t)m * sizeof(double),
                            (size_t)n, hipMemcpyDeviceToDevice, us));
    TQ_HIP(hipMemcpy2DAsync(Bc, (size_t)m * sizeof(double), B, (size_t)ldb * sizeof(double), (size_t)m * sizeof(double),
                            (size_t)nrhs, hipMemcpyDeviceToDevice, us));
    tileqr_opts of = o;
    of.flags &= ~(unsigned)TILEQR_FLAG_ASYNC;
    if ((rc = tileqr_factor_tree(m, n, Ac, m, nb, ib, leaves, Fc, &of))) return rc;
    if ((rc = tileqr_apply_qt_tree(m, n, nrhs, Ac, m, nb, ib, leaves, Fc, Bc, m))) return rc;
    // X = R^{-1} (Q^T B)(0:n): R (the first n rows of Ac) as tiles, the
    // right-hand sides as row blocks, the persistent triangular solve.
    {
        std::lock_guard<std::mutex> lock(g_mu);
        Workspace *W = workspace(us);
        if (!W) return hip_fail(hipErrorNoDevice, "workspace");
        const int q = (int)cdiv(n, nb);
        const int ldt = (int)(cdiv(nrhs, kStripWidth) * kStripWidth);
        const int64_t fcap = trsm_flags_needed(n, ldt);
        if ((rc = W->tiles.ensure((size_t)q * q * nb * nb * sizeof(double)))) return rc;
        if ((rc = W->rows.ensure((size_t)q * nb * ldt * sizeof(double)))) return rc;
        if ((rc = W->tflags.ensure((size_t)fcap * sizeof(int)))) return rc;
        if ((rc = W->status.ensure(256))) return rc;
        int *dstatus = (int *)W->status.ptr;
        TQ_HIP(hipMemsetAsync(dstatus, 0, sizeof(int), us));
        TQ_HIP(launch_cm2tile(Ac, m, n, n, (double *)W->tiles.ptr, (int)nb, q, q, dstatus, us));
        TQ_HIP(launch_cm2rows(Bc, m, n, nrhs, (double *)W->rows.ptr, (int64_t)q * nb, ldt, us));
        TQ_HIP(launch_trsm((int)nb, (const double *)W->tiles.ptr, q, n, (double *)W->rows.ptr, ldt, true,
                           (int *)W->tflags.ptr, fcap, dstatus, (int64_t)1 << 26, us));
        TQ_HIP(launch_rows2cm(X, ldx, n, nrhs, (const double *)W->rows.ptr, ldt, us));
        if (ms) TQ_HIP(hipEventRecord(e1, us));
        rc = check_status(W, dstatus, us);
    }
    if (ms) {
        float t = 0.f;
        TQ_HIP(hipEventSynchronize(e1));
        TQ_HIP(hipEventElapsedTime(&t, e0, e1));
        *ms = t;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return rc;
}
