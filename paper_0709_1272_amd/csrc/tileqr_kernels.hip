// Tiled QR kernels instantiated for FP64 arithmetic, the scheduler set-up,
// Q / Q^T application and the layout conversions (Section 3.2.1,
// Algorithm 2; Section 4).  The device building blocks and the storage
// conventions are in tileqr_tile.h.
#include "tileqr_tile.h"

namespace tq {

// Counters <- in-degrees, queues cleared, GEQRT(0, 0) of every matrix queued.
__global__ void k_sched_init(SchedDev S)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t gid = tid0; gid < S.total_ids; gid += stride) {
        const int mi = find_mat(S, gid);
        const MatDev &M = S.mats[mi];
        const Grid g = make_grid(M.p, M.q, S.ns, S.np);
        const Task t = decode(g, gid - M.task_base);
        S.counters[gid] = valid(g, t) ? indegree(g, t) : -1;
    }
    for (int64_t e = tid0; e < S.qslot_total; e += stride) S.qslot[e] = 0;
    for (int64_t e = tid0; e < NQUEUE; e += stride) {
        S.qhead[e * QSTRIDE] = 0;
        S.qtail[e * QSTRIDE] = 0;
    }
    if (tid0 == 0) {
        *S.done = 0;
        *S.trace_count = 0;
    }
}

__global__ void k_sched_seed(SchedDev S)
{
    // Runs after k_sched_init (stream order): queue every GEQRT(0, 0) (id 0
    // of its matrix).
    // Every matrix in the list is non-empty (the host drops empty ones).
    for (int mi = threadIdx.x; mi < S.nmat; mi += blockDim.x)
        S.qslot[S.qoff[queue_index(0, 0)] + mi] = (int32_t)(S.mats[mi].task_base + 1);
    __syncthreads();
    if (threadIdx.x == 0) S.qtail[queue_index(0, 0) * QSTRIDE] = (uint32_t)S.nmat;
}

// -------------------------------------------------- applying Q and Q^T

// B <- Q^T B (TRANS) or Q B for Q of a finished factorisation, B held in
// row blocks of nb rows (row-major, leading dimension D.ldb, a multiple of
// the strip width).  Q^T applies, for k = 0, 1, ..: Q_kk^T to block k, then
// Q_ik^T to blocks (k, i) for i = k+1, k+2, .. (the order in which the
// factorisation applied them to A); Q applies the transposes in reverse.
// Each tile reflector is the product of its nb/ib inner panels, taken in
// groups of D.group consecutive panels, and the work is spread over (step,
// group) pairs: workgroup (k, g) applies the panels of group g of every
// reflector of step k, row block after row block.  Panel l of the TS
// reflector (k, i) touches only rows [l ib, (l+1) ib) of block k and all of
// block i, so workgroup (k, g) on block i waits only for group g-1 (TRANS;
// g+1 for Q) of the same step to have finished block i, and the first group
// of a step for the previous step (in the product's order) to have finished
// it: a wavefront over (row block, group) instead of a chain of whole tiles.
// Larger groups mean fewer links in the wavefront and fewer waits per panel,
// at the price of more work per link; the host picks the size.  A strip of
// a block stays in registers across the group's panels.  Every panel is applied with the same operands
// and in the same order whatever the grouping, so the result does not depend
// on it.  Progress flags (the last block done) sit PROG_STRIDE words apart in
// D.prog, one per (step, group).  A workgroup waits only for lower-numbered
// ones, which were dispatched first, so the waits make progress; every wait
// is bounded.
template <int NB, int IB, bool TRANS>
__global__ __launch_bounds__(2 * NB) void k_apply(ApplyDev D)
{
    __shared__ Smem<NB, IB> sm;
    __shared__ int s_abort;
    using C = Cfg<NB, IB>;
    constexpr int NP = C::NPAN;
    const int tid = threadIdx.x;
    const int kmax = D.kmax, p = D.M.p, G = D.group, NG = NP / G;
    const int sidx = (int)blockIdx.x / NG, gidx = (int)blockIdx.x % NG;
    const int k = TRANS ? sidx : kmax - 1 - sidx;
    const int grp = TRANS ? gidx : NG - 1 - gidx;
    // Panels of the group in the order they are applied: ascending for Q^T,
    // descending for Q.
    auto panel_of = [&](int j) { return TRANS ? grp * G + j : grp * G + G - 1 - j; };
    if (*D.status != 0) return;   // input rejected (non-finite factor)
    const gdouble *tkk = tile_ptr(D.M, NB, k, k);
    gdouble *Bk = (gdouble *)(D.B + (size_t)k * NB * D.ldb);
    // The first group of a step (in the product's order) follows the last
    // group of the previous step; the others follow the neighbouring group of
    // the same step.
    const bool first = gidx == 0;
    const int *pred = nullptr;
    if (!first) pred = &D.prog[(k * NG + (TRANS ? grp - 1 : grp + 1)) * PROG_STRIDE];
    else if (TRANS ? k > 0 : k + 1 < kmax) pred = &D.prog[((TRANS ? k - 1 : k + 1) * NG + (TRANS ? NG - 1 : 0)) * PROG_STRIDE];
    const int nrow = p - k;   // blocks k .. p-1
    // Q^T: k, k+1, .., p-1.   Q: p-1, .., k+1, then k.
    auto row_of = [&](int qq) { return TRANS ? k + qq : (qq + 1 < nrow ? p - 1 - qq : k); };
    auto stage = [&](Stage<NB, IB> &S, int qq, int j) {
        const int r = row_of(qq), l = panel_of(j);
        apply_panel_stage<NB, IB>(S, r == k ? tkk : tile_ptr(D.M, NB, r, k), tblock_ptr(D.M, NB, IB, k, r), l, r == k);
    };
    // Panels are staged one ahead: the first before the first wait, each
    // later one while the previous panel is applied (the factor is final).
    Stage<NB, IB> S;
    stage(S, 0, 0);
    // Rows of block k the group may change: the diagonal panels from the
    // group's lowest one on; rows above it belong to other groups.
    const int rlo_diag = grp * G * IB;
    for (int q = 0; q < nrow; ++q) {
        const int r = row_of(q);
        const bool diag = r == k;
        // Block k under Q never sees step k+1 (which starts at block k+1).
        const bool wait = pred != nullptr && !(first && !TRANS && diag);
        if (tid == 0) {
            int abort = 0;
            if (wait) {
                int64_t spins = 0;
                int backoff = 0;
                for (;;) {
                    const int v = __hip_atomic_load(pred, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (TRANS ? v >= r : v <= r) break;
                    if (__hip_atomic_load(D.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        ++spins > D.spin_limit) {
                        __hip_atomic_fetch_or(D.status, STATUS_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        abort = 1;
                        break;
                    }
                    // Short back-off (up to about 0.4 us between polls): the
                    // predecessor is usually one block ahead.
                    backoff = backoff < 3 ? backoff + 1 : 3;
                    for (int z = 0; z < (1 << backoff); ++z) __builtin_amdgcn_s_sleep(2);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            s_abort = abort;
        }
        __syncthreads();
        if (s_abort) return;
        gdouble *Br = (gdouble *)(D.B + (size_t)r * NB * D.ldb);
        gdouble *x = diag ? Bk : Br;
        const bool last_row = q + 1 == nrow;
#pragma unroll 1
        for (int st = 0; st < D.nstrip; ++st) {
            const int col0 = st * WS;
            // Column blocks of the strip that hold right-hand sides.
            const int cbn = min(CB, (D.ncol - col0 + 15) / 16);
            Strip<NB, IB> X;
            load_strip<NB, IB>(X, x, D.ldb, col0, cbn);
#pragma unroll 1
            for (int j = 0; j < G; ++j) {
                const int l = panel_of(j), c0 = l * IB;
                gdouble *tp = diag ? nullptr : Bk + (size_t)c0 * D.ldb + col0;
                double tv[C::EPT] = {};
                if (!diag) load_top<NB, IB>(tv, tp, D.ldb, 16 * cbn);
                stage_store_rows<NB, IB>(sm, S, diag ? c0 : 0, diag, c0);
                // Stage the next panel: the group's next one, else the first
                // one for the next strip or row (after the very last, reload).
                int qn = q, jn = j + 1;
                if (jn == G) {
                    jn = 0;
                    if (st + 1 == D.nstrip) {
                        if (last_row) jn = G - 1;
                        else qn = q + 1;
                    }
                }
                stage(S, qn, jn);
                apply_panel<NB, IB, TRANS, true>(sm, X, diag ? c0 : 0, tp, D.ldb, cbn, tv);
            }
            store_strip<NB, IB>(X, x, D.ldb, col0, cbn, diag ? rlo_diag : 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&D.prog[(k * NG + grp) * PROG_STRIDE], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Progress flags before an apply, one per (step, panel): -1 for Q^T (rows
// are taken in ascending order), p for Q (descending).
__global__ void k_apply_init(int *prog, int nflag, int p, int trans)
{
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nflag; f += gridDim.x * blockDim.x)
        prog[f * PROG_STRIDE] = trans ? -1 : p;
}

// Column-major (B, ldb) m x nrhs <-> row blocks: Bt[(R) * ldt + c], rows
// R < p nb and columns c < ldt; padding rows and columns are zero.
__global__ void k_cm2rows(const double *B, int64_t ldb, int64_t m, int64_t nrhs, double *Bt, int64_t rows,
                          int ldt)
{
    const int64_t total = rows * ldt;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t R = e / ldt, c = e % ldt;
        Bt[e] = (R < m && c < nrhs) ? B[c * ldb + R] : 0.0;
    }
}

__global__ void k_rows2cm(double *B, int64_t ldb, int64_t m, int64_t nrhs, const double *Bt, int ldt)
{
    const int64_t total = m * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / m, R = e % m;
        B[c * ldb + R] = Bt[R * ldt + c];
    }
}

// ------------------------------------------------------ layout conversion

// Column-major (A, lda) -> zero-padded row-major tiles, one 64 x 64 block
// `blk` of one matrix via an LDS transpose.  Flags NaN/Inf in *status.
__device__ __forceinline__ void cm2tile_block(const double *A, int64_t lda, int64_t m, int64_t n, double *tiles,
                                              int nb, int p, int64_t blk, int *status)
{
    __shared__ double buf[64][65];
    const int sub = nb / 64;
    const int si = (int)(blk % sub), sj = (int)((blk / sub) % sub);
    const int64_t tl = blk / ((int64_t)sub * sub);
    const int ti = (int)(tl % p), tj = (int)(tl / p);
    const int64_t row0 = (int64_t)ti * nb + si * 64, col0 = (int64_t)tj * nb + sj * 64;
    const int t = threadIdx.x;
    bool bad = false;
    for (int it = 0; it < 16; ++it) {
        const int cc = it * 4 + t / 64, rr = t % 64;
        const int64_t r = row0 + rr, c = col0 + cc;
        double v = 0.0;
        if (r < m && c < n) {
            v = A[c * lda + r];
            bad |= !isfinite(v);
        }
        buf[cc][rr] = v;
    }
    if (bad) atomicOr(status, STATUS_NONFINITE);
    __syncthreads();
    double *tile = tiles + ((size_t)tj * p + ti) * (size_t)nb * nb;
    for (int it = 0; it < 16; ++it) {
        const int rr = it * 4 + t / 64, cc = t % 64;
        tile[(size_t)(si * 64 + rr) * nb + sj * 64 + cc] = buf[cc][rr];
    }
}

// Tiles -> column-major (A, lda), entries inside m x n only, one 64 x 64
// block.
__device__ __forceinline__ void tile2cm_block(double *A, int64_t lda, int64_t m, int64_t n, const double *tiles,
                                              int nb, int p, int64_t blk)
{
    __shared__ double buf[64][65];
    const int sub = nb / 64;
    const int si = (int)(blk % sub), sj = (int)((blk / sub) % sub);
    const int64_t tl = blk / ((int64_t)sub * sub);
    const int ti = (int)(tl % p), tj = (int)(tl / p);
    const int64_t row0 = (int64_t)ti * nb + si * 64, col0 = (int64_t)tj * nb + sj * 64;
    const int t = threadIdx.x;
    const double *tile = tiles + ((size_t)tj * p + ti) * (size_t)nb * nb;
    for (int it = 0; it < 16; ++it) {
        const int rr = it * 4 + t / 64, cc = t % 64;
        buf[cc][rr] = tile[(size_t)(si * 64 + rr) * nb + sj * 64 + cc];
    }
    __syncthreads();
    for (int it = 0; it < 16; ++it) {
        const int cc = it * 4 + t / 64, rr = t % 64;
        const int64_t r = row0 + rr, c = col0 + cc;
        if (r < m && c < n) A[c * lda + r] = buf[cc][rr];
    }
}

__global__ __launch_bounds__(256) void k_cm2tile(const double *A, int64_t lda, int64_t m, int64_t n,
                                                 double *tiles, int nb, int p, int q, int *status)
{
    cm2tile_block(A, lda, m, n, tiles, nb, p, blockIdx.x, status);
}

// Skipped when the status flags an error so that A is left as the caller
// gave it.
__global__ __launch_bounds__(256) void k_tile2cm(double *A, int64_t lda, int64_t m, int64_t n,
                                                 const double *tiles, int nb, int p, int q,
                                                 const int *status)
{
    if (*status != 0) return;
    tile2cm_block(A, lda, m, n, tiles, nb, p, blockIdx.x);
}

// Matrix of a batched conversion that owns block `blk` (blocks of the
// matrices are numbered consecutively from D[i].blk0).
__device__ __forceinline__ int conv_owner(const ConvDesc *D, int nmat, int64_t blk)
{
    int lo = 0, hi = nmat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (D[mid].blk0 <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_cm2tile_batched(const ConvDesc *D, int nmat, int nb, int *status)
{
    const int64_t blk = blockIdx.x;
    const ConvDesc &d = D[conv_owner(D, nmat, blk)];
    cm2tile_block(d.A, d.lda, d.m, d.n, d.tiles, nb, d.p, blk - d.blk0, status);
}

// All or nothing: with any input rejected no matrix is written back.
__global__ __launch_bounds__(256) void k_tile2cm_batched(const ConvDesc *D, int nmat, int nb, const int *status)
{
    if (*status != 0) return;
    const int64_t blk = blockIdx.x;
    const ConvDesc &d = D[conv_owner(D, nmat, blk)];
    tile2cm_block(d.A, d.lda, d.m, d.n, d.tiles, nb, d.p, blk - d.blk0);
}

// p[0..n) <- v (a kernel, so that it may sit in a captured graph).
__global__ void k_fill_int(int *p, int n, int v)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) p[e] = v;
}

// A[e] <- uniform(-1, 1) from a counter-based hash of (seed, e): synthetic
// matrices for timing runs only.
__global__ void k_fill_uniform(double *A, int64_t count, uint64_t seed)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t x = seed * 0x9e3779b97f4a7c15ULL + (uint64_t)e;
        x = mix64(x + 0x632be59bd9b4e019ULL);
        A[e] = (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

// ------------------------------------------------------------ host launchers

hipError_t launch_cm2tile(const double *A, int64_t lda, int64_t m, int64_t n, double *tiles, int nb,
                          int p, int q, int *status, hipStream_t st)
{
    const int64_t nblk = (int64_t)p * q * (nb / 64) * (nb / 64);
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cm2tile, dim3((unsigned)nblk), dim3(256), 0, st, A, lda, m, n, tiles, nb, p, q,
                       status);
    return hipGetLastError();
}

hipError_t launch_tile2cm(double *A, int64_t lda, int64_t m, int64_t n, const double *tiles, int nb,
                          int p, int q, const int *status, hipStream_t st)
{
    const int64_t nblk = (int64_t)p * q * (nb / 64) * (nb / 64);
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile2cm, dim3((unsigned)nblk), dim3(256), 0, st, A, lda, m, n, tiles, nb, p, q,
                       status);
    return hipGetLastError();
}

#define TQ_DISPATCH(nb, ib, CALL)                                   \
    do {                                                            \
        if (nb == 64 && ib == 16) { CALL(64, 16); }                 \
        else if (nb == 64 && ib == 32) { CALL(64, 32); }            \
        else if (nb == 128 && ib == 16) { CALL(128, 16); }          \
        else if (nb == 128 && ib == 32) { CALL(128, 32); }          \
        else if (nb == 256 && ib == 16) { CALL(256, 16); }          \
        else if (nb == 256 && ib == 32) { CALL(256, 32); }          \
        else return hipErrorInvalidValue;                           \
    } while (0)

hipError_t launch_cm2tile_batched(const ConvDesc *D, int nmat, int64_t nblk, int nb, int *status, hipStream_t st)
{
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cm2tile_batched, dim3((unsigned)nblk), dim3(256), 0, st, D, nmat, nb, status);
    return hipGetLastError();
}

hipError_t launch_tile2cm_batched(const ConvDesc *D, int nmat, int64_t nblk, int nb, const int *status,
                                  hipStream_t st)
{
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile2cm_batched, dim3((unsigned)nblk), dim3(256), 0, st, D, nmat, nb, status);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int n, int v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)std::min(1024, (n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_uniform(double *A, int64_t count, uint64_t seed, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 16384);
    hipLaunchKernelGGL(k_fill_uniform, dim3((unsigned)blocks), dim3(256), 0, st, A, count, seed);
    return hipGetLastError();
}

hipError_t launch_factor_serial(int nb, int ib, int prec, const MatDev &M, const int *status, hipStream_t st)
{
    if (prec != PREC_FP64) {
        if (ib != 32) return hipErrorInvalidValue;
        if (prec == PREC_BF16X2) return launch_serial_mx<PREC_BF16X2>(nb, M, status, st);
        if (prec == PREC_FP16X2) return launch_serial_mx<PREC_FP16X2>(nb, M, status, st);
        if (prec == PREC_BF16X3) return launch_serial_mx<PREC_BF16X3>(nb, M, status, st);
        return hipErrorInvalidValue;
    }
#define TQ_CALL(NB, IB) return serial_impl<NB, IB, PREC_FP64>(M, status, st)
    TQ_DISPATCH(nb, ib, TQ_CALL);
#undef TQ_CALL
}

// Panels per workgroup of k_apply.  The wavefront has about kmax np / G + p
// links of a cost that grows with G, so few row blocks per step (square
// matrices) favour larger groups and many (tall ones) single panels; a group
// size is a power of two dividing np.
int apply_group(int np, int kmax, int p)
{
    int g = 1;
    while (2 * g <= np && 2 * g <= 8 && (int64_t)3 * kmax * np >= (int64_t)p * (2 * g) * (2 * g)) g *= 2;
    return g;
}

template <int NB, int IB>
static hipError_t apply_impl(ApplyDev D, bool trans, hipStream_t st)
{
    constexpr int NP = Cfg<NB, IB>::NPAN;
    if (D.group < 1 || NP % D.group != 0) D.group = apply_group(NP, D.kmax, D.M.p);
    const int nflag = D.kmax * (NP / D.group);
    hipLaunchKernelGGL(k_apply_init, dim3(1), dim3(256), 0, st, D.prog, nflag, D.M.p, trans ? 1 : 0);
    if (trans)
        hipLaunchKernelGGL((k_apply<NB, IB, true>), dim3(nflag), dim3(Cfg<NB, IB>::NT), 0, st, D);
    else
        hipLaunchKernelGGL((k_apply<NB, IB, false>), dim3(nflag), dim3(Cfg<NB, IB>::NT), 0, st, D);
    return hipGetLastError();
}

hipError_t launch_apply(int nb, int ib, const ApplyDev &D, bool trans, hipStream_t st)
{
    if (D.kmax <= 0) return hipSuccess;
#define TQ_CALL(NB, IB) return apply_impl<NB, IB>(D, trans, st)
    TQ_DISPATCH(nb, ib, TQ_CALL);
#undef TQ_CALL
}

hipError_t launch_cm2rows(const double *B, int64_t ldb, int64_t m, int64_t nrhs, double *Bt, int64_t rows, int ldt,
                          hipStream_t st)
{
    const int64_t total = rows * ldt;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cm2rows, dim3((unsigned)blocks), dim3(256), 0, st, B, ldb, m, nrhs, Bt, rows, ldt);
    return hipGetLastError();
}

hipError_t launch_rows2cm(double *B, int64_t ldb, int64_t m, int64_t nrhs, const double *Bt, int ldt, hipStream_t st)
{
    const int64_t total = m * nrhs;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rows2cm, dim3((unsigned)blocks), dim3(256), 0, st, B, ldb, m, nrhs, Bt, ldt);
    return hipGetLastError();
}

hipError_t launch_sched_init(const SchedDev &S, hipStream_t st)
{
    int64_t work = S.total_ids > S.qslot_total ? S.total_ids : S.qslot_total;
    int64_t blocks = (work + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_sched_init, dim3((unsigned)blocks), dim3(256), 0, st, S);
    hipLaunchKernelGGL(k_sched_seed, dim3(1), dim3(256), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_worker(int nb, int ib, int prec, const SchedDev &S, int workers, hipStream_t st)
{
    if (prec != PREC_FP64) {
        if (ib != 32) return hipErrorInvalidValue;
        if (prec == PREC_BF16X2) return launch_worker_mx<PREC_BF16X2>(nb, S, workers, st);
        if (prec == PREC_FP16X2) return launch_worker_mx<PREC_FP16X2>(nb, S, workers, st);
        if (prec == PREC_BF16X3) return launch_worker_mx<PREC_BF16X3>(nb, S, workers, st);
        return hipErrorInvalidValue;
    }
#define TQ_CALL(NB, IB) return worker_impl<NB, IB, PREC_FP64>(S, workers, st)
    TQ_DISPATCH(nb, ib, TQ_CALL);
#undef TQ_CALL
}

int worker_occupancy(int nb, int ib, int prec)
{
    if (prec != PREC_FP64) {
        if (prec == PREC_BF16X2) return worker_occupancy_mx<PREC_BF16X2>(nb);
        if (prec == PREC_FP16X2) return worker_occupancy_mx<PREC_FP16X2>(nb);
        if (prec == PREC_BF16X3) return worker_occupancy_mx<PREC_BF16X3>(nb);
        return 1;
    }
#define TQ_CALL(NB, IB) return worker_occupancy_impl<NB, IB, PREC_FP64>()
    do {
        if (nb == 64 && ib == 16) { TQ_CALL(64, 16); }
        else if (nb == 64 && ib == 32) { TQ_CALL(64, 32); }
        else if (nb == 128 && ib == 16) { TQ_CALL(128, 16); }
        else if (nb == 128 && ib == 32) { TQ_CALL(128, 32); }
        else if (nb == 256 && ib == 16) { TQ_CALL(256, 16); }
        else if (nb == 256 && ib == 32) { TQ_CALL(256, 32); }
    } while (0);
    return 1;
#undef TQ_CALL
}

}  // namespace tq
