// Host side of the C-ABI library declared in include/tileqr.h: argument
// checks, workspace, schedule set-up and the host-only DAG utilities.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

#include "../../include/tileqr.h"
#include "tileqr_dag.h"
#include "tileqr_host.h"
#include "tileqr_internal.h"

using namespace tq;

namespace tq {

namespace {
char g_hip_error[256] = "";
std::vector<Workspace *> g_ws;
}  // namespace

std::mutex g_mu;

int hip_fail(hipError_t e, const char *what)
{
    snprintf(g_hip_error, sizeof g_hip_error, "%s: %s", what, hipGetErrorString(e));
    return TILEQR_EHIP;
}

int DevBuf::ensure(size_t need)
{
    if (need <= bytes) return 0;
    if (arena) {
        const size_t off = (arena->used + 255) & ~(size_t)255;
        if (off > arena->cap || need > arena->cap - off) return TILEQR_ENOMEM;
        ptr = arena->base + off;
        bytes = need;
        arena->used = off + need;
        return 0;
    }
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
    if (hipMalloc(&ptr, need) != hipSuccess) {
        (void)hipGetLastError();
        return TILEQR_ENOMEM;
    }
    bytes = need;
    return 0;
}

void DevBuf::release()
{
    if (ptr && !arena) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

void SchedBufs::release()
{
    counters.release();
    qslot.release();
    qctl.release();
    mats.release();
}

Workspace *workspace(hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    for (auto *w : g_ws)
        if (w->device == dev && w->stream == stream) return w;
    auto *w = new Workspace;
    w->device = dev;
    w->stream = stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) w->num_cu = prop.multiProcessorCount;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess) w->wall_hz = khz * 1e3;
    if (hipHostMalloc((void **)&w->host_status, 64, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&w->host_small, 4096 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete w;
        return nullptr;
    }
    g_ws.push_back(w);
    return w;
}

Workspace *g_last_timed = nullptr;
Workspace *g_last_traced = nullptr;

std::vector<TuneEntry> *tuned_entries(bool create)
{
    static std::vector<TuneEntry> table;
    return (table.empty() && !create) ? nullptr : &table;
}

}  // namespace tq

// ------------------------------------------------------------------ basics

extern "C" void tileqr_opts_default(tileqr_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->precision = TILEQR_FP64;
    o->max_iter = 30;
    o->tol = 1e-14;
    o->drop_edge = -1;
}

extern "C" int tileqr_blocking_supported(int64_t nb, int64_t ib)
{
    if (nb != 64 && nb != 128 && nb != 256) return 0;
    if (ib != 16 && ib != 32) return 0;
    return nb % ib == 0 && ib <= nb;
}

namespace tq {

// tileqr_choose_blocking with g_mu already held by the caller.
void choose_blocking_held(int64_t m, int64_t n, int precision, int64_t *nb, int64_t *ib)
{
    tileqr_tuning t;
    if (tuned_single(m, n, precision, &t)) {
        if (nb) *nb = t.nb;
        if (ib) *ib = t.ib;
        return;
    }
    // Measured with one task per inner panel (the automatic split for up to
    // 32 tile steps) and, at ib = 32, PUPD tasks for the in-tile updates:
    // tall matrices and all but small ones run best with 256 x 256 tiles and
    // ib = 32 (65536 x 1024: 15.0 ms against 17.7 with ib = 16 and 18.4 with
    // nb = 128); near-square ones up to 2048 with 128 / 16 (2048^2: 3.6 ms
    // against 3.9 with 256 / 32), tiny ones with 64 / 16.
    const int64_t k = std::min(m, n);
    int64_t b = 256, s = 32;
    if (k <= 256) { b = 64; s = 16; }
    else if (m < 4 * n && n < 4 * m && k <= 2048) { b = 128; s = 16; }
    if (precision != TILEQR_FP64) s = 32;   // the split products take ib = 32
    if (nb) *nb = b;
    if (ib) *ib = s;
}

}  // namespace tq

extern "C" int tileqr_choose_blocking(int64_t m, int64_t n, int precision, int64_t *nb, int64_t *ib)
{
    std::lock_guard<std::mutex> lock(g_mu);
    choose_blocking_held(m, n, precision, nb, ib);
    return 0;
}

extern "C" size_t tileqr_t_size(int64_t m, int64_t n, int64_t nb, int64_t ib)
{
    if (m <= 0 || n <= 0 || !tileqr_blocking_supported(nb, ib)) return 0;
    const int64_t p = cdiv(m, nb), q = cdiv(n, nb), kmax = std::min(p, q);
    return (size_t)(kmax * p * ib * nb);
}

extern "C" double tileqr_flops_lapack(int64_t m, int64_t n)
{
    const double M = (double)m, N = (double)n;
    if (m >= n) return 2.0 * M * N * N - 2.0 * N * N * N / 3.0;
    return 2.0 * N * M * M - 2.0 * M * M * M / 3.0;
}

extern "C" double tileqr_flops_tiled(int64_t m, int64_t n, int64_t nb, int64_t ib)
{
    if (m <= 0 || n <= 0 || nb <= 0 || ib <= 0) return 0.0;
    const int p = (int)cdiv(m, nb), q = (int)cdiv(n, nb);
    const Grid g = make_grid(p, q, 1, 1);
    double f = 0.0;
    for (int64_t id = 0; id < g.total; ++id) {
        const Task t = decode(g, id);
        if (valid(g, t)) f += task_flops(t, (int)nb, (int)ib, 1, 1);
    }
    return f;
}

extern "C" int64_t tileqr_dag_counts(int64_t p, int64_t q, int64_t strips, int64_t panels, int64_t counts[5])
{
    int64_t c[NTYPE] = {0, 0, 0, 0, 0};
    if (p > 0 && q > 0 && strips > 0 && panels > 0) {
        const Grid g = make_grid((int)p, (int)q, (int)strips, (int)panels);
        for (int64_t id = 0; id < g.total; ++id) {
            const Task t = decode(g, id);
            if (valid(g, t)) ++c[t.type];
        }
    }
    if (counts)
        for (int k = 0; k < NTYPE; ++k) counts[k] = c[k];
    return c[0] + c[1] + c[2] + c[3] + c[4];
}

// ------------------------------------------------------- DAG self-check

namespace {

// Regions: strip s of tile (i, j), plus the R rows of each inner panel and
// the V half of the diagonal tiles.
struct RegionMap {
    int p, q, ns, np;
    int64_t strip(int i, int j, int s) const { return ((int64_t)j * p + i) * ns + s; }
    int64_t rrows(int k, int l) const { return (int64_t)p * q * ns + (int64_t)k * np + l; }
    int64_t vpart(int k) const { return (int64_t)p * q * ns + (int64_t)std::min(p, q) * np + k; }
    int64_t size() const { return (int64_t)p * q * ns + (int64_t)std::min(p, q) * (np + 1); }
};

// Reads and writes of a task (Algorithm 2, the table in tileqr_dag.h).  A
// panel task of tile (i, k) is modelled as touching every strip of it;
// GEQRT(k, l) also rewrites the R rows of panels l.. (its trailing update
// reaches every row below the panel's first), TSQRT(k, ., l) the R rows of
// panel l only.
void task_access(const RegionMap &R, const Task &t, std::vector<int64_t> &rd, std::vector<int64_t> &wr)
{
    rd.clear();
    wr.clear();
    switch (t.type) {
    case GEQRT:
        for (int s = 0; s < R.ns; ++s) {
            rd.push_back(R.strip(t.k, t.k, s));
            wr.push_back(R.strip(t.k, t.k, s));
        }
        for (int l = t.l; l < R.np; ++l) wr.push_back(R.rrows(t.k, l));
        wr.push_back(R.vpart(t.k));
        break;
    case LARFB:
        rd.push_back(R.vpart(t.k));
        rd.push_back(R.strip(t.k, t.j, t.s));
        wr.push_back(R.strip(t.k, t.j, t.s));
        break;
    case TSQRT:
        rd.push_back(R.rrows(t.k, t.l));
        wr.push_back(R.rrows(t.k, t.l));
        for (int s = 0; s < R.ns; ++s) {
            rd.push_back(R.strip(t.i, t.k, s));
            wr.push_back(R.strip(t.i, t.k, s));
        }
        break;
    default:
        for (int s = 0; s < R.ns; ++s) rd.push_back(R.strip(t.i, t.k, s));
        rd.push_back(R.strip(t.k, t.j, t.s));
        rd.push_back(R.strip(t.i, t.j, t.s));
        wr.push_back(R.strip(t.k, t.j, t.s));
        wr.push_back(R.strip(t.i, t.j, t.s));
        break;
    }
}

// With PUPD tasks (one panel per strip) the regions are finer: block
// (a, s) of tile (i, j) is rows of panel a in strip s, and a block on a
// tile's diagonal (a == s) has two halves, its strict lower part (V on the
// diagonal tile) and its upper part (R).  T_l of tile (i, k) is a region of
// its own, so the reads of V and T by the update tasks are checked too.
struct BlockMap {
    int p, q, n;   // n = panels = strips per tile
    int64_t blk(int i, int j, int s, int a, int h) const
    {
        return (((((int64_t)j * p + i) * n + s) * n + a) * 2) + h;
    }
    int64_t tblk(int k, int i, int l) const { return (int64_t)p * q * n * n * 2 + ((int64_t)k * p + i) * n + l; }
    int64_t size() const { return (int64_t)p * q * n * n * 2 + (int64_t)std::min(p, q) * p * n; }
    // Every half of blocks a0.. of strip s of tile (i, j).
    void strip(std::vector<int64_t> &v, int i, int j, int s, int a0 = 0) const
    {
        for (int a = a0; a < n; ++a) {
            v.push_back(blk(i, j, s, a, 0));
            if (a == s) v.push_back(blk(i, j, s, a, 1));
        }
    }
    // V of panel l of the diagonal tile (k, k): blocks below the diagonal
    // block and its lower half.
    void vpanel(std::vector<int64_t> &v, int k, int l) const
    {
        for (int a = l; a < n; ++a) v.push_back(blk(k, k, l, a, 0));
    }
};

void task_access_pu(const BlockMap &B, const Task &t, std::vector<int64_t> &rd, std::vector<int64_t> &wr)
{
    rd.clear();
    wr.clear();
    const int k = t.k;
    switch (t.type) {
    case GEQRT:   // factor strip l of tile (k, k) from row l ib down; write T_l
        B.strip(rd, k, k, t.l, t.l);
        B.strip(wr, k, k, t.l, t.l);
        wr.push_back(B.tblk(k, k, t.l));
        break;
    case TSQRT:   // R triangle of panel l, strip l of tile (i, k); write T_l
        rd.push_back(B.blk(k, k, t.l, t.l, 1));
        wr.push_back(B.blk(k, k, t.l, t.l, 1));
        B.strip(rd, t.i, k, t.l);
        B.strip(wr, t.i, k, t.l);
        wr.push_back(B.tblk(k, t.i, t.l));
        break;
    case PUPD:
        rd.push_back(B.tblk(k, t.i, t.l));
        if (t.i == k) {
            B.vpanel(rd, k, t.l);
            B.strip(rd, k, k, t.s, t.l);
            B.strip(wr, k, k, t.s, t.l);
        } else {
            B.strip(rd, t.i, k, t.l);
            rd.push_back(B.blk(k, k, t.s, t.l, 0));
            wr.push_back(B.blk(k, k, t.s, t.l, 0));
            B.strip(rd, t.i, k, t.s);
            B.strip(wr, t.i, k, t.s);
        }
        break;
    case LARFB:
        for (int l = 0; l < B.n; ++l) {
            B.vpanel(rd, k, l);
            rd.push_back(B.tblk(k, k, l));
        }
        B.strip(rd, k, t.j, t.s);
        B.strip(wr, k, t.j, t.s);
        break;
    default:
        for (int l = 0; l < B.n; ++l) {
            B.strip(rd, t.i, k, l);
            rd.push_back(B.tblk(k, t.i, l));
        }
        B.strip(rd, k, t.j, t.s);
        B.strip(rd, t.i, t.j, t.s);
        B.strip(wr, k, t.j, t.s);
        B.strip(wr, t.i, t.j, t.s);
        break;
    }
}

}  // namespace

extern "C" int tileqr_dag_selfcheck(int64_t p, int64_t q, int64_t strips, int64_t panels, int64_t trials,
                                   uint64_t seed)
{
    if (p <= 0 || q <= 0 || strips <= 0 || panels <= 0) return 0;
    const Grid g = make_grid((int)p, (int)q, (int)strips, (int)panels);
    const RegionMap R{(int)p, (int)q, (int)strips, (int)panels};
    const BlockMap B{(int)p, (int)q, (int)panels};
    auto access = [&](const Task &t, std::vector<int64_t> &rd, std::vector<int64_t> &wr) {
        if (g.pu) task_access_pu(B, t, rd, wr);
        else task_access(R, t, rd, wr);
    };
    const int64_t nregion = g.pu ? B.size() : R.size();
    std::vector<int64_t> rd, wr;
    // Reference: Algorithm 2's loop order (a tile kernel's inner panels in
    // order, each followed by its trailing update strip by strip).
    std::vector<int64_t> order;
    auto panels_of = [&](int k, int i) {
        for (int l = 0; l < g.np; ++l) {
            order.push_back(id_panel(g, k, i, l));
            if (g.pu)
                for (int s = l + 1; s < g.np; ++s) order.push_back(id_pupd(g, k, i, l, s));
        }
    };
    for (int k = 0; k < g.kmax; ++k) {
        panels_of(k, k);
        for (int j = k + 1; j < g.q; ++j)
            for (int s = 0; s < g.ns; ++s) order.push_back(id_larfb(g, k, j, s));
        for (int i = k + 1; i < g.p; ++i) {
            panels_of(k, i);
            for (int j = k + 1; j < g.q; ++j)
                for (int s = 0; s < g.ns; ++s) order.push_back(id_ssrfb(g, k, i, j, s));
        }
    }
    std::vector<std::vector<int64_t>> expect(g.total);
    {
        std::vector<int64_t> ver(nregion, 0);
        for (int64_t id : order) {
            access(decode(g, id), rd, wr);
            for (int64_t r : rd) expect[id].push_back(ver[r]);
            for (int64_t w : wr) ++ver[w];
        }
    }
    int64_t ntasks = (int64_t)order.size();
    std::mt19937_64 rng(seed);
    for (int64_t trial = 0; trial < trials; ++trial) {
        std::vector<int32_t> cnt(g.total, -1);
        std::vector<int64_t> ready;
        for (int64_t id = 0; id < g.total; ++id) {
            const Task t = decode(g, id);
            if (valid(g, t)) {
                cnt[id] = indegree(g, t);
                if (cnt[id] == 0) ready.push_back(id);
            }
        }
        std::vector<int64_t> ver(nregion, 0);
        int64_t executed = 0;
        while (!ready.empty()) {
            const size_t pick = (size_t)(rng() % ready.size());
            const int64_t id = ready[pick];
            ready[pick] = ready.back();
            ready.pop_back();
            const Task t = decode(g, id);
            access(t, rd, wr);
            for (size_t e = 0; e < rd.size(); ++e)
                if (ver[rd[e]] != expect[id][e]) return (int)(trial + 1);
            for (int64_t w : wr) ++ver[w];
            ++executed;
            const int ns = nsucc(g, t);
            for (int n = 0; n < ns; ++n) {
                const int64_t s = succ(g, t, n);
                if (s < 0 || s >= g.total || !valid(g, decode(g, s))) return (int)(trial + 1);
                if (--cnt[s] == 0) ready.push_back(s);
                if (cnt[s] < 0) return (int)(trial + 1);
            }
        }
        if (executed != ntasks) return (int)(trial + 1);
        for (int64_t id = 0; id < g.total; ++id)
            if (cnt[id] > 0) return (int)(trial + 1);
    }
    // The queue capacities the scheduler derives by index ranges must equal
    // the number of tasks each queue receives.
    for (int mat : {0, 1, 7}) {
        int64_t a[NQUEUE] = {0}, b[NQUEUE] = {0};
        for (int64_t id = 0; id < g.total; ++id) {
            const Task t = decode(g, id);
            if (valid(g, t)) ++a[queue_of(t, g.ns, mat)];
        }
        count_queue_tasks(g, mat, b);
        for (int l = 0; l < NQUEUE; ++l)
            if (a[l] != b[l]) return (int)(trials + 1);
    }
    return 0;
}

// ------------------------------------------------------------ factorisation

namespace tq {

// Split-precision updates run with ib = 32 (one K step of the narrow MFMA
// per wave), for every supported nb.
bool panel_tasks_ok(int64_t panel_tasks, int64_t nb, int64_t ib)
{
    return panel_tasks == 0 || panel_tasks == 1 || panel_tasks == nb / ib;
}

bool precision_supported(int precision, int64_t ib)
{
    if (precision == TILEQR_FP64) return true;
    if (precision == TILEQR_BF16X2 || precision == TILEQR_FP16X2 || precision == TILEQR_BF16X3) return ib == 32;
    return false;
}

int check_status(Workspace *W, int *dstatus, hipStream_t st)
{
    TQ_HIP(hipMemcpyAsync(W->host_status, dstatus, sizeof(int), hipMemcpyDeviceToHost, st));
    TQ_HIP(hipStreamSynchronize(st));
    const int s = *W->host_status;
    if (s & STATUS_NONFINITE) return TILEQR_ENONFINITE;
    if (s & STATUS_TIMEOUT) return TILEQR_ETIMEOUT;
    if (s & STATUS_SINGULAR) return TILEQR_ESINGULAR;
    return TILEQR_OK;
}

int prepare_schedule(Workspace *W, SchedBufs &B, std::vector<MatDev> &mats, int nb, int ib, const tileqr_opts &o,
                     hipStream_t st, SchedDev &S, int *workers)
{
    const int ns = strips_per_tile(nb, o.precision);
    const int nmat = (int)mats.size();
    // GEQRT / TSQRT tasks per tile.  One matrix with few tile steps is
    // bound by its chain of panel tasks, so each inner panel becomes a task
    // of its own and the panels of one step overlap; otherwise the update
    // throughput dominates and whole tile kernels (panels chained through
    // LDS, fewer tasks) do better.
    int64_t kmax_all = 0;
    for (const MatDev &M : mats) kmax_all = std::max<int64_t>(kmax_all, std::min(M.p, M.q));
    const int np = o.panel_tasks > 0 ? (int)o.panel_tasks : (nmat == 1 && kmax_all <= 32 ? nb / ib : 1);
    // Tasks per ready queue, counted by index ranges (no id decoding):
    // GEQRT and TSQRT have one queue each; strip tasks go to the queue of
    // their level and XCD hash.
    int64_t counts[NQUEUE] = {0};
    int64_t total_ids = 0, ntask = 0, kmax_max = 0;
    double panel_flops = 0.0, all_flops = 0.0;
    const double b3 = (double)nb * nb * nb;
    for (int mi = 0; mi < nmat; ++mi) {
        MatDev &M = mats[mi];
        const Grid g = make_grid(M.p, M.q, ns, np);
        M.task_base = total_ids;
        total_ids += g.total;
        kmax_max = std::max<int64_t>(kmax_max, g.kmax);
        count_queue_tasks(g, mi, counts);
        for (int k = 0; k < g.kmax; ++k) {
            const int64_t rows = g.p - k - 1;
            ntask += (int64_t)(1 + rows) * np + (int64_t)(1 + rows) * (g.q - k - 1) * ns;
            if (g.pu) ntask += (int64_t)(1 + rows) * np * (np - 1) / 2;   // PUPD
            panel_flops += (4.0 / 3.0) * b3 + 2.0 * b3 * rows;
            all_flops += (double)(g.q - k - 1) * (2.0 * b3 + (4.0 * b3 + (double)ib * nb * nb) * rows);
        }
    }
    all_flops += panel_flops;
    int rc;
    if ((rc = B.counters.ensure((size_t)total_ids * sizeof(int32_t)))) return rc;
    if ((rc = B.qslot.ensure((size_t)std::max<int64_t>(ntask, 1) * sizeof(int32_t)))) return rc;
    const size_t qctl_bytes = 2 * NQUEUE * QSTRIDE * sizeof(uint32_t) + 256 + NQUEUE * sizeof(int64_t);
    if ((rc = B.qctl.ensure(qctl_bytes))) return rc;
    if ((rc = B.mats.ensure((size_t)nmat * sizeof(MatDev)))) return rc;
    TQ_HIP(hipMemcpyAsync(B.mats.ptr, mats.data(), (size_t)nmat * sizeof(MatDev), hipMemcpyHostToDevice, st));
    std::memset(&S, 0, sizeof S);
    S.mats = (MatDev *)B.mats.ptr;
    S.nmat = nmat;
    S.ns = ns;
    S.np = np;
    S.total_ids = total_ids;
    S.total_tasks = (uint32_t)ntask;
    S.counters = (int32_t *)B.counters.ptr;
    S.qslot = (int32_t *)B.qslot.ptr;
    S.qslot_total = ntask;
    int64_t qoff[NQUEUE];
    int64_t off = 0;
    for (int l = 0; l < NQUEUE; ++l) {
        qoff[l] = off;
        off += counts[l];
    }
    S.qhead = (uint32_t *)B.qctl.ptr;
    S.qtail = S.qhead + NQUEUE * QSTRIDE;
    S.done = S.qtail + NQUEUE * QSTRIDE;
    S.trace_count = S.done + 1;
    int64_t *qoff_dev = (int64_t *)((char *)B.qctl.ptr + 2 * NQUEUE * QSTRIDE * sizeof(uint32_t) + 256);
    TQ_HIP(hipMemcpyAsync(qoff_dev, qoff, sizeof qoff, hipMemcpyHostToDevice, st));
    S.qoff = qoff_dev;
    S.status = (int32_t *)W->status.ptr;
    S.spin_limit = o.spin_limit > 0 ? o.spin_limit : (int64_t)1 << 24;
    S.shuffle = (o.flags & TILEQR_FLAG_SHUFFLE) ? 1 : 0;
    S.seed = o.seed;
    S.drop_edge = o.drop_edge;
    S.trace = nullptr;
    if (o.flags & TILEQR_FLAG_TRACE) {
        if ((rc = W->trace.ensure((size_t)std::max<int64_t>(ntask, 1) * TRACE_WORDS * sizeof(int64_t)))) return rc;
        S.trace = (int64_t *)W->trace.ptr;
        S.trace_cap = (uint32_t)ntask;
        W->trace_events = ntask;
    }
    // Panel workers.  A share of the workgroups in proportion to the panel
    // flops suits many matrices, and one matrix split into panel tasks,
    // whose panel wavefront holds up to nb/ib tasks per step in flight
    // (tall matrices: many; square ones: few, so at least 16 there).  One
    // matrix with whole tile kernels has one panel chain per step in
    // flight: 16 workgroups when there are at most 32 tile steps, else 8
    // (the updates dominate and every panel workgroup is one fewer for
    // them).  Update workers: the rest of what fits at once.
    const int occ = worker_occupancy(nb, ib, o.precision);
    const int capacity = std::max(2, std::max(1, W->num_cu) * occ);
    const int share = (int)std::lround(1.5 * capacity * panel_flops / std::max(all_flops, 1.0));
    int panel;
    if (o.panel_workers > 0) panel = (int)o.panel_workers;
    else if (nmat > 1) panel = share;
    else if (np > 1) panel = (int)std::min<int64_t>(std::max(share, 16), (int64_t)np * kmax_max);
    else panel = (int)std::min<int64_t>(kmax_max <= 32 ? 16 : 8, kmax_max);
    panel = std::max(1, std::min(panel, capacity / 2));
    int update = o.workers > 0 ? (int)o.workers : capacity - panel;
    update = std::max(1, std::min(update, capacity - panel));
    S.npanel = panel;
    *workers = panel + update;
    return 0;
}

}  // namespace tq

namespace {

// Runs the factorisation of the tiles already in W->tiles (status already
// cleared and set by the conversion).  Either the serial Algorithm 2 driver
// or the persistent DAG scheduler.
int run_factor(Workspace *W, int nb, int ib, int p, int q, double *T, const tileqr_opts &o, hipStream_t st,
               hipEvent_t ev_setup_done)
{
    int *dstatus = (int *)W->status.ptr;
    MatDev M;
    M.tiles = (double *)W->tiles.ptr;
    M.T = T;
    M.vsplit = nullptr;
    if (o.precision != TILEQR_FP64) {
        int rc;
        const int parts = o.precision == TILEQR_BF16X3 ? 3 : 2;
        if ((rc = W->vsplit.ensure(vsplit_bytes(p, std::min(p, q), nb, ib, parts)))) return rc;
        M.vsplit = W->vsplit.ptr;
    }
    M.p = p;
    M.q = q;
    M.task_base = 0;
    if (o.flags & TILEQR_FLAG_SERIAL) {
        if (ev_setup_done) TQ_HIP(hipEventRecord(ev_setup_done, st));
        TQ_HIP(launch_factor_serial(nb, ib, o.precision, M, dstatus, st));
        return 0;
    }
    std::vector<MatDev> mats(1, M);
    SchedDev S;
    int workers = 0, rc;
    if ((rc = prepare_schedule(W, W->sched, mats, nb, ib, o, st, S, &workers))) return rc;
    TQ_HIP(launch_sched_init(S, st));
    if (ev_setup_done) TQ_HIP(hipEventRecord(ev_setup_done, st));
    TQ_HIP(launch_worker(nb, ib, o.precision, S, workers, st));
    return 0;
}

}  // namespace

extern "C" int tileqr_factor_ex(int64_t m, int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib,
                                double *T, const tileqr_opts *opts)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (A == nullptr && m > 0 && n > 0) return -3;
    if (lda < std::max<int64_t>(1, m)) return -4;
    if (nb <= 0) return -5;
    if (ib <= 0 || ib > nb || nb % ib != 0) return -6;
    if (m == 0 || n == 0) return TILEQR_OK;
    if (T == nullptr) return -7;
    if (!tileqr_blocking_supported(nb, ib)) return TILEQR_EUNSUPPORTED;
    tileqr_opts o;
    tileqr_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision < TILEQR_FP64 || o.precision > TILEQR_BF16X3) return -8;
    if (!panel_tasks_ok(o.panel_tasks, nb, ib)) return -8;
    if (!precision_supported(o.precision, ib)) return TILEQR_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    hipStream_t st = (hipStream_t)o.stream;
    Workspace *W = workspace(st);
    if (!W) return hip_fail(hipErrorNoDevice, "workspace");
    const int p = (int)cdiv(m, nb), q = (int)cdiv(n, nb);
    int rc;
    if ((rc = W->tiles.ensure((size_t)p * q * nb * nb * sizeof(double)))) return rc;
    if ((rc = W->status.ensure(256))) return rc;
    W->trace_events = 0;
    if (o.flags & TILEQR_FLAG_TRACE) g_last_traced = W;
    const bool timing = (o.flags & TILEQR_FLAG_TIMING) && !(o.flags & TILEQR_FLAG_ASYNC);
    W->have_timing = false;
    if (timing && !W->ev[0])
        for (auto &e : W->ev) TQ_HIP(hipEventCreate(&e));
    TQ_HIP(hipMemsetAsync(W->status.ptr, 0, sizeof(int), st));
    if (timing) TQ_HIP(hipEventRecord(W->ev[0], st));
    TQ_HIP(launch_cm2tile(A, lda, m, n, (double *)W->tiles.ptr, (int)nb, p, q, (int *)W->status.ptr, st));
    if (timing) TQ_HIP(hipEventRecord(W->ev[1], st));
    if ((rc = run_factor(W, (int)nb, (int)ib, p, q, T, o, st, timing ? W->ev[2] : nullptr))) return rc;
    if (timing) TQ_HIP(hipEventRecord(W->ev[3], st));
    TQ_HIP(launch_tile2cm(A, lda, m, n, (double *)W->tiles.ptr, (int)nb, p, q, (const int *)W->status.ptr, st));
    if (timing) TQ_HIP(hipEventRecord(W->ev[4], st));
    if (o.flags & TILEQR_FLAG_ASYNC) return TILEQR_OK;
    rc = check_status(W, (int *)W->status.ptr, st);
    if (timing) {
        for (int s = 0; s < 4; ++s) {
            float ms = 0.f;
            TQ_HIP(hipEventElapsedTime(&ms, W->ev[s], W->ev[s + 1]));
            W->last_ms[s] = ms;
        }
        W->have_timing = true;
        g_last_timed = W;
    }
    return rc;
}

extern "C" int tileqr_last_timing(double ms[4])
{
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace *W = g_last_timed;
    if (!W || !W->have_timing) return TILEQR_EUNSUPPORTED;
    for (int s = 0; s < 4; ++s) ms[s] = W->last_ms[s];
    return TILEQR_OK;
}

extern "C" int tileqr_factor(int64_t m, int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib, double *T)
{
    return tileqr_factor_ex(m, n, A, lda, nb, ib, T, nullptr);
}

// ----------------------------------------------------------------- trace

extern "C" int64_t tileqr_trace(int64_t *events, int64_t cap)
{
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace *W = g_last_traced;
    if (!W || W->trace_events == 0 || !W->trace.ptr) return 0;
    const int64_t n = std::min(cap, W->trace_events);
    if (events && n > 0) {
        if (hipDeviceSynchronize() != hipSuccess) return 0;
        if (hipMemcpy(events, W->trace.ptr, (size_t)n * TRACE_WORDS * sizeof(int64_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return 0;
    }
    return W->trace_events;
}

extern "C" double tileqr_trace_clock_hz(void)
{
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
        return 0.0;
    return khz * 1e3;
}

// ------------------------------------------------------------------ misc

extern "C" const char *tileqr_status_string(int s)
{
    if (s < 0) return "invalid argument";
    switch (s) {
    case TILEQR_OK: return "ok";
    case TILEQR_EHIP: return "HIP runtime error";
    case TILEQR_ENONFINITE: return "input holds NaN or Inf";
    case TILEQR_ENOCONV: return "refinement did not converge";
    case TILEQR_ETIMEOUT: return "scheduler watchdog timeout";
    case TILEQR_ENOMEM: return "out of device memory";
    case TILEQR_EUNSUPPORTED: return "unsupported blocking";
    case TILEQR_ESINGULAR: return "singular triangular factor";
    case TILEQR_ENOTSPD: return "matrix not positive definite";
    default: return "unknown status";
    }
}

extern "C" const char *tileqr_last_hip_error(void) { return g_hip_error; }

extern "C" int tileqr_finalize(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto *w : g_ws) {
        if (hipSetDevice(w->device) == hipSuccess) {
            (void)hipDeviceSynchronize();
            w->tiles.release();
            w->vsplit.release();
            w->bvsplit.release();
            w->sched.release();
            w->btiles.release();
            w->bconv.release();
            w->lsT.release();
            w->lswork.release();
            w->lsdesc.release();
            w->lsout.release();
            for (auto &b : w->bsched) b.release();
            if (w->bgraph) (void)hipGraphExecDestroy(w->bgraph);
            if (w->cap_stream) (void)hipStreamDestroy(w->cap_stream);
            w->status.release();
            w->trace.release();
            w->misc.release();
            w->luinv.release();
            w->lulup.release();
            w->lupiv.release();
            w->rows.release();
            w->prog.release();
            w->tws.release();
            w->solve.release();
            w->part.release();
            w->tflags.release();
            if (w->host_small) (void)hipHostFree(w->host_small);
            for (auto &e : w->ev)
                if (e) (void)hipEventDestroy(e);
            if (w->host_status) (void)hipHostFree(w->host_status);
        }
        delete w;
    }
    g_ws.clear();
    g_last_timed = g_last_traced = nullptr;
    (void)hipSetDevice(cur);
    return TILEQR_OK;
}
// ------------------------------------------------------------- applying Q

namespace {

// Q^T or Q on row blocks `rows` (leading dimension ldt) with the factor
// already in W->tiles.  W->prog must hold min(p, q) nb/ib flags (PROG_STRIDE apart).
hipError_t apply_rows(Workspace *W, int nb, int ib, int p, int q, const double *T, double *rows, int ldt, int ncol,
                      bool trans, hipStream_t st, int group = 0)
{
    ApplyDev D;
    D.M.tiles = (double *)W->tiles.ptr;
    D.M.T = const_cast<double *>(T);
    D.M.vsplit = nullptr;
    D.M.p = p;
    D.M.q = q;
    D.M.task_base = 0;
    D.B = rows;
    D.ldb = ldt;
    D.nstrip = ldt / kStripWidth;
    D.ncol = ncol;
    D.kmax = std::min(p, q);
    D.group = group;
    D.prog = (int32_t *)W->prog.ptr;
    D.status = (int32_t *)W->status.ptr;
    D.spin_limit = (int64_t)1 << 26;
    return launch_apply(nb, ib, D, trans, st);
}

// B := Q^T B or Q B with the factor (A, T) of tileqr_factor.  The factor is
// converted to tiles, B to row blocks, and the apply kernel runs the steps.
int apply_common(bool trans, int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, int64_t nb,
                 int64_t ib, const double *T, double *B, int64_t ldb)
{
    if (m < 0) return -1;
    if (n < 0) return -2;
    if (nrhs < 0) return -3;
    if (A == nullptr && m > 0 && n > 0) return -4;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (nb <= 0) return -6;
    if (ib <= 0 || ib > nb || nb % ib != 0) return -7;
    if (T == nullptr && m > 0 && n > 0) return -8;
    if (B == nullptr && m > 0 && nrhs > 0) return -9;
    if (ldb < std::max<int64_t>(1, m)) return -10;
    if (m == 0 || n == 0 || nrhs == 0) return TILEQR_OK;
    if (!tileqr_blocking_supported(nb, ib)) return TILEQR_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    hipStream_t st = nullptr;
    Workspace *W = workspace(st);
    if (!W) return hip_fail(hipErrorNoDevice, "workspace");
    const int p = (int)cdiv(m, nb), q = (int)cdiv(n, nb), kmax = std::min(p, q);
    const int nstrip = (int)cdiv(nrhs, kStripWidth);
    const int ldt = nstrip * kStripWidth;
    int rc;
    if ((rc = W->tiles.ensure((size_t)p * q * nb * nb * sizeof(double)))) return rc;
    if ((rc = W->rows.ensure((size_t)p * nb * ldt * sizeof(double)))) return rc;
    if ((rc = W->prog.ensure((size_t)kmax * (nb / ib) * PROG_STRIDE * sizeof(int32_t) + 64))) return rc;
    if ((rc = W->status.ensure(256))) return rc;
    TQ_HIP(hipMemsetAsync(W->status.ptr, 0, sizeof(int), st));
    TQ_HIP(launch_cm2tile(A, lda, m, n, (double *)W->tiles.ptr, (int)nb, p, q, (int *)W->status.ptr, st));
    TQ_HIP(launch_cm2rows(B, ldb, m, nrhs, (double *)W->rows.ptr, (int64_t)p * nb, ldt, st));
    TQ_HIP(apply_rows(W, (int)nb, (int)ib, p, q, T, (double *)W->rows.ptr, ldt, (int)nrhs, trans, st));
    TQ_HIP(launch_rows2cm(B, ldb, m, nrhs, (double *)W->rows.ptr, ldt, st));
    return check_status(W, (int *)W->status.ptr, st);
}

}  // namespace

extern "C" int tileqr_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, int64_t nb,
                               int64_t ib, const double *T, double *B, int64_t ldb)
{
    return apply_common(true, m, n, nrhs, A, lda, nb, ib, T, B, ldb);
}

extern "C" int tileqr_apply_q(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, int64_t nb,
                              int64_t ib, const double *T, double *B, int64_t ldb)
{
    return apply_common(false, m, n, nrhs, A, lda, nb, ib, T, B, ldb);
}

// ------------------------------------------------------------ least squares

namespace {

// Row-block buffers of the solver, each p nb x ldt doubles.
enum { SB = 0, SX, SR, SF, SG, SS, SXB, SNUM };

struct SolveCtx {
    Workspace *W;
    hipStream_t st;
    const double *A;
    int64_t lda, m, n;
    int nrhs, ldt, nb, ib, p, q;
    int group;       // inner panels per workgroup of the Q applications (0: automatic)
    double *buf[SNUM];
    double *T;
    double *part;
    int64_t part_cap;
    double *small;   // device: norms
};

// Device scratch of the solver's norms (W->misc): results in doubles
// [0, SMALL_PART) (per-column results at 0, 64, 128, 192, 256, 320), partial
// sums of the norm kernels in [SMALL_PART, SMALL_PART + SMALL_PART_CAP),
// enough for COLSQ_BLOCKS blocks times the largest nrhs (64).
constexpr int64_t SMALL_PART = 1024;
constexpr int64_t SMALL_PART_CAP = (int64_t)COLSQ_BLOCKS * 64;
constexpr int NPROBE = 8;

// Backward errors of the iterate in buf[SX], per column v, from the residual
// S = B - A X (formed here into buf[SS]):
//   eta_ls[v]  = ||A^T S_v||_2 / (||A||_F (||A||_F ||X_v||_2 + ||B_v||_2))
//   eta_inf[v] = ||S_v||_inf / (||A||_inf ||X_v||_inf)     (square systems only)
int eta_of(SolveCtx &c, double normA, double normAinf, const double *normb, bool square, double *eta_ls,
           double *eta_inf)
{
    Workspace *W = c.W;
    double *S = c.buf[SS];
    TQ_HIP(launch_axpy_rows(c.buf[SB], S, c.ldt, c.m, c.nrhs, 2, c.st));
    TQ_HIP(launch_gemv_n(c.A, c.lda, c.m, c.n, c.buf[SX], c.ldt, c.nrhs, -1.0, 1.0, S, c.part, c.part_cap, c.st));
    double *AtS = c.buf[SG];   // scratch n x nrhs (SG is recomputed before use)
    TQ_HIP(launch_gemv_t(c.A, c.lda, c.m, c.n, S, c.ldt, c.nrhs, 1.0, 0.0, AtS, c.part, c.part_cap, c.st));
    double *dev = c.small;
    TQ_HIP(launch_colsq(AtS, c.ldt, c.n, c.nrhs, dev + SMALL_PART, SMALL_PART_CAP, dev, c.st));
    TQ_HIP(launch_colsq(c.buf[SX], c.ldt, c.n, c.nrhs, dev + SMALL_PART, SMALL_PART_CAP, dev + 64, c.st));
    if (square) {
        TQ_HIP(launch_colmax(S, c.ldt, c.m, c.nrhs, dev + SMALL_PART, SMALL_PART_CAP, dev + 256, c.st));
        TQ_HIP(launch_colmax(c.buf[SX], c.ldt, c.n, c.nrhs, dev + SMALL_PART, SMALL_PART_CAP, dev + 320, c.st));
    }
    TQ_HIP(hipMemcpyAsync(W->host_small, dev, 128 * sizeof(double), hipMemcpyDeviceToHost, c.st));
    if (square)
        TQ_HIP(hipMemcpyAsync(W->host_small + 256, dev + 256, 128 * sizeof(double), hipMemcpyDeviceToHost, c.st));
    TQ_HIP(hipStreamSynchronize(c.st));
    for (int v = 0; v < c.nrhs; ++v) {
        const double num = std::sqrt(W->host_small[v]);
        const double den = normA * (normA * std::sqrt(W->host_small[64 + v]) + normb[v]);
        eta_ls[v] = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
        eta_inf[v] = 0.0;
        if (square) {
            const double r = W->host_small[256 + v], d = normAinf * W->host_small[320 + v];
            eta_inf[v] = d > 0.0 ? r / d : (r > 0.0 ? INFINITY : 0.0);
        }
    }
    return 0;
}

// beta_fact estimate ||A - Q [R; 0]||_F / ||A||_F from NPROBE Gaussian probes
// z (E ||E z||^2 = ||E||_F^2): A Z against Q [R Z; 0], with A the caller's
// matrix and the factor in W->tiles / c.T.  Uses buf[SF], buf[SG], buf[SS].
int beta_fact_probe(SolveCtx &c, double normA, uint64_t seed, double *out)
{
    Workspace *W = c.W;
    double *Z = c.buf[SG], *Y = c.buf[SF], *V = c.buf[SS];
    const size_t slot = (size_t)c.p * c.nb * c.ldt;
    TQ_HIP(hipMemsetAsync(Z, 0, slot * sizeof(double), c.st));
    TQ_HIP(hipMemsetAsync(Y, 0, slot * sizeof(double), c.st));
    TQ_HIP(launch_fill_normal(Z, c.ldt, c.n, NPROBE, seed, c.st));
    TQ_HIP(launch_gemv_n(c.A, c.lda, c.m, c.n, Z, c.ldt, NPROBE, 1.0, 0.0, Y, c.part, c.part_cap, c.st));
    TQ_HIP(launch_trmm(c.nb, (double *)W->tiles.ptr, c.p, c.n, V, Z, c.ldt, c.st));
    ApplyDev D;
    D.M.tiles = (double *)W->tiles.ptr;
    D.M.T = c.T;
    D.M.vsplit = nullptr;
    D.M.p = c.p;
    D.M.q = c.q;
    D.M.task_base = 0;
    D.B = V;
    D.ldb = c.ldt;
    D.nstrip = c.ldt / kStripWidth;
    D.ncol = NPROBE;
    D.kmax = std::min(c.p, c.q);
    D.group = c.group;
    D.prog = (int32_t *)W->prog.ptr;
    D.status = (int32_t *)W->status.ptr;
    D.spin_limit = (int64_t)1 << 26;
    TQ_HIP(launch_apply(c.nb, c.ib, D, false, c.st));
    TQ_HIP(launch_axpy_rows(V, Y, c.ldt, c.m, NPROBE, 0, c.st));   // Y = Q [R Z; 0] - A Z
    TQ_HIP(launch_colsq(Y, c.ldt, c.m, NPROBE, c.small + SMALL_PART, SMALL_PART_CAP, c.small + 384, c.st));
    TQ_HIP(hipMemcpyAsync(W->host_small + 384, c.small + 384, NPROBE * sizeof(double), hipMemcpyDeviceToHost,
                          c.st));
    TQ_HIP(hipStreamSynchronize(c.st));
    double ss = 0.0;
    for (int v = 0; v < NPROBE; ++v) ss += W->host_small[384 + v];
    *out = normA > 0.0 ? std::sqrt(ss / NPROBE) / normA : 0.0;
    return 0;
}

}  // namespace

extern "C" int tileqr_solve_ls(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                               int64_t ldb, double *X, int64_t ldx, const tileqr_opts *opts, tileqr_info *info)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (nrhs < 0 || nrhs > 64) return -3;
    if (A == nullptr && m > 0 && n > 0) return -4;
    if (lda < std::max<int64_t>(1, m)) return -5;
    if (B == nullptr && m > 0 && nrhs > 0) return -6;
    if (ldb < std::max<int64_t>(1, m)) return -7;
    if (X == nullptr && n > 0 && nrhs > 0) return -8;
    if (ldx < std::max<int64_t>(1, n)) return -9;
    tileqr_opts o;
    tileqr_opts_default(&o);
    if (opts) o = *opts;
    if (o.max_iter < 0 || o.max_iter > 64 || !(o.tol >= 0.0)) return -10;
    if (o.precision < TILEQR_FP64 || o.precision > TILEQR_BF16X3) return -10;
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->beta_fact_est = -1.0;
    }
    if (n == 0 || nrhs == 0) return TILEQR_OK;
    int64_t nb = o.nb, ib = o.ib;
    if (nb == 0 || ib == 0) tileqr_choose_blocking(m, n, o.precision, &nb, &ib);
    if (!tileqr_blocking_supported(nb, ib)) return TILEQR_EUNSUPPORTED;
    if (!panel_tasks_ok(o.panel_tasks, nb, ib)) return -10;
    if (o.apply_group != 0 && (o.apply_group > 8 || (o.apply_group & (o.apply_group - 1)) != 0 ||
                               (nb / ib) % o.apply_group != 0))
        return -10;
    if (!precision_supported(o.precision, ib)) return TILEQR_EUNSUPPORTED;

    std::lock_guard<std::mutex> lock(g_mu);
    hipStream_t st = (hipStream_t)o.stream;
    Workspace *W = workspace(st);
    if (!W) return hip_fail(hipErrorNoDevice, "workspace");
    const int p = (int)cdiv(m, nb), q = (int)cdiv(n, nb);
    const int ldt = (int)cdiv(nrhs, kStripWidth) * kStripWidth;
    const size_t slot = (size_t)p * nb * ldt;
    const bool square = m == n;
    int rc;
    if ((rc = W->tiles.ensure((size_t)p * q * nb * nb * sizeof(double)))) return rc;
    if ((rc = W->tws.ensure(std::max<size_t>(1, tileqr_t_size(m, n, nb, ib)) * sizeof(double)))) return rc;
    if ((rc = W->solve.ensure(SNUM * slot * sizeof(double)))) return rc;
    const int64_t part_cap = std::max<int64_t>(m * 32 * 16, 1 << 20);
    if ((rc = W->part.ensure((size_t)part_cap * sizeof(double)))) return rc;
    if ((rc = W->misc.ensure((SMALL_PART + SMALL_PART_CAP) * sizeof(double)))) return rc;
    if ((rc = W->prog.ensure((size_t)std::min(p, q) * (nb / ib) * PROG_STRIDE * sizeof(int32_t) + 64))) return rc;
    const int64_t tflags_cap = trsm_flags_needed(n, ldt);
    if ((rc = W->tflags.ensure((size_t)tflags_cap * sizeof(int32_t)))) return rc;
    const int64_t spin = o.spin_limit > 0 ? o.spin_limit : (int64_t)1 << 24;
    if ((rc = W->status.ensure(256))) return rc;
    if (!W->ev[0])
        for (auto &e : W->ev) TQ_HIP(hipEventCreate(&e));

    SolveCtx c;
    c.W = W;
    c.st = st;
    c.A = A;
    c.lda = lda;
    c.m = m;
    c.n = n;
    c.nrhs = (int)nrhs;
    c.ldt = ldt;
    c.nb = (int)nb;
    c.ib = (int)ib;
    c.p = p;
    c.q = q;
    c.group = (int)o.apply_group;
    for (int i = 0; i < SNUM; ++i) c.buf[i] = (double *)W->solve.ptr + i * slot;
    c.T = (double *)W->tws.ptr;
    c.part = (double *)W->part.ptr;
    c.part_cap = part_cap;
    c.small = (double *)W->misc.ptr;
    int *dstatus = (int *)W->status.ptr;

    // Factor a copy of A (A itself is never written).
    TQ_HIP(hipEventRecord(W->ev[0], st));
    TQ_HIP(hipMemsetAsync(dstatus, 0, sizeof(int), st));
    TQ_HIP(launch_cm2tile(A, lda, m, n, (double *)W->tiles.ptr, (int)nb, p, q, dstatus, st));
    tileqr_opts fo = o;
    fo.flags &= ~(unsigned)(TILEQR_FLAG_ASYNC | TILEQR_FLAG_TIMING | TILEQR_FLAG_TRACE);
    if ((rc = run_factor(W, (int)nb, (int)ib, p, q, c.T, fo, st, W->ev[3]))) return rc;
    TQ_HIP(hipEventRecord(W->ev[1], st));
    if ((rc = check_status(W, dstatus, st))) return rc;

    // Norms fixed for the whole refinement.
    TQ_HIP(hipMemsetAsync(W->solve.ptr, 0, SNUM * slot * sizeof(double), st));
    TQ_HIP(launch_cm2rows(B, ldb, m, nrhs, c.buf[SB], (int64_t)p * nb, ldt, st));
    TQ_HIP(launch_frob2(A, lda, m, n, c.small + SMALL_PART, SMALL_PART_CAP, c.small + 128, st));
    TQ_HIP(launch_colsq(c.buf[SB], ldt, m, c.nrhs, c.small + SMALL_PART, SMALL_PART_CAP, c.small + 192, st));
    if (square) TQ_HIP(launch_norm_inf(A, lda, m, n, c.part, part_cap, c.small + 129, st));
    TQ_HIP(hipMemcpyAsync(W->host_small + 128, c.small + 128, 128 * sizeof(double), hipMemcpyDeviceToHost, st));
    TQ_HIP(hipStreamSynchronize(st));
    const double normA = std::sqrt(W->host_small[128]);
    const double normAinf = square ? W->host_small[129] : 0.0;
    double normb[64], eta_ls[64], eta_inf[64];
    for (int v = 0; v < c.nrhs; ++v) normb[v] = std::sqrt(W->host_small[192 + v]);

    // Optional check of the factorisation (not part of the solve proper).
    if ((o.flags & TILEQR_FLAG_CHECK) && info) {
        double bf = -1.0;
        if ((rc = beta_fact_probe(c, normA, o.seed ^ 0x5eedULL, &bf))) return rc;
        info->beta_fact_est = bf;
        info->probes = NPROBE;
        TQ_HIP(hipMemsetAsync(W->solve.ptr, 0, SNUM * slot * sizeof(double), st));
        TQ_HIP(launch_cm2rows(B, ldb, m, nrhs, c.buf[SB], (int64_t)p * nb, ldt, st));
    }

    // x0 = R^{-1} (Q^T b)(0:n),  r0 = b - A x0.
    TQ_HIP(launch_axpy_rows(c.buf[SB], c.buf[SX], ldt, m, c.nrhs, 2, st));
    TQ_HIP(apply_rows(W, c.nb, c.ib, p, q, c.T, c.buf[SX], ldt, c.nrhs, true, st, c.group));
    TQ_HIP(launch_trsm(c.nb, (double *)W->tiles.ptr, p, n, c.buf[SX], ldt, true, (int *)W->tflags.ptr, tflags_cap,
                       dstatus, spin, st));
    // zero the rows n.. of x (they held (Q^T b)(n:m))
    TQ_HIP(hipMemsetAsync(c.buf[SX] + (size_t)n * ldt, 0, (size_t)(p * nb - n) * ldt * sizeof(double), st));
    if (!square) {
        TQ_HIP(launch_axpy_rows(c.buf[SB], c.buf[SR], ldt, m, c.nrhs, 2, st));
        TQ_HIP(launch_gemv_n(A, lda, m, n, c.buf[SX], ldt, c.nrhs, -1.0, 1.0, c.buf[SR], c.part, part_cap, st));
    }
    if ((rc = check_status(W, dstatus, st))) return rc;

    // The stopping measure: eta_LS, and for square systems also the
    // infinity-norm backward error of Section 3.2.4 (whichever is larger).
    auto measure = [&](double &worst, double &wls, double &winf) {
        worst = wls = winf = 0.0;
        for (int v = 0; v < c.nrhs; ++v) {
            wls = std::max(wls, eta_ls[v]);
            winf = std::max(winf, eta_inf[v]);
            worst = std::max(worst, std::max(eta_ls[v], eta_inf[v]));
        }
    };
    double eta, e_ls, e_inf;
    if ((rc = eta_of(c, normA, normAinf, normb, square, eta_ls, eta_inf))) return rc;
    measure(eta, e_ls, e_inf);
    double best = eta, best_ls = e_ls, best_inf = e_inf;
    TQ_HIP(launch_axpy_rows(c.buf[SX], c.buf[SXB], ldt, n, c.nrhs, 2, st));
    if (info) info->eta_hist[0] = eta;
    int it = 0, stall = 0;
    double prev = eta;
    while (eta > o.tol && it < o.max_iter) {
        ++it;
        double *F = c.buf[SF], *G = c.buf[SG];
        if (square) {
            // Classical refinement (the augmented system with m = n, whose
            // least-squares residual is zero): dx = R^{-1} Q^T (b - A x), with
            // the residual b - A x that eta_of left in buf[SS].
            TQ_HIP(launch_axpy_rows(c.buf[SS], F, ldt, m, c.nrhs, 2, st));
            TQ_HIP(apply_rows(W, c.nb, c.ib, p, q, c.T, F, ldt, c.nrhs, true, st, c.group));
            TQ_HIP(launch_trsm(c.nb, (double *)W->tiles.ptr, p, n, F, ldt, true, (int *)W->tflags.ptr, tflags_cap,
                               dstatus, spin, st));
            TQ_HIP(launch_axpy_rows(F, c.buf[SX], ldt, n, c.nrhs, 1, st));
        } else {
            // Refinement of the augmented system [I A; A^T 0][r; x] = [b; 0]
            // (residuals in FP64 on the original A, corrections through the
            // factors): f = b - r - A x ;  g = -A^T r
            TQ_HIP(launch_axpy_rows(c.buf[SB], F, ldt, m, c.nrhs, 2, st));
            TQ_HIP(launch_axpy_rows(c.buf[SR], F, ldt, m, c.nrhs, 0, st));   // F = R - F = r - b
            TQ_HIP(launch_axpy_rows(nullptr, F, ldt, m, c.nrhs, 3, st));     // F = b - r
            TQ_HIP(launch_gemv_n(A, lda, m, n, c.buf[SX], ldt, c.nrhs, -1.0, 1.0, F, c.part, part_cap, st));
            TQ_HIP(launch_gemv_t(A, lda, m, n, c.buf[SR], ldt, c.nrhs, -1.0, 0.0, G, c.part, part_cap, st));
            // [f1; f2] = Q^T f ;  d1 = R^{-T} g ;  dx = R^{-1} (f1 - d1) ;  dr = Q [d1; f2]
            TQ_HIP(apply_rows(W, c.nb, c.ib, p, q, c.T, F, ldt, c.nrhs, true, st, c.group));
            TQ_HIP(launch_trsm(c.nb, (double *)W->tiles.ptr, p, n, G, ldt, false, (int *)W->tflags.ptr, tflags_cap,
                               dstatus, spin, st));
            double *DX = c.buf[SS];
            TQ_HIP(launch_axpy_rows(F, DX, ldt, n, c.nrhs, 2, st));
            TQ_HIP(launch_axpy_rows(G, DX, ldt, n, c.nrhs, 0, st));          // DX = G - DX = d1 - f1
            TQ_HIP(launch_axpy_rows(nullptr, DX, ldt, n, c.nrhs, 3, st));    // DX = f1 - d1
            TQ_HIP(hipMemsetAsync(DX + (size_t)n * ldt, 0, (size_t)(p * nb - n) * ldt * sizeof(double), st));
            TQ_HIP(launch_trsm(c.nb, (double *)W->tiles.ptr, p, n, DX, ldt, true, (int *)W->tflags.ptr, tflags_cap,
                               dstatus, spin, st));
            TQ_HIP(launch_axpy_rows(DX, c.buf[SX], ldt, n, c.nrhs, 1, st));
            TQ_HIP(launch_axpy_rows(G, F, ldt, n, c.nrhs, 2, st));             // F = [d1; f2]
            TQ_HIP(apply_rows(W, c.nb, c.ib, p, q, c.T, F, ldt, c.nrhs, false, st, c.group));
            TQ_HIP(launch_axpy_rows(F, c.buf[SR], ldt, m, c.nrhs, 1, st));
        }
        if ((rc = eta_of(c, normA, normAinf, normb, square, eta_ls, eta_inf))) return rc;
        measure(eta, e_ls, e_inf);
        if (info && it < 65) info->eta_hist[it] = eta;
        if (eta < best) {
            best = eta;
            best_ls = e_ls;
            best_inf = e_inf;
            TQ_HIP(launch_axpy_rows(c.buf[SX], c.buf[SXB], ldt, n, c.nrhs, 2, st));
        }
        stall = eta > 0.5 * prev ? stall + 1 : 0;
        prev = eta;
        if (stall >= 2) break;
    }
    TQ_HIP(launch_rows2cm(X, ldx, n, nrhs, c.buf[SXB], ldt, st));
    TQ_HIP(hipEventRecord(W->ev[2], st));
    rc = check_status(W, dstatus, st);
    if (info) {
        info->iterations = it;
        info->converged = best <= o.tol;
        info->eta = best;
        info->eta_ls = best_ls;
        info->eta_inf = best_inf;
        info->nb = nb;
        info->ib = ib;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, W->ev[0], W->ev[1]) == hipSuccess) info->ms_factor = ms;
        if (hipEventElapsedTime(&ms, W->ev[0], W->ev[2]) == hipSuccess) info->ms_total = ms;
        if (hipEventElapsedTime(&ms, W->ev[3], W->ev[1]) == hipSuccess) info->ms_worker = ms;
    }
    if (rc) return rc;
    return best <= o.tol ? TILEQR_OK : TILEQR_ENOCONV;
}
