// Batched tiled QR: many independent factorisations in one persistent
// launch per (nb, ib) group, one global task space over all of them (each
// matrix its own DAG of Section 4), captured into a HIP graph and replayed;
// and the autotuner that picks nb, ib and the split of the workgroups
// between the panel and update roles by timing trial runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/tileqr.h"
#include "tileqr_dag.h"
#include "tileqr_host.h"
#include "tileqr_internal.h"

using namespace tq;

namespace {

struct Group {
    int nb, ib;
    std::vector<int64_t> members;   // batch indices (non-empty matrices only)
    std::vector<ConvDesc> conv;
    int64_t nblk = 0;               // 64 x 64 conversion blocks
    SchedDev S;
    int workers = 0;
};

// ceil(log2(x)) for x >= 1, else 0.
int64_t clog2(int64_t x)
{
    int64_t b = 0;
    while (b < 62 && ((int64_t)1 << b) < x) ++b;
    return b;
}

// Size class of a shape key (precision, batch, (m, n) pairs): precision,
// ceil(log2) of the batch size, of the flop-weighted typical min(m, n), and
// of the largest m and n.  Shapes in one class get the same blocking from a
// tuned entry when no entry has exactly their shapes.
std::vector<int64_t> tune_bucket(const std::vector<int64_t> &key)
{
    const int64_t batch = key.size() >= 2 ? key[1] : 0;
    double wsum = 0.0, ksum = 0.0;
    int64_t mmax = 0, nmax = 0;
    for (int64_t i = 0; i < batch && 3 + 2 * i < (int64_t)key.size(); ++i) {
        const int64_t m = key[2 + 2 * i], n = key[3 + 2 * i];
        const double f = std::max(1.0, tileqr_flops_lapack(std::max(m, n), std::min(m, n)));
        wsum += f;
        ksum += f * (double)std::min(m, n);
        mmax = std::max(mmax, m);
        nmax = std::max(nmax, n);
    }
    const int64_t kt = wsum > 0.0 ? (int64_t)(ksum / wsum + 0.5) : 0;
    return {key.empty() ? 0 : key[0], clog2(batch), clog2(kt), clog2(mmax), clog2(nmax)};
}

// Architecture name and compute-unit count of the current device (cached
// per device), false without a device.
bool device_signature(std::string &arch, int &cu)
{
    static std::vector<std::pair<int, std::pair<std::string, int>>> seen;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    for (auto &e : seen)
        if (e.first == dev) {
            arch = e.second.first;
            cu = e.second.second;
            return true;
        }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    if (colon != std::string::npos) a.resize(colon);
    seen.push_back({dev, {a, prop.multiProcessorCount}});
    arch = a;
    cu = prop.multiProcessorCount;
    return true;
}

// The entry for exactly these shapes on this kind of device, else one of the
// same size class (the most recently added).
const tileqr_tuning *lookup_tuned(const std::string &arch, int cu, const std::vector<int64_t> &key)
{
    const std::vector<TuneEntry> *tab = tuned_entries(false);
    if (!tab) return nullptr;
    for (const auto &e : *tab)
        if (e.arch == arch && e.cu == cu && e.key == key) return &e.best;
    const std::vector<int64_t> bucket = tune_bucket(key);
    for (auto it = tab->rbegin(); it != tab->rend(); ++it)
        if (it->arch == arch && it->cu == cu && it->bucket == bucket) return &it->best;
    return nullptr;
}

const tileqr_tuning *find_tuned(const std::vector<int64_t> &key)
{
    if (!tuned_entries(false)) return nullptr;   // no HIP call while nothing is tuned
    std::string arch;
    int cu = 0;
    if (!device_signature(arch, cu)) return nullptr;
    return lookup_tuned(arch, cu, key);
}

std::vector<int64_t> shape_key(int64_t batch, const int64_t *m, const int64_t *n, int precision)
{
    std::vector<std::pair<int64_t, int64_t>> sh((size_t)batch);
    for (int64_t i = 0; i < batch; ++i) sh[(size_t)i] = {m[i], n[i]};
    std::sort(sh.begin(), sh.end());
    std::vector<int64_t> key;
    key.reserve(2 + 2 * (size_t)batch);
    key.push_back(precision);
    key.push_back(batch);
    for (const auto &s : sh) {
        key.push_back(s.first);
        key.push_back(s.second);
    }
    return key;
}

// Blocking for a whole batch without a tuned entry: the one a single matrix
// of the flop-weighted typical size would get.
void default_batch_blocking(int64_t batch, const int64_t *m, const int64_t *n, int precision, int64_t *nb,
                            int64_t *ib)
{
    double wsum = 0.0, ksum = 0.0;
    for (int64_t i = 0; i < batch; ++i) {
        const double f = tileqr_flops_lapack(m[i], n[i]);
        wsum += f;
        ksum += f * (double)std::min(m[i], n[i]);
    }
    const int64_t k = wsum > 0.0 ? (int64_t)(ksum / wsum) : 1;
    choose_blocking_held(k, k, precision, nb, ib);   // g_mu is held by every caller
}

// Per-matrix blocking of a batched call: the caller's, or the tuner's entry
// for these shapes (with its split of the workgroups), or the default.
void batch_blocking(int64_t batch, const int64_t *m, const int64_t *n, const int64_t *nb, const int64_t *ib,
                    tileqr_opts &o, std::vector<int64_t> &nbv, std::vector<int64_t> &ibv)
{
    if (nb) {
        nbv.assign(nb, nb + batch);
        ibv.assign(ib, ib + batch);
        return;
    }
    int64_t b = 0, s = 0;
    const tileqr_tuning *t = find_tuned(shape_key(batch, m, n, o.precision));
    if (t) {
        b = t->nb;
        s = t->ib;
        if (o.panel_workers == 0 && o.workers == 0) {
            o.panel_workers = t->panel_workers;
            o.workers = t->workers;
        }
    } else {
        default_batch_blocking(batch, m, n, o.precision, &b, &s);
    }
    nbv.assign((size_t)batch, b);
    ibv.assign((size_t)batch, s);
}

int argcheck(int64_t batch, const int64_t *m, const int64_t *n, double *const *A, const int64_t *lda,
             const int64_t *nb, const int64_t *ib, double *const *T)
{
    if (batch < 0) return -1;
    if (batch > 0 && (!m || !n || !A || !lda || !T)) return !m ? -2 : !n ? -3 : !A ? -4 : !lda ? -5 : -8;
    if ((nb == nullptr) != (ib == nullptr)) return nb == nullptr ? -6 : -7;
    for (int64_t i = 0; i < batch; ++i) {
        if (m[i] < 0 || m[i] > INT32_MAX) return -2;
        if (n[i] < 0 || n[i] > INT32_MAX) return -3;
        const bool empty = m[i] == 0 || n[i] == 0;
        if (!empty && A[i] == nullptr) return -4;
        if (lda[i] < std::max<int64_t>(1, m[i])) return -5;
        if (nb) {
            if (nb[i] <= 0) return -6;
            if (ib[i] <= 0 || ib[i] > nb[i] || nb[i] % ib[i] != 0) return -7;
        }
        if (!empty && T[i] == nullptr) return -8;
    }
    return 0;
}

// The kernels of one call in stream order: clear the status, convert every
// matrix to tiles, then per group the scheduler set-up and the persistent
// workers, then (with `back`) convert every matrix back.  No memset nodes,
// so that the sequence may be captured.
int enqueue_batched(Workspace *W, std::vector<Group> &groups, const ConvDesc *conv_dev, int precision,
                    hipStream_t st, bool back = true)
{
    int *dstatus = (int *)W->status.ptr;
    TQ_HIP(launch_fill_int(dstatus, 1, 0, st));
    size_t off = 0;
    for (auto &g : groups) {
        TQ_HIP(launch_cm2tile_batched(conv_dev + off, (int)g.members.size(), g.nblk, g.nb, dstatus, st));
        off += g.members.size();
    }
    for (auto &g : groups) {
        TQ_HIP(launch_sched_init(g.S, st));
        TQ_HIP(launch_worker(g.nb, g.ib, precision, g.S, g.workers, st));
    }
    if (!back) return 0;
    off = 0;
    for (auto &g : groups) {
        TQ_HIP(launch_tile2cm_batched(conv_dev + off, (int)g.members.size(), g.nblk, g.nb, dstatus, st));
        off += g.members.size();
    }
    return 0;
}

// Arguments already checked, g_mu held.  nbv/ibv: per-matrix blocking.
// With tiles_out (least squares): the factored tiles stay in the workspace,
// A is only read (no conversion back), the kernels are launched directly,
// and tiles_out[i] receives matrix i's first tile.
int run_batched(Workspace *W, int64_t batch, const int64_t *m, const int64_t *n, double *const *A,
                const int64_t *lda, const int64_t *nbv, const int64_t *ibv, double *const *T, const tileqr_opts &o,
                hipStream_t st, std::vector<const double *> *tiles_out = nullptr)
{
    std::vector<Group> groups;
    int64_t tile_doubles = 0;
    for (int64_t i = 0; i < batch; ++i) {
        if (m[i] == 0 || n[i] == 0) continue;
        if (!tileqr_blocking_supported(nbv[i], ibv[i]) || !precision_supported(o.precision, ibv[i]))
            return TILEQR_EUNSUPPORTED;
        if (!panel_tasks_ok(o.panel_tasks, nbv[i], ibv[i])) return -9;
        Group *g = nullptr;
        for (auto &x : groups)
            if (x.nb == nbv[i] && x.ib == ibv[i]) g = &x;
        if (!g) {
            groups.emplace_back();
            g = &groups.back();
            g->nb = (int)nbv[i];
            g->ib = (int)ibv[i];
        }
        g->members.push_back(i);
        const int64_t p = cdiv(m[i], nbv[i]), q = cdiv(n[i], nbv[i]);
        tile_doubles += p * q * nbv[i] * nbv[i];
    }
    if (groups.empty()) return TILEQR_OK;
    int rc;
    if ((rc = W->btiles.ensure((size_t)tile_doubles * sizeof(double)))) return rc;
    // Split modes: the split images of every matrix, back to back.
    const int parts = o.precision == TILEQR_BF16X3 ? 3 : 2;
    size_t vs_bytes = 0;
    if (o.precision != TILEQR_FP64) {
        for (auto &g : groups)
            for (int64_t i : g.members) {
                const int p = (int)cdiv(m[i], g.nb), q = (int)cdiv(n[i], g.nb);
                vs_bytes += vsplit_bytes(p, std::min(p, q), g.nb, g.ib, parts);
            }
        if ((rc = W->bvsplit.ensure(vs_bytes))) return rc;
    }
    char *vsp = (char *)W->bvsplit.ptr;
    if ((rc = W->status.ensure(256))) return rc;
    int64_t nconv = 0;
    for (auto &g : groups) nconv += (int64_t)g.members.size();
    if ((rc = W->bconv.ensure((size_t)nconv * sizeof(ConvDesc)))) return rc;
    if (W->bsched.size() < groups.size()) W->bsched.resize(groups.size());

    // Descriptors: tiles of all matrices back to back in the workspace.
    double *tiles = (double *)W->btiles.ptr;
    std::vector<ConvDesc> conv_all;
    conv_all.reserve((size_t)nconv);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        Group &g = groups[gi];
        std::vector<MatDev> mats;
        mats.reserve(g.members.size());
        for (int64_t i : g.members) {
            ConvDesc d;
            d.A = A[i];
            d.lda = lda[i];
            d.m = m[i];
            d.n = n[i];
            d.tiles = tiles;
            d.p = (int32_t)cdiv(m[i], g.nb);
            d.q = (int32_t)cdiv(n[i], g.nb);
            d.blk0 = g.nblk;
            g.nblk += (int64_t)d.p * d.q * (g.nb / 64) * (g.nb / 64);
            conv_all.push_back(d);
            MatDev M;
            M.tiles = tiles;
            M.T = T[i];
            M.vsplit = nullptr;
            if (o.precision != TILEQR_FP64) {
                M.vsplit = vsp;
                vsp += vsplit_bytes(d.p, std::min(d.p, d.q), g.nb, g.ib, parts);
            }
            M.p = d.p;
            M.q = d.q;
            M.task_base = 0;
            mats.push_back(M);
            if (tiles_out) (*tiles_out)[(size_t)i] = tiles;
            tiles += (size_t)d.p * d.q * g.nb * g.nb;
        }
        if ((rc = prepare_schedule(W, W->bsched[gi], mats, g.nb, g.ib, o, st, g.S, &g.workers))) return rc;
    }
    const ConvDesc *conv_dev = (const ConvDesc *)W->bconv.ptr;
    TQ_HIP(hipMemcpyAsync(W->bconv.ptr, conv_all.data(), conv_all.size() * sizeof(ConvDesc), hipMemcpyHostToDevice,
                          st));

    if (tiles_out) return enqueue_batched(W, groups, conv_dev, o.precision, st, false);
    if (o.flags & TILEQR_FLAG_NO_GRAPH) return enqueue_batched(W, groups, conv_dev, o.precision, st);

    // Everything the captured launches hold by value.
    std::vector<int64_t> key;
    key.push_back(o.precision);
    key.push_back((int64_t)(intptr_t)W->status.ptr);
    key.push_back((int64_t)(intptr_t)conv_dev);
    for (auto &g : groups) {
        key.push_back(g.nb);
        key.push_back(g.ib);
        key.push_back((int64_t)g.members.size());
        key.push_back(g.nblk);
        key.push_back(g.workers);
        int64_t words[sizeof(SchedDev) / sizeof(int64_t) + 1] = {0};
        std::memcpy(words, &g.S, sizeof(SchedDev));
        key.insert(key.end(), words, words + sizeof(words) / sizeof(words[0]));
    }
    if (!W->bgraph || key != W->bgraph_key) {
        if (!W->cap_stream) TQ_HIP(hipStreamCreateWithFlags(&W->cap_stream, hipStreamNonBlocking));
        if (W->bgraph) {
            TQ_HIP(hipGraphExecDestroy(W->bgraph));
            W->bgraph = nullptr;
            W->bgraph_key.clear();
        }
        hipGraph_t graph = nullptr;
        TQ_HIP(hipStreamBeginCapture(W->cap_stream, hipStreamCaptureModeThreadLocal));
        const int erc = enqueue_batched(W, groups, conv_dev, o.precision, W->cap_stream);
        const hipError_t ce = hipStreamEndCapture(W->cap_stream, &graph);
        if (erc) {
            if (graph) (void)hipGraphDestroy(graph);
            return erc;
        }
        TQ_HIP(ce);
        const hipError_t ie = hipGraphInstantiate(&W->bgraph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        TQ_HIP(ie);
        W->bgraph_key = key;
    }
    TQ_HIP(hipGraphLaunch(W->bgraph, st));
    return 0;
}

}  // namespace

extern "C" int tileqr_factor_batched(int64_t batch, const int64_t *m, const int64_t *n, double *const *A,
                                     const int64_t *lda, const int64_t *nb, const int64_t *ib, double *const *T,
                                     const tileqr_opts *opts)
{
    int rc = argcheck(batch, m, n, A, lda, nb, ib, T);
    if (rc) return rc;
    tileqr_opts o;
    tileqr_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision < TILEQR_FP64 || o.precision > TILEQR_BF16X3) return -9;
    if (o.flags & (TILEQR_FLAG_SERIAL | TILEQR_FLAG_TRACE)) return TILEQR_EUNSUPPORTED;
    if (batch == 0) return TILEQR_OK;
    std::lock_guard<std::mutex> lock(g_mu);
    hipStream_t st = (hipStream_t)o.stream;
    Workspace *W = workspace(st);
    if (!W) return hip_fail(hipErrorNoDevice, "workspace");
    std::vector<int64_t> nbv, ibv;
    batch_blocking(batch, m, n, nb, ib, o, nbv, ibv);
    const bool timing = (o.flags & TILEQR_FLAG_TIMING) && !(o.flags & TILEQR_FLAG_ASYNC);
    W->have_timing = false;
    if (timing && !W->ev[0])
        for (auto &e : W->ev) TQ_HIP(hipEventCreate(&e));
    if (timing) TQ_HIP(hipEventRecord(W->ev[0], st));
    if ((rc = run_batched(W, batch, m, n, A, lda, nbv.data(), ibv.data(), T, o, st))) return rc;
    if (timing) TQ_HIP(hipEventRecord(W->ev[1], st));
    if (o.flags & TILEQR_FLAG_ASYNC) return TILEQR_OK;
    rc = check_status(W, (int *)W->status.ptr, st);
    if (timing) {
        float ms = 0.f;
        TQ_HIP(hipEventElapsedTime(&ms, W->ev[0], W->ev[1]));
        W->last_ms[0] = W->last_ms[1] = W->last_ms[3] = 0.0;
        W->last_ms[2] = ms;
        W->have_timing = true;
        g_last_timed = W;
    }
    return rc;
}

// ------------------------------------------------------------------ tuner

namespace tq {

// Tuned blocking for one m x n matrix, if tileqr_tune has seen it.
bool tuned_single(int64_t m, int64_t n, int precision, tileqr_tuning *out)
{
    const tileqr_tuning *t = find_tuned(shape_key(1, &m, &n, precision));
    if (!t) return false;
    *out = *t;
    return true;
}

}  // namespace tq

extern "C" int tileqr_tune(int64_t batch, const int64_t *m, const int64_t *n, int precision, int trials,
                           tileqr_tuning *best)
{
    if (batch < 1) return -1;
    if (!m) return -2;
    if (!n) return -3;
    for (int64_t i = 0; i < batch; ++i) {
        if (m[i] < 0 || m[i] > INT32_MAX) return -2;
        if (n[i] < 0 || n[i] > INT32_MAX) return -3;
    }
    if (precision < TILEQR_FP64 || precision > TILEQR_BF16X3) return -4;
    if (trials < 1 || trials > 100) return -5;
    if (!best) return -6;
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace *W = workspace(nullptr);
    if (!W) return hip_fail(hipErrorNoDevice, "workspace");
    if (!W->ev[0])
        for (auto &e : W->ev) TQ_HIP(hipEventCreate(&e));

    int64_t maxdim = 1, elems = 0;
    for (int64_t i = 0; i < batch; ++i) {
        maxdim = std::max(maxdim, std::max(m[i], n[i]));
        elems += m[i] * n[i];
    }
    // Candidate blockings: every supported (nb, ib) the precision allows,
    // skipping tile sizes larger than every matrix (their runs only pad).
    std::vector<std::pair<int64_t, int64_t>> blockings;
    for (int64_t b : {64, 128, 256})
        for (int64_t s : {16, 32})
            if ((b == 64 || b <= maxdim) && tileqr_blocking_supported(b, s) && precision_supported(precision, s))
                blockings.push_back({b, s});
    // Candidate splits of the workgroups: automatic, then fixed panel shares.
    std::vector<int64_t> panels = {0};
    if (batch == 1) {
        panels.push_back(1);
        panels.push_back(4);
    } else {
        const int64_t cu = std::max(1, W->num_cu);
        panels.push_back(cu / 8);
        panels.push_back(cu / 4);
        panels.push_back(cu / 2 - 1);
    }

    // Scratch matrices (column-major, lda = m) and T areas sized for the
    // largest T over the candidates.
    std::vector<int64_t> lda(m, m + batch);
    for (auto &x : lda) x = std::max<int64_t>(1, x);
    int64_t tdoubles = 0;
    for (int64_t i = 0; i < batch; ++i) {
        int64_t mx = 0;
        for (auto &bs : blockings) mx = std::max<int64_t>(mx, (int64_t)tileqr_t_size(m[i], n[i], bs.first, bs.second));
        tdoubles += mx;
    }
    DevBuf Abuf, Tbuf;
    int rc;
    if ((rc = Abuf.ensure((size_t)std::max<int64_t>(elems, 1) * sizeof(double)))) return rc;
    if ((rc = Tbuf.ensure((size_t)std::max<int64_t>(tdoubles, 1) * sizeof(double)))) {
        Abuf.release();
        return rc;
    }
    std::vector<double *> Ap((size_t)batch), Tp((size_t)batch);
    {
        double *a = (double *)Abuf.ptr, *t = (double *)Tbuf.ptr;
        for (int64_t i = 0; i < batch; ++i) {
            Ap[(size_t)i] = a;
            Tp[(size_t)i] = t;
            a += m[i] * n[i];
            int64_t mx = 0;
            for (auto &bs : blockings)
                mx = std::max<int64_t>(mx, (int64_t)tileqr_t_size(m[i], n[i], bs.first, bs.second));
            t += mx;
        }
    }
    hipStream_t st = nullptr;
    tileqr_tuning top;
    top.ms = -1.0;
    for (auto &bs : blockings) {
        std::vector<int64_t> nbv((size_t)batch, bs.first), ibv((size_t)batch, bs.second);
        for (int64_t pw : panels) {
            tileqr_opts o;
            tileqr_opts_default(&o);
            o.precision = precision;
            o.panel_workers = pw;
            o.flags = TILEQR_FLAG_NO_GRAPH;
            double bestms = -1.0;
            // One untimed run first: the first launch of a kernel
            // instantiation and the growth of the workspace would otherwise
            // weigh on whichever configuration meets them first.
            if ((rc = launch_fill_uniform((double *)Abuf.ptr, elems, 1233, st)) != hipSuccess) {
                rc = hip_fail((hipError_t)rc, "fill");
                break;
            }
            if ((rc = run_batched(W, batch, m, n, Ap.data(), lda.data(), nbv.data(), ibv.data(), Tp.data(), o, st)))
                break;
            if ((rc = check_status(W, (int *)W->status.ptr, st))) break;
            for (int r = 0; r < trials && rc == 0; ++r) {
                if ((rc = launch_fill_uniform((double *)Abuf.ptr, elems, 1234 + r, st)) != hipSuccess) {
                    rc = hip_fail((hipError_t)rc, "fill");
                    break;
                }
                if ((rc = hipEventRecord(W->ev[0], st)) != hipSuccess) {
                    rc = hip_fail((hipError_t)rc, "event");
                    break;
                }
                rc = run_batched(W, batch, m, n, Ap.data(), lda.data(), nbv.data(), ibv.data(), Tp.data(), o, st);
                if (rc) break;
                if ((rc = hipEventRecord(W->ev[1], st)) != hipSuccess) {
                    rc = hip_fail((hipError_t)rc, "event");
                    break;
                }
                if ((rc = check_status(W, (int *)W->status.ptr, st))) break;
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, W->ev[0], W->ev[1]);
                if (bestms < 0.0 || ms < bestms) bestms = ms;
            }
            if (rc) break;
            if (top.ms < 0.0 || bestms < top.ms) {
                top.nb = bs.first;
                top.ib = bs.second;
                top.panel_workers = pw;
                top.workers = 0;
                top.ms = bestms;
            }
        }
        if (rc) break;
    }
    (void)hipStreamSynchronize(st);
    Abuf.release();
    Tbuf.release();
    if (rc) return rc;
    std::string arch;
    int cu = 0;
    if (!device_signature(arch, cu)) return hip_fail(hipErrorNoDevice, "device properties");
    const std::vector<int64_t> key = shape_key(batch, m, n, precision);
    std::vector<TuneEntry> *tab = tuned_entries(true);
    for (auto it = tab->begin(); it != tab->end(); ++it)
        if (it->arch == arch && it->cu == cu && it->key == key) {
            tab->erase(it);
            break;
        }
    TuneEntry e;
    e.arch = arch;
    e.cu = cu;
    e.key = key;
    e.bucket = tune_bucket(key);
    e.best = top;
    tab->push_back(e);
    *best = top;
    return TILEQR_OK;
}

// ------------------------------------------------------- tuner table files
//
// One entry per line, whitespace-separated:
//   tileqr-tune-1 <arch> <cu> <nb> <ib> <panel_workers> <workers> <ms> <key length> <key...>
// The size class is recomputed from the key on loading.

extern "C" int64_t tileqr_tune_save(const char *path)
{
    if (!path) return -1;
    std::lock_guard<std::mutex> lock(g_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return -2;
    int64_t count = 0;
    bool ok = true;
    if (const std::vector<TuneEntry> *tab = tuned_entries(false))
        for (const auto &e : *tab) {
            ok = ok && std::fprintf(f, "tileqr-tune-1 %s %d %lld %lld %lld %lld %.17g %zu", e.arch.c_str(), e.cu,
                                    (long long)e.best.nb, (long long)e.best.ib, (long long)e.best.panel_workers,
                                    (long long)e.best.workers, e.best.ms, e.key.size()) > 0;
            for (int64_t v : e.key) ok = ok && std::fprintf(f, " %lld", (long long)v) > 0;
            ok = ok && std::fputc('\n', f) != EOF;
            ++count;
        }
    ok = std::fclose(f) == 0 && ok;
    return ok ? count : -2;
}

extern "C" int64_t tileqr_tune_load(const char *path)
{
    if (!path) return -1;
    std::ifstream in(path);
    if (!in) return -2;
    std::vector<TuneEntry> got;
    std::string line;
    while (std::getline(in, line)) {
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        std::istringstream ls(line);
        std::string tag;
        TuneEntry e;
        size_t klen = 0;
        long long nb = 0, ib = 0, pw = 0, wk = 0;
        if (!(ls >> tag >> e.arch >> e.cu >> nb >> ib >> pw >> wk >> e.best.ms >> klen) || tag != "tileqr-tune-1" ||
            klen < 4 || klen > ((size_t)1 << 24))
            return -3;
        e.key.resize(klen);
        for (auto &v : e.key) {
            long long x;
            if (!(ls >> x)) return -3;
            v = x;
        }
        std::string extra;
        if (ls >> extra) return -3;
        // The key is (precision, batch, then batch (m, n) pairs), and the
        // blocking one the library supports.
        if (e.key[0] < TILEQR_FP64 || e.key[0] > TILEQR_BF16X3 || e.key[1] < 1 ||
            klen != (size_t)(2 + 2 * e.key[1]) || !tileqr_blocking_supported(nb, ib) ||
            !precision_supported((int)e.key[0], ib) || pw < 0 || wk < 0 || e.cu <= 0)
            return -3;
        for (size_t i = 2; i < klen; ++i)
            if (e.key[i] < 0) return -3;
        e.best.nb = nb;
        e.best.ib = ib;
        e.best.panel_workers = pw;
        e.best.workers = wk;
        e.bucket = tune_bucket(e.key);
        got.push_back(std::move(e));
    }
    std::lock_guard<std::mutex> lock(g_mu);
    std::vector<TuneEntry> *tab = tuned_entries(true);
    for (auto &e : got) {
        for (auto it = tab->begin(); it != tab->end(); ++it)
            if (it->arch == e.arch && it->cu == e.cu && it->key == e.key) {
                tab->erase(it);
                break;
            }
        tab->push_back(std::move(e));
    }
    return (int64_t)got.size();
}

extern "C" int tileqr_tune_lookup(const char *arch, int cu, int64_t batch, const int64_t *m, const int64_t *n,
                                  int precision, tileqr_tuning *out)
{
    if (!arch) return -1;
    if (batch < 1) return -3;
    if (!m) return -4;
    if (!n) return -5;
    if (precision < TILEQR_FP64 || precision > TILEQR_BF16X3) return -6;
    if (!out) return -7;
    std::lock_guard<std::mutex> lock(g_mu);
    const tileqr_tuning *t = lookup_tuned(arch, cu, shape_key(batch, m, n, precision));
    if (!t) return 0;
    *out = *t;
    return 1;
}

extern "C" void tileqr_tune_clear(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (std::vector<TuneEntry> *tab = tuned_entries(false)) tab->clear();
}

extern "C" int tileqr_solve_ls_batched(int64_t batch, const int64_t *m, const int64_t *n, const double *const *A,
                                       const int64_t *lda, const double *const *b, double *const *x,
                                       const tileqr_opts *opts, double *eta, int32_t *iterations,
                                       tileqr_batch_info *info)
{
    if (batch < 0) return -1;
    if (batch > 0 && (!m || !n || !A || !lda || !b || !x)) return !m ? -2 : !n ? -3 : !A ? -4 : !lda ? -5 : !b ? -6 : -7;
    for (int64_t i = 0; i < batch; ++i) {
        if (m[i] < 0 || m[i] > INT32_MAX) return -2;
        if (n[i] < 0 || n[i] > m[i]) return -3;
        if (n[i] > 0 && A[i] == nullptr) return -4;
        if (lda[i] < std::max<int64_t>(1, m[i])) return -5;
        if (n[i] > 0 && b[i] == nullptr) return -6;
        if (n[i] > 0 && x[i] == nullptr) return -7;
    }
    tileqr_opts o;
    tileqr_opts_default(&o);
    if (opts) o = *opts;
    if (o.precision < TILEQR_FP64 || o.precision > TILEQR_BF16X3) return -8;
    if (o.max_iter < 0 || o.max_iter > 64 || !(o.tol >= 0.0)) return -8;
    if ((o.nb == 0) != (o.ib == 0)) return -8;
    if (o.flags & (TILEQR_FLAG_SERIAL | TILEQR_FLAG_TRACE | TILEQR_FLAG_ASYNC)) return TILEQR_EUNSUPPORTED;
    if (info) std::memset(info, 0, sizeof *info);
    if (batch == 0) return TILEQR_OK;
    std::lock_guard<std::mutex> lock(g_mu);
    hipStream_t st = (hipStream_t)o.stream;
    Workspace *W = workspace(st);
    if (!W) return hip_fail(hipErrorNoDevice, "workspace");
    std::vector<int64_t> nbv, ibv, nbu, ibu;
    if (o.nb) {
        nbu.assign((size_t)batch, o.nb);
        ibu.assign((size_t)batch, o.ib);
    }
    batch_blocking(batch, m, n, o.nb ? nbu.data() : nullptr, o.nb ? ibu.data() : nullptr, o, nbv, ibv);
    for (int64_t i = 0; i < batch; ++i)
        if (n[i] > 0 && (!tileqr_blocking_supported(nbv[(size_t)i], ibv[(size_t)i]) ||
                         !precision_supported(o.precision, ibv[(size_t)i])))
            return TILEQR_EUNSUPPORTED;
    // T blocks and the solver's scratch vectors, per matrix, back to back.
    std::vector<size_t> toff((size_t)batch + 1, 0), woff((size_t)batch + 1, 0);
    for (int64_t i = 0; i < batch; ++i) {
        const bool empty = n[i] == 0;
        toff[(size_t)i + 1] = toff[(size_t)i] + (empty ? 0 : tileqr_t_size(m[i], n[i], nbv[(size_t)i], ibv[(size_t)i]));
        woff[(size_t)i + 1] = woff[(size_t)i] + (empty ? 0 : (size_t)7 * cdiv(m[i], nbv[(size_t)i]) * nbv[(size_t)i]);
    }
    int rc;
    if ((rc = W->lsT.ensure(std::max<size_t>(1, toff.back()) * sizeof(double)))) return rc;
    if ((rc = W->lswork.ensure(std::max<size_t>(1, woff.back()) * sizeof(double)))) return rc;
    std::vector<double *> Tp((size_t)batch), Ap((size_t)batch);
    std::vector<int64_t> mf((size_t)batch), nf((size_t)batch);
    for (int64_t i = 0; i < batch; ++i) {
        Tp[(size_t)i] = (double *)W->lsT.ptr + toff[(size_t)i];
        Ap[(size_t)i] = const_cast<double *>(A[i]);   // only read: no conversion back in this mode
        mf[(size_t)i] = n[i] == 0 ? 0 : m[i];           // m > 0 = n: nothing to factor or solve
        nf[(size_t)i] = n[i];
    }
    const bool timing = (o.flags & TILEQR_FLAG_TIMING) != 0 || info != nullptr;
    if (timing && !W->ev[0])
        for (auto &e : W->ev) TQ_HIP(hipEventCreate(&e));
    if (timing) TQ_HIP(hipEventRecord(W->ev[0], st));
    std::vector<const double *> tiles((size_t)batch, nullptr);
    if ((rc = run_batched(W, batch, mf.data(), nf.data(), Ap.data(), lda, nbv.data(), ibv.data(), Tp.data(), o, st,
                          &tiles)))
        return rc;
    if (timing) TQ_HIP(hipEventRecord(W->ev[1], st));
    if ((rc = check_status(W, (int *)W->status.ptr, st))) return rc;

    // One workgroup per matrix, the largest first.
    std::vector<int64_t> order;
    for (int64_t i = 0; i < batch; ++i)
        if (n[i] > 0) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t c) {
        return tileqr_flops_lapack(m[a], n[a]) > tileqr_flops_lapack(m[c], n[c]);
    });
    std::vector<LsDesc> descs;
    descs.reserve(order.size());
    for (int64_t i : order) {
        LsDesc d;
        d.A = A[i];
        d.lda = lda[i];
        d.b = b[i];
        d.x = x[i];
        d.tiles = tiles[(size_t)i];
        d.T = Tp[(size_t)i];
        d.work = (double *)W->lswork.ptr + woff[(size_t)i];
        d.m = (int32_t)m[i];
        d.n = (int32_t)n[i];
        d.nb = (int32_t)nbv[(size_t)i];
        d.ib = (int32_t)ibv[(size_t)i];
        d.p = (int32_t)cdiv(m[i], d.nb);
        d.q = (int32_t)cdiv(n[i], d.nb);
        descs.push_back(d);
    }
    const int count = (int)descs.size();
    if ((rc = W->lsdesc.ensure(std::max<size_t>(1, descs.size()) * sizeof(LsDesc)))) return rc;
    if ((rc = W->lsout.ensure(std::max<size_t>(1, descs.size()) * sizeof(LsOut)))) return rc;
    if (count > 0) {
        TQ_HIP(hipMemcpyAsync(W->lsdesc.ptr, descs.data(), descs.size() * sizeof(LsDesc), hipMemcpyHostToDevice, st));
        TQ_HIP(launch_ls_batched((const LsDesc *)W->lsdesc.ptr, count, o.tol, o.max_iter, (LsOut *)W->lsout.ptr,
                                 (int *)W->status.ptr, st));
    }
    if (timing) TQ_HIP(hipEventRecord(W->ev[2], st));
    std::vector<LsOut> res(descs.size());
    if (count > 0)
        TQ_HIP(hipMemcpyAsync(res.data(), W->lsout.ptr, res.size() * sizeof(LsOut), hipMemcpyDeviceToHost, st));
    rc = check_status(W, (int *)W->status.ptr, st);   // synchronises st
    int64_t conv = 0, noconv = 0;
    int maxit = 0;
    double maxeta = 0.0;
    for (size_t u = 0; u < order.size(); ++u) {
        const int64_t i = order[u];
        if (eta) eta[i] = res[u].eta;
        if (iterations) iterations[i] = res[u].iterations;
        if (res[u].eta <= o.tol) ++conv;
        else ++noconv;
        maxit = std::max(maxit, (int)res[u].iterations);
        maxeta = std::max(maxeta, res[u].eta);
    }
    for (int64_t i = 0; i < batch; ++i)
        if (n[i] == 0) {
            if (eta) eta[i] = 0.0;
            if (iterations) iterations[i] = 0;
        }
    if (info) {
        info->converged = conv;
        info->not_converged = noconv;
        info->max_iterations = maxit;
        info->max_eta = maxeta;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, W->ev[0], W->ev[1]) == hipSuccess) info->ms_factor = ms;
        if (hipEventElapsedTime(&ms, W->ev[0], W->ev[2]) == hipSuccess) info->ms_total = ms;
    }
    if (rc) return rc;
    return noconv > 0 ? TILEQR_ENOCONV : TILEQR_OK;
}
