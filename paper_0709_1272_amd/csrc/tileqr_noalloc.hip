// tileqr_factor_noalloc: the factorisation of tileqr_factor_ex with every
// buffer of the library (tile workspace, status word, scheduler counters and
// queues, split images of V and T) carved from one fixed device array of
// this file instead of allocated.  Same kernels, same schedule, same bits.
//
// The array lives in the code object: each device the library runs on holds
// its own copy, for the life of the process.  Host code never passes the
// array's name to a kernel or a copy (on the host it only stands for the
// symbol); it passes the device address hipGetSymbolAddress returns, looked
// up once per device at the first call with that device current.
//
// Calls on one device share the array and keep the last call's contents;
// whatever must start from zero is cleared by a kernel at every call.
// Calls that overlap on one device (asynchronous calls on two streams, or
// two host threads with TILEQR_FLAG_ASYNC) race on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/tileqr.h"
#include "tileqr_host.h"
#include "tileqr_internal.h"

using namespace tq;

namespace {

constexpr size_t kScratchBytes = (size_t)TILEQR_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (current), looked up once.
int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices) return TILEQR_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                             "hipGetSymbolAddress(scratch)");
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return 0;
}

}  // namespace

extern "C" int tileqr_factor_noalloc(int64_t m, int64_t n, double *A, int64_t lda, int64_t nb, int64_t ib,
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
    if (o.flags & (TILEQR_FLAG_TRACE | TILEQR_FLAG_TIMING)) return TILEQR_EUNSUPPORTED;
    if (!precision_supported(o.precision, ib)) return TILEQR_EUNSUPPORTED;

    std::lock_guard<std::mutex> lock(g_mu);
    hipStream_t st = (hipStream_t)o.stream;
    int dev = 0, rc;
    TQ_HIP(hipGetDevice(&dev));
    void *base = nullptr;
    if ((rc = scratch_address(dev, &base))) return rc;

    // Every buffer comes from the array, sized before anything is launched:
    // a shape that does not fit returns TILEQR_ENOMEM with A untouched.
    Arena arena;
    arena.base = (char *)base;
    arena.cap = kScratchBytes;
    Workspace W;
    W.device = dev;
    W.stream = st;
    for (DevBuf *b : {&W.tiles, &W.status, &W.vsplit, &W.sched.counters, &W.sched.qslot, &W.sched.qctl,
                      &W.sched.mats})
        b->arena = &arena;
    int cus = 0;
    TQ_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    W.num_cu = cus;
    const int p = (int)cdiv(m, nb), q = (int)cdiv(n, nb);
    if ((rc = W.status.ensure(256))) return rc;
    if ((rc = W.tiles.ensure((size_t)p * q * nb * nb * sizeof(double)))) return rc;
    MatDev M;
    std::memset(&M, 0, sizeof M);
    M.tiles = (double *)W.tiles.ptr;
    M.T = T;
    M.vsplit = nullptr;
    if (o.precision != TILEQR_FP64) {
        const int parts = o.precision == TILEQR_BF16X3 ? 3 : 2;
        if ((rc = W.vsplit.ensure(vsplit_bytes(p, std::min(p, q), (int)nb, (int)ib, parts)))) return rc;
        M.vsplit = W.vsplit.ptr;
    }
    M.p = p;
    M.q = q;
    M.task_base = 0;
    int *dstatus = (int *)W.status.ptr;
    const bool serial = (o.flags & TILEQR_FLAG_SERIAL) != 0;
    SchedDev S;
    int workers = 0;
    if (!serial) {
        std::vector<MatDev> mats(1, M);
        if ((rc = prepare_schedule(&W, W.sched, mats, (int)nb, (int)ib, o, st, S, &workers))) return rc;
    }

    // The status word starts from zero (a fill kernel, not a memset: the
    // call may sit in a captured graph).
    TQ_HIP(launch_fill_int(dstatus, 1, 0, st));
    TQ_HIP(launch_cm2tile(A, lda, m, n, M.tiles, (int)nb, p, q, dstatus, st));
    if (serial) {
        TQ_HIP(launch_factor_serial((int)nb, (int)ib, o.precision, M, dstatus, st));
    } else {
        TQ_HIP(launch_sched_init(S, st));
        TQ_HIP(launch_worker((int)nb, (int)ib, o.precision, S, workers, st));
    }
    TQ_HIP(launch_tile2cm(A, lda, m, n, M.tiles, (int)nb, p, q, dstatus, st));
    if (o.flags & TILEQR_FLAG_ASYNC) return TILEQR_OK;
    int s = 0;
    TQ_HIP(hipMemcpyAsync(&s, dstatus, sizeof s, hipMemcpyDeviceToHost, st));
    TQ_HIP(hipStreamSynchronize(st));
    if (s & STATUS_NONFINITE) return TILEQR_ENONFINITE;
    if (s & STATUS_TIMEOUT) return TILEQR_ETIMEOUT;
    return TILEQR_OK;
}
