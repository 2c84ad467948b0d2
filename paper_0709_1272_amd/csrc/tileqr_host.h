// Host-side internals shared by the library's translation units: error
// reporting, device workspaces and the set-up of the persistent scheduler.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/tileqr.h"
#include "tileqr_dag.h"
#include "tileqr_internal.h"

namespace tq {

// Records the failed call in the text tileqr_last_hip_error returns.
int hip_fail(hipError_t e, const char *what);

#define TQ_HIP(expr)                                      \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

constexpr int kStripWidth = 32;   // columns per LARFB/SSRFB strip task

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// A fixed region of device memory that buffers are carved from in order
// (256-byte aligned), for calls that must not allocate.
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
};

// Grow-only device buffer.  With `arena` set, ensure() takes the buffer from
// the arena instead of allocating, and fails with TILEQR_ENOMEM when the
// arena is too small; release() then frees nothing.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    Arena *arena = nullptr;
    int ensure(size_t need);
    void release();
};

// Device arrays of one persistent-scheduler launch: in-degree counters,
// queue slots, queue heads / tails / counters and the matrix list.
struct SchedBufs {
    DevBuf counters, qslot, qctl, mats;
    void release();
};

// Best blocking and schedule found by tileqr_tune for a set of shapes, on a
// device of architecture `arch` with `cu` compute units.
struct TuneEntry {
    std::string arch;
    int cu = 0;
    std::vector<int64_t> key;      // precision, batch, then (m, n) sorted
    std::vector<int64_t> bucket;   // size class of the key (tune_bucket)
    tileqr_tuning best;
};

// Library workspace of one (device, stream) pair: calls on different
// streams never share buffers, so asynchronous calls on two streams (or a
// captured graph and calls on another stream) cannot race on them.
struct Workspace {
    int device = -1;
    hipStream_t stream = nullptr;
    DevBuf tiles, status, trace, misc, rows, prog, tws, solve, part, tflags;
    DevBuf vsplit;                        // split images of V and T (split modes)
    DevBuf luinv;                         // tiled LU: the inverses of the L_up triangles
    DevBuf lulup, lupiv;                  // tiled LU solve: its own L_up and pivots
    SchedBufs sched;                      // single-matrix calls
    // Batched calls keep their own buffers so that a captured graph stays
    // valid across single-matrix calls.
    DevBuf btiles, bconv, bvsplit;
    DevBuf lsT, lswork, lsdesc, lsout;    // batched least squares
    std::vector<SchedBufs> bsched;        // one per (nb, ib) group
    hipGraphExec_t bgraph = nullptr;
    std::vector<int64_t> bgraph_key;
    hipStream_t cap_stream = nullptr;     // private stream for graph capture
    double *host_small = nullptr;         // pinned, for norms read back by the solver
    int *host_status = nullptr;           // pinned
    int64_t trace_events = 0;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double last_ms[4] = {0, 0, 0, 0};
    bool have_timing = false;
    int num_cu = 0;
    double wall_hz = 0.0;
};

extern std::mutex g_mu;
// The workspace of the current device and `stream`, created on first use
// (nullptr without a device).
Workspace *workspace(hipStream_t stream);
// Workspaces of the last synchronous timed call and of the last traced call.
extern Workspace *g_last_timed;
extern Workspace *g_last_traced;
// The tuner's table (entries made by tileqr_tune or loaded from a file, for
// any device); with create == false, nullptr while it is empty.
std::vector<TuneEntry> *tuned_entries(bool create);
// tileqr_choose_blocking for callers that hold g_mu.
void choose_blocking_held(int64_t m, int64_t n, int precision, int64_t *nb, int64_t *ib);
// Blocking and schedule tileqr_tune found for one m x n matrix (g_mu held).
bool tuned_single(int64_t m, int64_t n, int precision, tileqr_tuning *out);

// Split precisions need ib = 32.
bool precision_supported(int precision, int64_t ib);
// opts.panel_tasks is 0 (automatic), 1 or nb / ib.
bool panel_tasks_ok(int64_t panel_tasks, int64_t nb, int64_t ib);
// Reads the device status word (synchronises st) and maps it to a status.
int check_status(Workspace *W, int *dstatus, hipStream_t st);

// Scheduler set-up for matrices that share (nb, ib): assigns task_base,
// counts the tasks of every ready queue, uploads the matrix list and queue
// offsets on st and fills S.  npanel: panel-role workgroups (0 = automatic);
// nupdate: update-role workgroups (0 = all that fit).  Returns the launch
// width in *workers.
int prepare_schedule(Workspace *W, SchedBufs &B, std::vector<MatDev> &mats, int nb, int ib, const tileqr_opts &o,
                     hipStream_t st, SchedDev &S, int *workers);

}  // namespace tq
