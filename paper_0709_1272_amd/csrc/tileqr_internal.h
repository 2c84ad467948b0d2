// Internal interface between the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tq {

enum : int {
    STATUS_NONFINITE = 1,   // NaN or Inf in the input
    STATUS_TIMEOUT = 2,     // scheduler watchdog fired
    STATUS_SINGULAR = 4     // exact zero on the diagonal of R (triangular solve)
};

// One matrix as the kernels see it.
struct MatDev {
    double *tiles;       // p x q row-major nb x nb tiles (workspace)
    double *T;           // T factors (caller memory)
    void *vsplit;        // split modes: split images of V and T per TS tile and panel (workspace)
    int32_t p, q;        // tile grid
    int64_t task_base;   // first global task id of this matrix
};

// LARFB / SSRFB strip tasks per tile: 32-column strips in FP64; in the split
// modes the column-block width of the split SSRFB (64 columns for nb 128 and
// 256, 32 for nb 64).
__host__ __device__ constexpr int strips_per_tile(int nb, int prec)
{
    return prec == 0 ? nb / 32 : (nb >= 128 ? nb / 64 : nb / 32);
}

// Bytes of the split images of one matrix (p x q tiles, kmax steps): one
// block of 16-byte vectors per TS tile (k, i) and inner panel, holding V^T X
// and V W images of V (nb / 32 * 2 + nb / 16 vectors per lane and part), the
// T^T W images of T (2 per lane and part) and one header vector; laid out
// like T, by (k p + i).  parts: 3 for BF16 x3, 2 for the other splits.
inline size_t vsplit_bytes(int p, int kmax, int nb, int ib, int parts)
{
    const size_t vec = (size_t)(((nb / 32) * 2 + nb / 16 + 2) * parts * 64 + 1 + 7) / 8 * 8;
    return (size_t)kmax * p * (nb / ib) * vec * 16;
}

// Words of one trace event: type, k, i, j, strip, worker, then the device
// wall clock when the task was popped, when it started (after the acquire),
// when its body ended and when its successors were released.
constexpr int TRACE_WORDS = 10;

// Words between the head (or tail) words of two ready queues: 4 KiB, so
// that the queues' control words sit on different memory channels.
constexpr int QSTRIDE = 1024;

// Scheduler state in device memory (all pointers are device pointers).
struct SchedDev {
    MatDev *mats;
    int32_t nmat;
    int32_t ns;               // strips per tile
    int32_t np;               // GEQRT / TSQRT tasks per tile: 1 or nb / ib (one per inner panel)
    int32_t npanel;           // workgroups 0..npanel-1 take the panel role
    int64_t total_ids;        // size of the id space (with holes)
    uint32_t total_tasks;     // number of real tasks
    int32_t *counters;        // [total_ids] remaining predecessors
    int32_t *qslot;           // slots of all ready queues, back to back
    int64_t qslot_total;
    const int64_t *qoff;      // [NQUEUE] offset of each queue's slots
    uint32_t *qhead;          // [NQUEUE * QSTRIDE], word q * QSTRIDE for queue q
    uint32_t *qtail;          // [NQUEUE * QSTRIDE]
    uint32_t *done;           // completed tasks
    int32_t *status;          // STATUS_* flags
    int64_t spin_limit;       // idle polls without progress before STATUS_TIMEOUT
    int32_t shuffle;          // pseudo-random pop order
    uint64_t seed;
    int64_t drop_edge;        // debug: task whose first release is skipped (-1: none)
    int64_t *trace;           // [trace_cap * TRACE_WORDS] or NULL
    uint32_t *trace_count;
    uint32_t trace_cap;
};

// Words between two progress flags of the Q / Q^T application (256 bytes).
constexpr int PROG_STRIDE = 64;

// Applying Q or Q^T of a finished factorisation to row blocks of B.
struct ApplyDev {
    MatDev M;                 // factor tiles and T
    double *B;                // p row blocks of nb x ldb, row-major
    int32_t ldb;              // a multiple of the strip width
    int32_t nstrip;           // ldb / strip width
    int32_t ncol;             // columns that hold right-hand sides (the rest of ldb is zero padding)
    int32_t kmax;             // tile steps of the factorisation
    int32_t group = 0;        // inner panels per workgroup (0: chosen from the shape)
    int32_t *prog;            // [kmax * (nb / ib) * PROG_STRIDE] progress flags, one per 256 bytes
    int32_t *status;
    int64_t spin_limit;
};

// One matrix of a batched layout conversion.
struct ConvDesc {
    double *A;                // column-major caller matrix (device)
    int64_t lda, m, n;
    double *tiles;            // its tiles in the workspace
    int32_t p, q;
    int64_t blk0;             // index of its first 64 x 64 block in the launch
};

hipError_t launch_cm2tile_batched(const ConvDesc *D, int nmat, int64_t nblk, int nb, int *status, hipStream_t st);
hipError_t launch_tile2cm_batched(const ConvDesc *D, int nmat, int64_t nblk, int nb, const int *status,
                                  hipStream_t st);
hipError_t launch_fill_int(int *p, int n, int v, hipStream_t st);

// One matrix of a batched least-squares solve (tileqr_solve_ls_batched).
struct LsDesc {
    const double *A;          // caller's A, column-major m x n (untouched)
    int64_t lda;
    const double *b;          // caller's right-hand side (m)
    double *x;                // caller's solution (n), written
    const double *tiles;      // the factored tiles (p x q, row-major nb x nb inside)
    const double *T;          // their T blocks
    double *work;             // 7 p nb doubles of scratch
    int32_t m, n, p, q, nb, ib;
};
struct LsOut {
    double eta;               // backward error of the returned x
    int32_t iterations;       // refinement steps taken
    int32_t status;           // STATUS_* bits
};
// One workgroup per matrix: Q^T b, triangular solve and refinement to tol
// (at most max_iter steps); results in out[], status bits also or-ed into
// *status.
hipError_t launch_ls_batched(const LsDesc *descs, int count, double tol, int max_iter, LsOut *out, int *status,
                             hipStream_t st);
// Synthetic uniform(-1, 1) entries (timing runs of the tuner).
hipError_t launch_fill_uniform(double *A, int64_t count, uint64_t seed, hipStream_t st);

hipError_t launch_apply(int nb, int ib, const ApplyDev &D, bool trans, hipStream_t st);
hipError_t launch_cm2rows(const double *B, int64_t ldb, int64_t m, int64_t nrhs, double *Bt, int64_t rows, int ldt,
                          hipStream_t st);
hipError_t launch_rows2cm(double *B, int64_t ldb, int64_t m, int64_t nrhs, const double *Bt, int ldt, hipStream_t st);

// Triangular solves with the tiled R on row blocks C (ldt a multiple of 32):
// R X = C (upper) or R^T X = C, n = order of R.  One persistent launch;
// `flags` holds flags_cap ints, trsm_flags_needed(n, ldt) are needed
// (hipErrorInvalidValue otherwise).
constexpr int FLAG_STRIDE = 64;
int64_t trsm_flags_needed(int64_t n, int ldt);
hipError_t launch_trsm(int nb, const double *tiles, int p, int64_t n, double *C, int ldt, bool upper, int *flags,
                       int64_t flags_cap, int *status, int64_t spin_limit, hipStream_t st);
// Y = alpha A X + beta Y (column-major A, m x n; X, Y row blocks); `part`
// is scratch of part_cap doubles for the deterministic column-slice sums.
hipError_t launch_gemv_n(const double *A, int64_t lda, int64_t m, int64_t n, const double *X, int ldt, int nrhs,
                         double alpha, double beta, double *Y, double *part, int64_t part_cap, hipStream_t st);
// Y = alpha A^T R + beta Y; `part` is scratch of part_cap doubles for the
// deterministic row-slice sums (at least 32 n).
hipError_t launch_gemv_t(const double *A, int64_t lda, int64_t m, int64_t n, const double *R, int ldt, int nrhs,
                         double alpha, double beta, double *Y, double *part, int64_t part_cap, hipStream_t st);
// Partial sums per column of the two norm kernels below.
constexpr int COLSQ_BLOCKS = 256;
// out[v] = sum of squares of column v of Y (rows < m); part holds part_cap
// doubles and needs COLSQ_BLOCKS * nrhs (hipErrorInvalidValue otherwise).
hipError_t launch_colsq(const double *Y, int ldt, int64_t m, int nrhs, double *part, int64_t part_cap, double *out,
                        hipStream_t st);
// out[0] = ||A||_F^2; part: COLSQ_BLOCKS doubles.
hipError_t launch_frob2(const double *A, int64_t lda, int64_t m, int64_t n, double *part, int64_t part_cap,
                        double *out, hipStream_t st);
// out[v] = max |Y[r][v]| over rows r < m; part as for launch_colsq.
hipError_t launch_colmax(const double *Y, int ldt, int64_t m, int nrhs, double *part, int64_t part_cap, double *out,
                         hipStream_t st);
// out[0] = ||A||_inf (largest absolute row sum of column-major A); part holds
// part_cap doubles (column-slice row sums, then COLSQ_BLOCKS maxima).
hipError_t launch_norm_inf(const double *A, int64_t lda, int64_t m, int64_t n, double *part, int64_t part_cap,
                           double *out, hipStream_t st);
// Y (row blocks, rows < rows, columns < cols of ldt) <- N(0, 1) from a
// counter-based hash of (seed, position); other columns zero.
hipError_t launch_fill_normal(double *Y, int ldt, int64_t rows, int cols, uint64_t seed, hipStream_t st);
// W = R Z (row blocks of p nb rows; R the n x n upper triangle of the tiles).
hipError_t launch_trmm(int nb, const double *tiles, int p, int64_t n, double *W, const double *Z, int ldt,
                       hipStream_t st);
// op 0: Y = X - Y, 1: Y += X, 2: Y = X, 3: Y = -Y (rows < m, columns < nrhs).
hipError_t launch_axpy_rows(const double *X, double *Y, int ldt, int64_t m, int nrhs, int op, hipStream_t st);

hipError_t launch_cm2tile(const double *A, int64_t lda, int64_t m, int64_t n, double *tiles, int nb,
                          int p, int q, int *status, hipStream_t st);
hipError_t launch_tile2cm(double *A, int64_t lda, int64_t m, int64_t n, const double *tiles, int nb,
                          int p, int q, const int *status, hipStream_t st);
// Arithmetic of the block-reflector products (the values of tileqr_precision):
// 0 FP64; 1, 2, 3 split BF16 x2, FP16 x2, BF16 x3 on the narrow MFMAs with
// FP32 accumulation (ib = 32 only) in every block-reflector product; the
// reflectors and T are always formed in FP64.
hipError_t launch_factor_serial(int nb, int ib, int prec, const MatDev &M, const int *status, hipStream_t st);
hipError_t launch_sched_init(const SchedDev &S, hipStream_t st);
// The persistent scheduler: `workers` workgroups, the first S.npanel of
// which run the panel tasks (GEQRT, TSQRT) and the others the updates
// (LARFB, SSRFB).
hipError_t launch_worker(int nb, int ib, int prec, const SchedDev &S, int workers, hipStream_t st);
int worker_occupancy(int nb, int ib, int prec);

// The split-precision instantiations (one object per arithmetic, ib = 32).
template <int PREC> hipError_t launch_serial_mx(int nb, const MatDev &M, const int *status, hipStream_t st);
template <int PREC> hipError_t launch_worker_mx(int nb, const SchedDev &S, int workers, hipStream_t st);
template <int PREC> int worker_occupancy_mx(int nb);

}  // namespace tq
