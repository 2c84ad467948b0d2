// Device-side building blocks of the tiled QR (Section 3.2.1, Algorithm 2)
// for gfx950: tile kernels GEQRT / TSQRT / LARFB / SSRFB and the
// persistent DAG scheduler that runs them (Section 4).  Included by the
// translation units that instantiate the kernels for each arithmetic.
//
// Storage.  The matrix is copied into Block Data Layout (Section 3: tiles
// stored contiguously): tile (i, j) of nb x nb doubles sits at
// tiles + (j * p + i) * nb * nb and is ROW-major inside, so that the 16-wide
// column blocks the MFMA lanes own are 128-byte contiguous runs.  Ragged edges
// are zero-padded: a zero row or column changes no reflector (its entries
// add exact zeros to every norm and dot product, and a zero column below the
// diagonal yields tau = 0), so padded tiles factor exactly like the paper's
// pb x qb matrix.
//
// T factors.  Inner blocking (Section 3.2.3) gives one ib x ib upper
// triangular T_l per group of ib reflectors; the t = nb/ib blocks of tile
// (i, k) sit at T + (k * p + i) * ib * nb + l * ib * ib, row-major.
//
// Block reflector convention.  For forward-accumulated reflectors
// H_1 ... H_s = I - V T V^T, so Q^T = I - V T^T V^T.  The paper writes the
// LARFB/SSRFB updates as (I - V T V^T) applied to the tiles; applying Q^T
// needs T^T, which is what every update below does.
//
// Work unit.  Every task runs on one workgroup of nb/32 wave64s (2 nb
// threads), each wave owning 32 rows of a tile.  The GEMM-shaped parts use
// v_mfma_f64_16x16x4_f64.  For this instruction lane L (n = L % 16,
// g = L / 16) supplies A[n][g] and B[g][n] and holds D[4 r + g][n] in
// accumulator element r (r = 0..3).  A tile strip of 32 columns is held in
// accumulators: element r of row block rb (0..1) of wave w is row
// 32 w + 16 rb + 4 r + g, column 16 cb + n.  The same registers then serve
// directly as the B operand of the product V^T X (rows as the contracted
// index: K-chunk r covers rows 16 rb + 4 r .. + 3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "tileqr_dag.h"
#include "tileqr_internal.h"

namespace tq {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
// Tile and T pointers reach the kernels through structures in device memory,
// so the compiler cannot tell them from LDS or scratch pointers and would use
// flat instructions; the explicit global address space gives global loads and
// stores, which do not hold up LDS traffic behind the same counters.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) v2d gv2d;

constexpr int WS = 32;    // strip width (columns) of the GEMM-shaped kernels
constexpr int CB = WS / 16;

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int NB, int IB>
struct Cfg {
    static constexpr int NW = NB / 32;       // waves per workgroup
    static constexpr int NT = 64 * NW;       // threads per workgroup (= 2 nb, the launch bound)
    static constexpr int NSLOT = NW;         // LDS slots of the cross-wave reduction (one per wave)
    static constexpr int RB = 2;             // 16-row blocks per wave
    static constexpr int IBB = IB / 16;      // 16-wide blocks of the ib dimension
    static constexpr int NPAN = NB / IB;     // inner panels per tile
    static constexpr int LDP = IB + 2;       // LDS row stride of the panel buffer (16-byte rows)
    static constexpr int RG = NT / IB;       // row groups of the panel factorisation
    static constexpr int RPT = NB / RG;      // panel rows per thread
    static constexpr int NS = NB / WS;       // strips per tile
    static constexpr int VPT = NB * IB / 2 / NT;              // double2 per thread, full panel
    static constexpr int TPT = (IB * IB / 2 + NT - 1) / NT;   // double2 per thread, one T
    static constexpr int EPT = IB * WS / NT;                  // W entries per thread
    static_assert(NB % 64 == 0 && IB % 16 == 0 && NB % IB == 0 && IB <= WS, "blocking");
    static_assert(VPT >= 1 && EPT >= 1, "workgroup shape");
};

// A 32-column strip of a tile in accumulator layout (see the file header).
template <int NB, int IB>
struct Strip {
    d4 v[Cfg<NB, IB>::RB][CB];
};

// Register staging of one inner panel (nb x ib) and its T, so that the
// global loads of the next panel are in flight while the current one is
// being applied.
template <int NB, int IB>
struct Stage {
    v2d v[Cfg<NB, IB>::VPT];
    v2d t[Cfg<NB, IB>::TPT];
};

template <int NB, int IB>
struct alignas(16) Smem {
    using C = Cfg<NB, IB>;
    double P[(NB + IB) * C::LDP];    // panel / V: rows 0..nb-1 tile rows, nb.. head rows
    union {
        // Per-wave partial products, one slot per wave; their sum (W, or
        // the Gram matrix V^T V) is formed in place in slot 0.
        double Wp[C::NSLOT * IB * WS];
        // Reflector broadcast of the panel factorisation (double-buffered by
        // column parity); never live at the same time as the slots.
        double xb[2][NB];
    };
    double Wb[IB * WS];              // T^T W
    double Tl[IB * IB];              // T of the current inner panel
    double tau[IB];
    double sc[2][2];                 // tau of the broadcast reflector
    static_assert(C::NSLOT * IB * WS >= 2 * NB, "the broadcast buffers fit in the slots");
};

// ------------------------------------------------------------------ helpers

// The thread's index.  A unit that defines TQ_OPAQUE_TID to 1 makes it opaque
// to the optimiser, so that addresses derived from it are formed inside each
// task instead of being hoisted out of the persistent loop, where the task
// bodies of every role would keep all of them live at once.  The split units
// need that: their update tasks hold a 128 x 16 FP64 block per wave, and the
// hoisted addresses on top of it spill.  The FP64 units keep the index
// transparent: their hoisted addresses fit, and forming them per task is the
// slower of the two there.
#ifndef TQ_OPAQUE_TID
#define TQ_OPAQUE_TID 0
#endif
__device__ __forceinline__ int tidx()
{
    int t = threadIdx.x;
    if constexpr (TQ_OPAQUE_TID != 0) asm volatile("" : "+v"(t));
    return t;
}
__device__ __forceinline__ int lane_id() { return tidx() & 63; }
__device__ __forceinline__ int wave_id() { return tidx() >> 6; }

__device__ __forceinline__ gdouble *tile_ptr(const MatDev &M, int nb, int i, int j)
{
    return (gdouble *)(M.tiles + ((size_t)j * M.p + i) * (size_t)nb * nb);
}

__device__ __forceinline__ gdouble *tblock_ptr(const MatDev &M, int nb, int ib, int k, int i)
{
    return (gdouble *)(M.T + ((size_t)k * M.p + i) * (size_t)ib * nb);
}

// Stage <- columns [c0, c0 + ib) of rows [r0, nb) of a row-major tile
// (rows above r0 read as zero) and, with HAS_T, the ib x ib T block at Tg
// (else zeros).  Every thread issues the same loads whatever r0 (the rows
// above it are read and dropped), so that the compiler's count of loads in
// flight is exact and a later wait for older loads does not also wait for
// these.
template <int NB, int IB, bool HAS_T = true>
__device__ __forceinline__ void stage_load(Stage<NB, IB> &S, const gdouble *tile, int c0, int r0,
                                           const gdouble *Tg)
{
    using C = Cfg<NB, IB>;
    constexpr int H = IB / 2, TE = IB * IB / 2;
#pragma unroll
    for (int u = 0; u < C::VPT; ++u) {
        const int e = tidx() + u * C::NT, r = e / H, c2 = e % H;
        const v2d x = *reinterpret_cast<const gv2d *>(tile + (size_t)r * NB + c0 + 2 * c2);
        S.v[u] = r >= r0 ? x : v2d{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < C::TPT; ++u) {
        const int e = tidx() + u * C::NT;
        if constexpr (HAS_T) {
            const v2d t = reinterpret_cast<const gv2d *>(Tg)[e < TE ? e : TE - 1];
            S.t[u] = e < TE ? t : v2d{0.0, 0.0};
        } else {
            S.t[u] = v2d{0.0, 0.0};
        }
    }
}

// sm.P rows [r0, nb) <- staged panel; with `unit` the block's unit lower
// triangle is made explicit (ones on the diagonal of rows c0.., zeros above).
template <int NB, int IB>
__device__ __forceinline__ void stage_store(Smem<NB, IB> &sm, const Stage<NB, IB> &S, int r0, bool unit,
                                            int c0)
{
    using C = Cfg<NB, IB>;
    constexpr int H = IB / 2;
#pragma unroll
    for (int u = 0; u < C::VPT; ++u) {
        const int e = tidx() + u * C::NT, r = e / H, c = 2 * (e % H);
        if (r < r0) continue;
        double a = S.v[u].x, b = S.v[u].y;
        if (unit) {
            const int d = r - c0;
            a = d < c ? 0.0 : (d == c ? 1.0 : a);
            b = d < c + 1 ? 0.0 : (d == c + 1 ? 1.0 : b);
        }
        *reinterpret_cast<v2d *>(&sm.P[r * C::LDP + c]) = v2d{a, b};
    }
#pragma unroll
    for (int u = 0; u < C::TPT; ++u) {
        const int e = tidx() + u * C::NT;
        if (e < IB * IB / 2) reinterpret_cast<v2d *>(sm.Tl)[e] = S.t[u];
    }
}

// Staging for the update tasks with the rows split by wave: wave w loads
// and stores rows 32 w .. 32 w + 31 of the panel, the only rows its own
// products read (VᵀX and V W both take the wave's 32 rows).  No workgroup
// barrier is then needed between staging a panel and using it, nor before
// overwriting it with the next one.  Same contents as stage_load /
// stage_store.
template <int NB, int IB>
__device__ __forceinline__ int stage_row(int u)
{
    constexpr int H = IB / 2, RPP = 64 / H;   // column pairs per row, rows per pass
    return wave_id() * 32 + lane_id() / H + RPP * u;
}

template <int NB, int IB>
__device__ __forceinline__ void stage_load_rows(Stage<NB, IB> &S, const gdouble *tile, int c0, int r0, const gdouble *Tg)
{
    using C = Cfg<NB, IB>;
    constexpr int H = IB / 2, TE = IB * IB / 2;
    static_assert(C::VPT * (64 / H) == 32, "one pass per group of rows");
    const int c2 = lane_id() % H;
#pragma unroll
    for (int u = 0; u < C::VPT; ++u) {
        const int r = stage_row<NB, IB>(u);
        const v2d x = *reinterpret_cast<const gv2d *>(tile + (size_t)r * NB + c0 + 2 * c2);
        S.v[u] = r >= r0 ? x : v2d{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < C::TPT; ++u) {
        const int e = tidx() + u * C::NT;
        const v2d t = reinterpret_cast<const gv2d *>(Tg)[e < TE ? e : TE - 1];
        S.t[u] = e < TE ? t : v2d{0.0, 0.0};
    }
}

template <int NB, int IB>
__device__ __forceinline__ void stage_store_rows(Smem<NB, IB> &sm, const Stage<NB, IB> &S, int r0, bool unit, int c0)
{
    using C = Cfg<NB, IB>;
    constexpr int H = IB / 2;
    const int c = 2 * (lane_id() % H);
#pragma unroll
    for (int u = 0; u < C::VPT; ++u) {
        const int r = stage_row<NB, IB>(u);
        if (r < r0) continue;
        double a = S.v[u].x, b = S.v[u].y;
        if (unit) {
            const int d = r - c0;
            a = d < c ? 0.0 : (d == c ? 1.0 : a);
            b = d < c + 1 ? 0.0 : (d == c + 1 ? 1.0 : b);
        }
        *reinterpret_cast<v2d *>(&sm.P[r * C::LDP + c]) = v2d{a, b};
    }
#pragma unroll
    for (int u = 0; u < C::TPT; ++u) {
        const int e = tidx() + u * C::NT;
        if (e < IB * IB / 2) reinterpret_cast<v2d *>(sm.Tl)[e] = S.t[u];
    }
    // The wave reads these rows next: keep the compiler from moving its
    // LDS accesses across (the hardware runs one wave's LDS accesses in order).
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// X (accumulator layout) <- strip of a row-major tile: columns
// [col0, col0 + 16 cbn), rows of every row block.
template <int NB, int IB>
__device__ __forceinline__ void load_strip(Strip<NB, IB> &X, const gdouble *tile, int ld, int col0, int cbn)
{
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = wave_id() * 32;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rowbase + rb * 16 + 4 * r + g;
                X.v[rb][cb][r] = cb < cbn ? tile[(size_t)row * ld + col0 + cb * 16 + n] : 0.0;
            }
}

// Strip -> rows [rlo, rhi) of a row-major tile (both multiples of 16).
template <int NB, int IB>
__device__ __forceinline__ void store_strip(const Strip<NB, IB> &X, gdouble *tile, int ld, int col0, int cbn,
                                            int rlo, int rhi = NB)
{
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = wave_id() * 32;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        if (rowbase + rb * 16 < rlo || rowbase + rb * 16 >= rhi) continue;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            if (cb >= cbn) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rowbase + rb * 16 + 4 * r + g;
                tile[(size_t)row * ld + col0 + cb * 16 + n] = X.v[rb][cb][r];
            }
        }
    }
}

// Rows [rfrom, nb) of a full strip (rfrom a multiple of 16) -> columns
// 0 .. 31 of the panel buffer sm.P.
template <int NB, int IB>
__device__ __forceinline__ void strip_to_panel(Smem<NB, IB> &sm, const Strip<NB, IB> &X, int rfrom)
{
    using C = Cfg<NB, IB>;
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = wave_id() * 32;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        if (rowbase + rb * 16 < rfrom) continue;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.P[(rowbase + rb * 16 + 4 * r + g) * C::LDP + cb * 16 + n] = X.v[rb][cb][r];
    }
}

// Per-wave partial accumulators (BA x BB blocks of 16 x 16 in accumulator
// layout, row stride ld) -> sm.Wp slot w (the wave's own).  Ends with a
// barrier; sum_slots then adds the slots in wave order.
// GMAJ selects the accumulator row order: element r of lane group g is row
// 4 r + g (FP64 MFMA) or 4 g + r (the 16x16x32 narrow MFMAs).
template <int NB, int IB, int BA, int BB, bool GMAJ = false>
__device__ __forceinline__ void waves_to_slots(Smem<NB, IB> &sm, const d4 (&acc)[BA][BB], int ld)
{
    constexpr int SLOT = IB * WS;
    const int w = wave_id(), n = lane_id() & 15, g = lane_id() >> 4;
    const int gm = GMAJ ? 4 : 1, rm = GMAJ ? 1 : 4;
#pragma unroll
    for (int a = 0; a < BA; ++a)
#pragma unroll
        for (int b = 0; b < BB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sm.Wp[w * SLOT + (a * 16 + rm * r + gm * g) * ld + b * 16 + n] = acc[a][b][r];
    __syncthreads();
}

template <int NB, int IB>
__device__ __forceinline__ double sum_slots(const Smem<NB, IB> &sm, int e)
{
    constexpr int SLOT = IB * WS;
    double s = sm.Wp[e];
#pragma unroll
    for (int q = 1; q < Cfg<NB, IB>::NSLOT; ++q) s += sm.Wp[q * SLOT + e];
    return s;
}

// Rows 0..ib-1, columns 0..ncol-1 of the coupled upper tile block `top`
// (row stride ldtop) -> registers in the entry order of the reduced W in
// sm.Wp slot 0 (entry e = tid + u * NT is row e / WS, column e % WS;
// columns from ncol on read as zero).  The callers issue these loads ahead of the next panel's
// prefetch, so that waiting for them does not wait for the prefetch.
template <int NB, int IB>
__device__ __forceinline__ void load_top(double (&tv)[(Cfg<NB, IB>::EPT)], const gdouble *top, int ldtop, int ncol)
{
    using C = Cfg<NB, IB>;
#pragma unroll
    for (int u = 0; u < C::EPT; ++u) {
        const int e = tidx() + u * C::NT, kr = e / WS, c = e % WS;
        tv[u] = (top != nullptr && c < ncol) ? top[(size_t)kr * ldtop + c] : 0.0;
    }
}

// top <- tv - sm.Wb over the entries load_top read (a store only: the old
// values are already in tv).
template <int NB, int IB>
__device__ __forceinline__ void store_top(const Smem<NB, IB> &sm, const double (&tv)[Cfg<NB, IB>::EPT], gdouble *top,
                                          int ldtop, int ncol)
{
    using C = Cfg<NB, IB>;
#pragma unroll
    for (int u = 0; u < C::EPT; ++u) {
        const int e = tidx() + u * C::NT, kr = e / WS, c = e % WS;
        if (c < ncol) top[(size_t)kr * ldtop + c] = tv[u] - sm.Wb[e];
    }
}

// Apply the block reflector of one inner panel, held in LDS (sm.P rows
// 0..nb-1 = V, rows below `rlo` ignored; sm.Tl = T), to a strip X:
//   W = [top +] V^T X;  W <- T^T W;  [top -= W;]  X -= V W
// (with TRANS == false, W <- T W: the reflector itself instead of its
// transpose).
// `top` (may be NULL) points at the ib x (16 cbn) block of the coupled upper
// tile (the R rows the TS form also updates), row stride ldtop; tv holds
// that block as load_top read it.
// Three workgroup barriers; the products V^T X, T^T W and V W run on MFMA.
// With SKIP the column blocks from cbn on (which the caller neither loaded
// nor stores) are left out of the products; every output column depends
// only on its own input column, so the others come out the same.
template <int NB, int IB, bool TRANS = true, bool SKIP = false>
__device__ __forceinline__ void apply_panel(Smem<NB, IB> &sm, Strip<NB, IB> &X, int rlo, gdouble *top, int ldtop, int cbn,
                                            const double (&tv)[Cfg<NB, IB>::EPT])
{
    using C = Cfg<NB, IB>;
    const int tid = tidx(), w = wave_id();
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = w * 32;
    const int ncol = cbn * 16;
    auto live = [&](int cb) { return !SKIP || cb < cbn; };

    // W partial over this wave's rows.
    d4 Wacc[C::IBB][CB];
#pragma unroll
    for (int a = 0; a < C::IBB; ++a)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) Wacc[a][cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb) {
        if (rowbase + rb * 16 < rlo) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double *vrow = &sm.P[(rowbase + rb * 16 + 4 * r + g) * C::LDP + n];
#pragma unroll
            for (int a = 0; a < C::IBB; ++a) {
                const double va = vrow[a * 16];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
                    if (live(cb)) Wacc[a][cb] = mfma(va, X.v[rb][cb][r], Wacc[a][cb]);
            }
        }
    }
    waves_to_slots<NB, IB, C::IBB, CB>(sm, Wacc, WS);
#pragma unroll
    for (int u = 0; u < C::EPT; ++u) {
        const int e = tid + u * C::NT, c = e % WS;
        double s = sum_slots<NB, IB>(sm, e);
        if (top != nullptr && c < ncol) s = tv[u] + s;
        sm.Wp[e] = s;
    }
    __syncthreads();
    // T^T W: one 16 x 16 output block per wave.
    for (int blk = w; blk < C::IBB * CB; blk += C::NW) {
        const int a = blk / CB, cb = blk % CB;
        if (!live(cb)) continue;
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < IB / 4; ++kc)
            acc = mfma(TRANS ? sm.Tl[(4 * kc + g) * IB + a * 16 + n] : sm.Tl[(a * 16 + n) * IB + 4 * kc + g],
                       sm.Wp[(4 * kc + g) * WS + cb * 16 + n], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) sm.Wb[(a * 16 + 4 * r + g) * WS + cb * 16 + n] = acc[r];
    }
    __syncthreads();
    if (top != nullptr) store_top<NB, IB>(sm, tv, top, ldtop, ncol);
    // X -= V (T^T W)
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb) {
        if (rowbase + rb * 16 < rlo) continue;
#pragma unroll
        for (int kc = 0; kc < IB / 4; ++kc) {
            const double va = sm.P[(rowbase + rb * 16 + n) * C::LDP + 4 * kc + g];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                if (!live(cb)) continue;
                const double wb = -sm.Wb[(4 * kc + g) * WS + cb * 16 + n];
                X.v[rb][cb] = mfma(va, wb, X.v[rb][cb]);
            }
        }
    }
}

// ------------------------------------------------ split-precision products
//
// Mixed arithmetic for the GEMM-shaped updates (LARFB, SSRFB).  Every FP64
// operand x is written as a sum of narrow numbers x ~ x0 + x1 [+ x2]: x0 is x
// rounded to the narrow format and each further part is the rounded
// remainder (the remainders are exact in FP64).  A product of two split
// operands is the sum of the partial products that matter, run on
// v_mfma_f32_16x16x32_{bf16,f16} with FP32 accumulation:
//   PREC_BF16X2  2 bf16 parts; x0 y0 + x0 y1 + x1 y0 (16 significant bits)
//   PREC_FP16X2  2 fp16 parts, same three products (22 bits); V is scaled
//                by 2^12 (|v| <= 1)
//   PREC_BF16X3  3 bf16 parts; the six products of combined order <= 2
// In every mode each column of the right operand is scaled by a power of two
// so that its largest entry lands in [2^14, 2^15): the parts then stay in the
// narrow format's range whatever the magnitude of the column.
// The partial products of one wave (32 rows: one K step) are accumulated in
// FP32, converted to FP64, unscaled (exact) and summed across waves in FP64;
// reflectors, T, T^T W and the update of the coupled top tile stay FP64.
//
// Lane layout of the 16x16x32 instructions (checked on the device): lane L
// (n = L % 16, g = L / 16) supplies A[n][8 g + e] and B[8 g + e][n] in element
// e (0..7) and holds D[4 g + r][n] in element r (0..3).  Both contractions
// use the same trick as the FP64 path: the K index is permuted so that the
// strip's accumulator registers are the B operand of V^T X as they stand
// (element 4 rb + r of lane group g is row 16 rb + 4 r + g), and the rows of
// the A operand of V W are permuted (A row m is tile row 16 rb + 4 (m % 4) +
// m / 4) so that the result lands in the strip's own register layout.

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

enum { PREC_FP64 = 0, PREC_BF16X2 = 1, PREC_FP16X2 = 2, PREC_BF16X3 = 3 };

template <int PREC> struct Narrow;
template <> struct Narrow<PREC_BF16X2> { typedef bf8 vec; typedef __bf16 elem; static constexpr int NPART = 2; };
template <> struct Narrow<PREC_FP16X2> { typedef h8 vec; typedef _Float16 elem; static constexpr int NPART = 2; };
template <> struct Narrow<PREC_BF16X3> { typedef bf8 vec; typedef __bf16 elem; static constexpr int NPART = 3; };

template <int PREC>
struct Parts {
    typename Narrow<PREC>::vec p[Narrow<PREC>::NPART];
};

// P <- the narrow parts of x * scale (scale a power of two).
template <int PREC>
__device__ __forceinline__ void split8(const double (&x)[8], double scale, Parts<PREC> &P)
{
    using E = typename Narrow<PREC>::elem;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        double r = x[e] * scale;
#pragma unroll
        for (int q = 0; q < Narrow<PREC>::NPART; ++q) {
            const E h = (E)(float)r;
            P.p[q][e] = h;
            r = r - (double)(float)h;
        }
    }
}

template <int PREC>
__device__ __forceinline__ f4 mfma_narrow(const typename Narrow<PREC>::vec &a, const typename Narrow<PREC>::vec &b,
                                          f4 c)
{
    if constexpr (PREC == PREC_FP16X2) return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Sum of the kept partial products, smallest terms first.
template <int PREC>
__device__ __forceinline__ f4 split_product(const Parts<PREC> &A, const Parts<PREC> &B)
{
    f4 c = {0.f, 0.f, 0.f, 0.f};
    if constexpr (Narrow<PREC>::NPART == 3) {
        c = mfma_narrow<PREC>(A.p[2], B.p[0], c);
        c = mfma_narrow<PREC>(A.p[0], B.p[2], c);
        c = mfma_narrow<PREC>(A.p[1], B.p[1], c);
    }
    c = mfma_narrow<PREC>(A.p[1], B.p[0], c);
    c = mfma_narrow<PREC>(A.p[0], B.p[1], c);
    c = mfma_narrow<PREC>(A.p[0], B.p[0], c);
    return c;
}

// Power-of-two scale (and its inverse) for the fp16 parts of one column of
// an MFMA operand whose 32 entries sit in lanes n, n + 16, n + 32, n + 48.
__device__ __forceinline__ void column_scale(const double (&x)[8], double &scale, double &inv)
{
    double m = 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) m = fmax(m, fabs(x[e]));
    m = fmax(m, __shfl_xor(m, 16));
    m = fmax(m, __shfl_xor(m, 32));
    int ex = 0;
    if (m > 0.0) (void)frexp(m, &ex);   // m = f 2^ex, f in [0.5, 1)
    ex = ex < -1000 ? -1000 : (ex > 1000 ? 1000 : ex);
    scale = ldexp(1.0, 15 - ex);
    inv = ldexp(1.0, ex - 15);
}

// apply_panel (Q^T direction) with the two large products in split
// precision; ib = 32 so that each wave's share of a product is one K step.
// Waves whose 32 rows lie above rlo (a multiple of 32) sit the products out.
template <int NB, int IB, int PREC>
__device__ __forceinline__ void apply_panel_mx(Smem<NB, IB> &sm, Strip<NB, IB> &X, int rlo, gdouble *top, int ldtop,
                                               const double (&tv)[Cfg<NB, IB>::EPT])
{
    using C = Cfg<NB, IB>;
    static_assert(IB == 32, "split-precision updates take ib = 32");
    // Every right operand column is scaled by a power of two (exact): FP16
    // needs it for its narrow exponent range, the BF16 splits for entries
    // beyond the FP32 range their parts pass through.  V (|v| <= 1) needs
    // it only for FP16, whose low parts would otherwise go subnormal.
    constexpr bool SCALED = true;
    constexpr double VSCALE = PREC == PREC_FP16X2 ? 4096.0 : 1.0;
    const int tid = tidx(), w = wave_id();
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = w * 32;
    const bool active = rowbase >= rlo;

    // This wave's share of V^T X.
    d4 Wacc[C::IBB][CB];
    if (active) {
        Parts<PREC> Bx[CB];
        double xinv[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            double xv[8];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) xv[4 * rb + r] = X.v[rb][cb][r];
            double sc = 1.0;
            xinv[cb] = 1.0;
            if constexpr (SCALED) column_scale(xv, sc, xinv[cb]);
            split8<PREC>(xv, sc, Bx[cb]);
        }
#pragma unroll
        for (int a = 0; a < C::IBB; ++a) {
            double vv[8];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) vv[4 * rb + r] = sm.P[(rowbase + 16 * rb + 4 * r + g) * C::LDP + a * 16 + n];
            Parts<PREC> Av;
            split8<PREC>(vv, VSCALE, Av);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const f4 d = split_product<PREC>(Av, Bx[cb]);
                const double un = SCALED ? xinv[cb] * (1.0 / VSCALE) : 1.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) Wacc[a][cb][r] = SCALED ? (double)d[r] * un : (double)d[r];
            }
        }
    } else {
#pragma unroll
        for (int a = 0; a < C::IBB; ++a)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) Wacc[a][cb] = d4{0.0, 0.0, 0.0, 0.0};
    }
    waves_to_slots<NB, IB, C::IBB, CB, true>(sm, Wacc, WS);
#pragma unroll
    for (int u = 0; u < C::EPT; ++u) {
        const int e = tid + u * C::NT;
        double s = sum_slots<NB, IB>(sm, e);
        if (top != nullptr) s = tv[u] + s;
        sm.Wp[e] = s;
    }
    __syncthreads();
    // T^T W in FP64: one 16 x 16 output block per wave.
    for (int blk = w; blk < C::IBB * CB; blk += C::NW) {
        const int a = blk / CB, cb = blk % CB;
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < IB / 4; ++kc)
            acc = mfma(sm.Tl[(4 * kc + g) * IB + a * 16 + n], sm.Wp[(4 * kc + g) * WS + cb * 16 + n], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) sm.Wb[(a * 16 + 4 * r + g) * WS + cb * 16 + n] = acc[r];
    }
    __syncthreads();
    if (top != nullptr) store_top<NB, IB>(sm, tv, top, ldtop, WS);
    // X -= V (T^T W)
    if (active) {
        Parts<PREC> Bw[CB];
        double winv[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            double wv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) wv[e] = sm.Wb[(8 * g + e) * WS + cb * 16 + n];
            double sc = 1.0;
            winv[cb] = 1.0;
            if constexpr (SCALED) column_scale(wv, sc, winv[cb]);
            split8<PREC>(wv, sc, Bw[cb]);
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int row = rowbase + 16 * rb + 4 * (n & 3) + (n >> 2);
            double vv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) vv[e] = sm.P[row * C::LDP + 8 * g + e];
            Parts<PREC> Av;
            split8<PREC>(vv, VSCALE, Av);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const f4 d = split_product<PREC>(Av, Bw[cb]);
                const double un = SCALED ? winv[cb] * (1.0 / VSCALE) : 1.0;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    X.v[rb][cb][r] = X.v[rb][cb][r] - (SCALED ? (double)d[r] * un : (double)d[r]);
            }
        }
    }
}

// 1/d for a normal d: the hardware estimate refined by two Newton-Raphson
// steps for the reciprocal (y <- y + y (1 - d y)), which give full double
// precision (not always the correctly rounded quotient).
__device__ __forceinline__ double recip_nr(double d)
{
    double y = __builtin_amdgcn_rcp(d);
    double e = fma(-d, y, 1.0);
    y = fma(y, e, y);
    e = fma(-d, y, 1.0);
    return fma(y, e, y);
}

// sqrt(a) for a normal positive a: the hardware estimate y of 1/sqrt(a)
// refined by the coupled Newton iteration for g = a y -> sqrt(a) and
// h = y / 2 -> 1 / (2 sqrt(a)), two steps, then one residual correction
// g + (a - g^2) h.
__device__ __forceinline__ double sqrt_nr(double a)
{
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    return fma(fma(-g, g, a), h, g);
}

// Lane permutations by DPP on the two 32-bit halves of a double: xor 1 and
// xor 2 inside a quad, mirror inside 8 and inside 16 lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_perm(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum / max over the `W` consecutive lanes of a group (W a power of two
// dividing 64).  Each step pairs every lane with one of the other half of
// its current block (xor 1, xor 2, mirror in 8, mirror in 16, then xor 16
// and xor 32 across rows), so after the last step every lane holds the same
// bits: partners add the same two numbers in swapped order.
template <int W>
__device__ __forceinline__ double group_sum(double v)
{
    if (W >= 2) v += dpp_perm<0xB1>(v);
    if (W >= 4) v += dpp_perm<0x4E>(v);
    if (W >= 8) v += dpp_perm<0x141>(v);
    if (W >= 16) v += dpp_perm<0x140>(v);
    if (W >= 32) v += __shfl_xor(v, 16, 64);
    if (W >= 64) v += __shfl_xor(v, 32, 64);
    return v;
}

template <int W>
__device__ __forceinline__ double group_max(double v)
{
    if (W >= 2) v = fmax(v, dpp_perm<0xB1>(v));
    if (W >= 4) v = fmax(v, dpp_perm<0x4E>(v));
    if (W >= 8) v = fmax(v, dpp_perm<0x141>(v));
    if (W >= 16) v = fmax(v, dpp_perm<0x140>(v));
    if (W >= 32) v = fmax(v, __shfl_xor(v, 16, 64));
    if (W >= 64) v = fmax(v, __shfl_xor(v, 32, 64));
    return v;
}

}  // namespace tq

#include "tileqr_cols.h"

namespace tq {

// Householder factorisation of the ib columns held in sm.P (Section 3.2.1:
// DGEQRT's panel when ts == false, DTSQRT's when ts == true).
//   GEQRT: column j has its head (diagonal) at P row c0 + j and its tail in
//          P rows c0 + j + 1 .. nb - 1.
//   TSQRT: column j has its head at P row nb + j (row j of the triangle R)
//          and its tail in P rows 0 .. nb - 1 (the square tile); the rest of
//          R is untouched by this reflector.
// Reflector: beta = -sign(alpha) ||[alpha; x]|| (sign(0) = +1),
// tau = (beta - alpha) / beta, v = x / (alpha - beta); tau = 0 when x = 0.
// Column c is held by the RG consecutive lanes of one wave (rows rg, rg + RG,
// ... in registers), so norms and dot products reduce with lane shuffles.
// Per column one barrier: the group of column j forms its reflector and
// publishes v and tau through LDS (two buffers by column parity, so that
// column j+1 may publish while column j's updates still read), then every
// later column applies it.  The scalars take one square root and one
// division; extreme magnitudes go through a norm scaled by the largest
// entry.
template <int NB, int IB, bool TS>
__device__ __forceinline__ void panel_factor(Smem<NB, IB> &sm, int c0)
{
    using C = Cfg<NB, IB>;
    constexpr int RG = C::RG, RPT = C::RPT, LDP = C::LDP;
    static_assert(64 % RG == 0, "the threads of a column share one wave");
    static_assert(RPT % 4 == 0, "four partial sums per thread");
    // Register slot i of lane rg holds relative row rr = rg + i RG of the
    // column, absolute row rbase + rr: GEQRT counts from the diagonal block
    // (rows below nb are zero padding, which no reflector changes), so only
    // the slots i RG < ib can lie on or above a column's diagonal and need
    // a per-row test; TSQRT's tile rows are all below its head.
    constexpr int NHEAD = TS ? 0 : (IB + RG - 1) / RG;
    const int tid = tidx(), c = tid / RG, rg = tid % RG;
    const int rbase = TS ? 0 : c0;
    double pr[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int row = rbase + rg + i * RG;
        pr[i] = (TS || row < NB) ? sm.P[row * LDP + c] : 0.0;
    }
    // The later columns read the reflector buffers with a zero weight when a
    // column has no reflector (tau = 0), so they must hold finite numbers.
    for (int e = tid; e < 2 * NB; e += C::NT) (&sm.xb[0][0])[e] = 0.0;
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < IB; ++j) {
        const int hrow = NB + j;   // TSQRT: row j of the triangle, kept in P
        double *xb = sm.xb[j & 1];
        double *sc = sm.sc[j & 1];
        // tail(i): slot i is below column j's diagonal; head(i): on it.
        auto tail = [&](int i) { return TS || i >= NHEAD || rg + i * RG > j; };
        auto head = [&](int i) { return !TS && i < NHEAD && rg + i * RG == j; };
        if (c == j) {
            double alpha;
            if constexpr (TS) {
                alpha = sm.P[hrow * LDP + j];
            } else {
                double h = 0.0;
#pragma unroll
                for (int i = 0; i < NHEAD; ++i)
                    if (head(i)) h = pr[i];
                alpha = group_sum<RG>(h);   // only the owner contributes
            }
            // Sum of squares of the tail in four independent chains.
            double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const double x = tail(i) ? pr[i] : 0.0;
                q[i & 3] += x * x;
            }
            const double part = (q[0] + q[1]) + (q[2] + q[3]);
            const double sig = group_sum<RG>(part);
            double tau = 0.0, scal = 0.0, beta = alpha;
            if (sig <= 1.0e300 && sig >= 2.2250738585072014e-308 && fabs(alpha) < 1.0e150) {
                // Nothing over- or underflowed: one square root and one
                // reciprocal, 1 / (beta (alpha - beta)), give both scalars.
                const double h = sqrt_nr(alpha * alpha + sig);
                beta = alpha >= 0.0 ? -h : h;
                const double amb = alpha - beta;
                const double rd = recip_nr(beta * amb);
                scal = beta * rd;
                tau = (beta - alpha) * amb * rd;
            } else if (sig != 0.0 || group_max<RG>(part) != 0.0) {
                // Extreme magnitudes: the norm scaled by the largest entry.
                double mx = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; ++i)
                    if (tail(i)) mx = fmax(mx, fabs(pr[i]));
                const double mxa = group_max<RG>(mx);
                double p2 = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const double t = tail(i) ? pr[i] / mxa : 0.0;
                    p2 += t * t;
                }
                const double xnorm = mxa * sqrt(group_sum<RG>(p2));
                const double h = hypot(alpha, xnorm);
                beta = alpha >= 0.0 ? -h : h;
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            // (a zero tail: no reflector, tau = 0, the column stays as it is)
            if (tau != 0.0) {
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    if (tail(i)) {
                        pr[i] = pr[i] * scal;
                        xb[rg + i * RG] = pr[i];
                    }
                    if (head(i)) pr[i] = beta;
                }
                if (TS && rg == 0) sm.P[hrow * LDP + j] = beta;
            }
            if (rg == 0) {
                sc[0] = tau;
                sm.tau[j] = tau;
            }
        }
        __syncthreads();
        if (c > j) {
            // Loads of tau, v and the head entry are issued together; with
            // tau = 0 the update below subtracts exact zeros.
            const double tau = sc[0];
            double hc;
            if constexpr (TS) hc = sm.P[hrow * LDP + c];
            double q[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < RPT; ++i)
                if (tail(i)) q[i & 3] += xb[rg + i * RG] * pr[i];
            const double dot = group_sum<RG>((q[0] + q[1]) + (q[2] + q[3]));
            if constexpr (!TS) {
                double h = 0.0;
#pragma unroll
                for (int i = 0; i < NHEAD; ++i)
                    if (head(i)) h = pr[i];
                hc = group_sum<RG>(h);   // only the owner contributes
            }
            const double tw = tau * (hc + dot);
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                if (tail(i)) pr[i] -= xb[rg + i * RG] * tw;
                if (head(i)) pr[i] = hc - tw;
            }
            if (TS && rg == 0) sm.P[hrow * LDP + c] = hc - tw;
        }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int row = rbase + rg + i * RG;
        if (TS || row < NB) sm.P[row * LDP + c] = pr[i];
    }
    __syncthreads();
}

// T of the panel in sm.P (rows >= rlo; V with its unit diagonal explicit):
// G = V^T V on MFMA, then column by column (compact WY, forward)
//   T[j][j] = tau_j,  T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j]
// inside diagonal blocks of 16 (lane i builds row i of its block in
// registers: each new entry waits for one multiply-add after the previous
// one), and for ib = 32 the off-diagonal block from the two diagonal ones.
// Leaves T in sm.Tl and writes it to Tg (row-major ib x ib).
template <int NB, int IB>
__device__ __forceinline__ void build_t(Smem<NB, IB> &sm, int rlo, gdouble *Tg)
{
    using C = Cfg<NB, IB>;
    const int tid = tidx(), w = wave_id();
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = w * 32;
    d4 G[C::IBB][C::IBB];
#pragma unroll
    for (int a = 0; a < C::IBB; ++a)
#pragma unroll
        for (int b = 0; b < C::IBB; ++b) G[a][b] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb) {
        if (rowbase + rb * 16 < rlo) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double *vrow = &sm.P[(rowbase + rb * 16 + 4 * r + g) * C::LDP + n];
            double v[C::IBB];
#pragma unroll
            for (int a = 0; a < C::IBB; ++a) v[a] = vrow[a * 16];
#pragma unroll
            for (int a = 0; a < C::IBB; ++a)
#pragma unroll
                for (int b = 0; b < C::IBB; ++b) G[a][b] = mfma(v[a], v[b], G[a][b]);
        }
    }
    waves_to_slots<NB, IB, C::IBB, C::IBB>(sm, G, IB);
    for (int e = tid; e < IB * IB; e += C::NT) sm.Wp[e] = sum_slots<NB, IB>(sm, e);
    __syncthreads();
    // Diagonal blocks of 16 (T11, T22 for ib = 32) by the recurrence, on
    // wave 0: lane i < ib builds row i of its block in registers (lanes from
    // ib on repeat those rows and store nothing).  The loop has no branch,
    // so the loads of the block's tau and G entries are in flight together;
    // G is symmetric, and row j of the block holds the entries G[0:j, j]
    // contiguously.
    constexpr int HB = 16;
    if (w == 0) {
        const int i = lane_id() & (IB - 1), base = (i / HB) * HB, li = i - base;
        double tb[HB], trow[HB];
#pragma unroll
        for (int kk = 0; kk < HB; ++kk) tb[kk] = sm.tau[base + kk];
#pragma unroll
        for (int kk = 0; kk < HB; ++kk) trow[kk] = kk == li ? tb[kk] : 0.0;
#pragma unroll
        for (int j = 1; j < HB; ++j) {
            const double *grow = &sm.Wp[(base + j) * IB + base];
            double s = 0.0;
#pragma unroll
            for (int kk = 0; kk < j; ++kk) s += trow[kk] * grow[kk];
            trow[j] = li < j ? -tb[j] * s : trow[j];
        }
        if (lane_id() < IB) {
#pragma unroll
            for (int kk = 0; kk < HB; ++kk) {
                sm.Tl[i * IB + base + kk] = trow[kk];
                if constexpr (IB == 2 * HB) sm.Tl[i * IB + (HB - base) + kk] = 0.0;
            }
        }
        if constexpr (IB == 2 * HB) {
            // Off-diagonal block: the product of the two block reflectors
            // gives T12 = -T11 (V1^T V2) T22 (G12 = V1^T V2 is block (0, 1)
            // of G), two 16 x 16 x 16 products on MFMA via sm.Wb.  Only this
            // wave touches Tl and Wb here, and it runs its LDS accesses in
            // order, so the fences only keep the compiler from moving them.
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kc = 0; kc < HB / 4; ++kc)
                acc = mfma(sm.Wp[n * IB + HB + 4 * kc + g], sm.Tl[(HB + 4 * kc + g) * IB + HB + n], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.Wb[(4 * r + g) * HB + n] = acc[r];
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kc = 0; kc < HB / 4; ++kc)
                acc = mfma(sm.Tl[n * IB + 4 * kc + g], sm.Wb[(4 * kc + g) * HB + n], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) sm.Tl[(4 * r + g) * IB + HB + n] = -acc[r];
        }
    }
    __syncthreads();
    for (int e = tid; e < IB * IB; e += C::NT) Tg[e] = sm.Tl[e];
}

// ------------------------------------------------------------ tile kernels

// Trailing update inside GEQRT / TSQRT after the panel at c0 (its V in
// sm.P, its T in sm.Tl): the panel's reflector is applied to every strip
// right of it, the strip next to the panel last, with the products in the
// task's arithmetic (the reflectors themselves are always formed in FP64).  With ib equal to the
// strip width that strip is exactly the next panel, so when `chain` is set
// its result goes straight into sm.P (GEQRT also stores its rows above the
// next panel, which are final rows of R, to the tile) instead of a round
// trip through memory.
template <int NB, int IB, bool TS, int PREC>
__device__ __forceinline__ void panel_trailing(Smem<NB, IB> &sm, gdouble *tile, gdouble *tkk, int c0, bool chain)
{
    const int first = c0 + IB;
    if (first >= NB) return;
    const int rlo = TS ? 0 : c0;
    const int nst = (NB - first + WS - 1) / WS;
#pragma unroll 1
    for (int q = 0; q < nst; ++q) {
        const int col0 = first + (nst - 1 - q) * WS;
        const int cbn = min(CB, (NB - col0) / 16);
        Strip<NB, IB> X;
        load_strip<NB, IB>(X, tile, NB, col0, cbn);
        gdouble *top = TS ? tkk + (size_t)c0 * NB + col0 : nullptr;
        double tv[Cfg<NB, IB>::EPT] = {};
        if constexpr (TS) load_top<NB, IB>(tv, top, NB, cbn * 16);
        if constexpr (PREC == PREC_FP64) apply_panel<NB, IB>(sm, X, rlo, top, NB, cbn, tv);
        else apply_panel_mx<NB, IB, PREC>(sm, X, rlo, top, NB, tv);
        if (chain && q + 1 == nst) {
            if constexpr (!TS) store_strip<NB, IB>(X, tile, NB, col0, cbn, rlo, c0 + IB);
            __syncthreads();
            strip_to_panel<NB, IB>(sm, X, TS ? 0 : c0 + IB);
        } else {
            store_strip<NB, IB>(X, tile, NB, col0, cbn, rlo);
        }
    }
}

// Inner panel l of DGEQRT(A_kk) -> (V_kk, R_kk, T_kk): factor columns
// [l ib, (l+1) ib) (rows from l ib down), write V, R and T_l, and apply the
// panel's reflector to the columns right of it.  `from_lds`: the panel is
// already in sm.P (rows from l ib), chained there by panel l-1; `chain`:
// leave the next panel in sm.P (the strip next to this panel is then not
// written back below the next panel's first row).  With both false the
// panel is a self-contained task that reads and writes only memory.  Without
// `trailing` the columns right of the panel are left to PUPD tasks.
template <int NB, int IB, int PREC>
__device__ __forceinline__ void geqrt_panel(Smem<NB, IB> &sm, const MatDev &M, int k, int l, bool from_lds, bool chain,
                                            bool trailing = true)
{
    using C = Cfg<NB, IB>;
    gdouble *tkk = tile_ptr(M, NB, k, k);
    gdouble *Tk = tblock_ptr(M, NB, IB, k, k);
    const int c0 = l * IB;
    if (!from_lds) {
        Stage<NB, IB> S;
        stage_load<NB, IB, false>(S, tkk, c0, c0, nullptr);
        stage_store<NB, IB>(sm, S, c0, false, c0);
    }
    __syncthreads();
    panel_factor<NB, IB, false>(sm, c0);
    // Write R and V back; keep V with explicit unit diagonal in LDS.
    constexpr int H = IB / 2;
#pragma unroll
    for (int u = 0; u < C::VPT; ++u) {
        const int e = tidx() + u * C::NT, r = e / H, cc = 2 * (e % H);
        if (r < c0) continue;
        v2d v = *reinterpret_cast<v2d *>(&sm.P[r * C::LDP + cc]);
        *reinterpret_cast<gv2d *>(tkk + (size_t)r * NB + c0 + cc) = v;
        const int d = r - c0;
        if (d <= cc + 1) {
            v.x = d < cc ? 0.0 : (d == cc ? 1.0 : v.x);
            v.y = d < cc + 1 ? 0.0 : 1.0;
            *reinterpret_cast<v2d *>(&sm.P[r * C::LDP + cc]) = v;
        }
    }
    __syncthreads();
    build_t<NB, IB>(sm, c0, Tk + l * IB * IB);
    __syncthreads();
    if (!trailing) return;
    panel_trailing<NB, IB, false, PREC>(sm, tkk, nullptr, c0, chain);
    __syncthreads();
}

// DGEQRT(A_kk) -> (V_kk, R_kk, T_kk): the inner panels in order, each one
// chained to the next through LDS when ib equals the strip width.
template <int NB, int IB, int PREC>
__device__ __forceinline__ void task_geqrt(Smem<NB, IB> &sm, const MatDev &M, int k)
{
    constexpr bool CHAIN = IB == WS;
#pragma unroll 1
    for (int l = 0; l < Cfg<NB, IB>::NPAN; ++l) geqrt_panel<NB, IB, PREC>(sm, M, k, l, CHAIN && l > 0, CHAIN);
}

// Inner panel l of DTSQRT(R_kk, A_ik) -> (R_kk, V_ik, T_ik): factor
// [R_kk rows of panel l; columns [l ib, (l+1) ib) of A_ik], write them and
// T_l, and apply the reflector to the columns right of the panel (rows of
// the panel in R_kk, all rows of A_ik).  `from_lds` / `chain` / `trailing`
// as for geqrt_panel.
template <int NB, int IB, int PREC>
__device__ __forceinline__ void tsqrt_panel(Smem<NB, IB> &sm, const MatDev &M, int k, int i, int l, bool from_lds,
                                            bool chain, bool trailing = true)
{
    using C = Cfg<NB, IB>;
    gdouble *tkk = tile_ptr(M, NB, k, k);
    gdouble *tik = tile_ptr(M, NB, i, k);
    gdouble *Ti = tblock_ptr(M, NB, IB, k, i);
    constexpr int H = IB / 2;
    const int c0 = l * IB;
    if (!from_lds) {
        Stage<NB, IB> S;
        stage_load<NB, IB, false>(S, tik, c0, 0, nullptr);
        stage_store<NB, IB>(sm, S, 0, false, c0);
    }
    // The ib x ib triangle of R_kk at the panel (both loads of a thread in
    // flight together; the entries below its diagonal read as zero).
    {
        constexpr int TRI = (IB * IB + C::NT - 1) / C::NT;
        double tri[TRI];
#pragma unroll
        for (int u = 0; u < TRI; ++u) {
            const int e = min(tidx() + u * C::NT, IB * IB - 1);
            tri[u] = tkk[(size_t)(c0 + e / IB) * NB + c0 + e % IB];
        }
#pragma unroll
        for (int u = 0; u < TRI; ++u) {
            const int e = tidx() + u * C::NT, r = e / IB, c = e % IB;
            if (e < IB * IB) sm.P[(NB + r) * C::LDP + c] = r <= c ? tri[u] : 0.0;
        }
    }
    __syncthreads();
    panel_factor<NB, IB, true>(sm, c0);
    for (int e = tidx(); e < IB * IB; e += C::NT) {
        const int r = e / IB, c = e % IB;
        if (r <= c) tkk[(size_t)(c0 + r) * NB + c0 + c] = sm.P[(NB + r) * C::LDP + c];
    }
#pragma unroll
    for (int u = 0; u < C::VPT; ++u) {
        const int e = tidx() + u * C::NT, r = e / H, cc = 2 * (e % H);
        *reinterpret_cast<gv2d *>(tik + (size_t)r * NB + c0 + cc) =
            *reinterpret_cast<v2d *>(&sm.P[r * C::LDP + cc]);
    }
    build_t<NB, IB>(sm, 0, Ti + l * IB * IB);
    __syncthreads();
    // Split modes: the split images of V and T for the SSRFB tasks.
    if constexpr (PREC != PREC_FP64) write_vsplit<NB, IB, PREC>(sm, vsplit_ptr<NB, IB, PREC>(M, k, i, l));
    if (!trailing) return;
    panel_trailing<NB, IB, true, PREC>(sm, tik, tkk, c0, chain);
    __syncthreads();
}

// DTSQRT(R_kk, A_ik) -> (R_kk, V_ik, T_ik): the inner panels in order.
template <int NB, int IB, int PREC>
__device__ __forceinline__ void task_tsqrt(Smem<NB, IB> &sm, const MatDev &M, int k, int i)
{
    constexpr bool CHAIN = IB == WS;
#pragma unroll 1
    for (int l = 0; l < Cfg<NB, IB>::NPAN; ++l) tsqrt_panel<NB, IB, PREC>(sm, M, k, i, l, CHAIN && l > 0, CHAIN);
}

// One strip (32 columns at col0, row stride ldx) of X <- Q_kk^T X (TRANS)
// or Q_kk X, Q_kk the block reflector of the diagonal tile tkk with T
// blocks Tk.  Q_kk = H_0 ... H_{t-1} over the inner panels, so Q_kk^T runs
// the panels forward with T^T and Q_kk backward with T.
template <int NB, int IB, bool TRANS, int PREC = PREC_FP64>
__device__ __forceinline__ void apply_diag_strip(Smem<NB, IB> &sm, const gdouble *tkk, const gdouble *Tk, gdouble *x, int ldx,
                                 int col0)
{
    static_assert(PREC == PREC_FP64 || TRANS, "split precision is used for Q^T only");
    using C = Cfg<NB, IB>;
    Stage<NB, IB> S;
    const int l0 = TRANS ? 0 : C::NPAN - 1;
    stage_load_rows<NB, IB>(S, tkk, l0 * IB, l0 * IB, Tk + l0 * IB * IB);
    Strip<NB, IB> X;
    load_strip<NB, IB>(X, x, ldx, col0, CB);
    // Wait for the strip here, once: inside the loop the only loads in
    // flight are then the next panel's, and the products do not wait for them.
    __builtin_amdgcn_s_waitcnt(0);
    double tv[C::EPT] = {};
    // Each wave stages the panel rows it uses itself (stage_store_rows), so
    // the loop has only apply_panel's barriers; those also order sm.Tl's
    // rewrite after the previous panel's T^T W.
#pragma unroll 1
    for (int q = 0; q < C::NPAN; ++q) {
        const int l = TRANS ? q : C::NPAN - 1 - q;
        const int c0 = l * IB;
        stage_store_rows<NB, IB>(sm, S, c0, true, c0);
        // The next panel's prefetch (after the last panel a harmless reload
        // of this one, so that the loads issued do not depend on q).
        const int ln = q + 1 < C::NPAN ? (TRANS ? l + 1 : l - 1) : l;
        stage_load_rows<NB, IB>(S, tkk, ln * IB, ln * IB, Tk + ln * IB * IB);
        if constexpr (PREC == PREC_FP64) apply_panel<NB, IB, TRANS>(sm, X, c0, nullptr, 0, CB, tv);
        else apply_panel_mx<NB, IB, PREC>(sm, X, c0, nullptr, 0, tv);
    }
    store_strip<NB, IB>(X, x, ldx, col0, CB, 0);
}

// One strip of [top; X] <- Q_ik^T [top; X] (TRANS) or Q_ik [top; X], Q_ik
// the coupled block reflector of tile tik (reflectors [e; V2]) with T blocks
// Ti; `top` is the whole upper tile (its rows c0.. are the ones each inner
// panel touches).
template <int NB, int IB, bool TRANS, int PREC = PREC_FP64>
__device__ __forceinline__ void apply_ts_strip(Smem<NB, IB> &sm, const gdouble *tik, const gdouble *Ti, gdouble *top, int ldtop,
                               gdouble *x, int ldx, int col0)
{
    static_assert(PREC == PREC_FP64 || TRANS, "split precision is used for Q^T only");
    using C = Cfg<NB, IB>;
    Stage<NB, IB> S;
    const int l0 = TRANS ? 0 : C::NPAN - 1;
    stage_load_rows<NB, IB>(S, tik, l0 * IB, 0, Ti + l0 * IB * IB);
    Strip<NB, IB> X;
    load_strip<NB, IB>(X, x, ldx, col0, CB);
    // As in apply_diag_strip: the strip is waited for once, before the loop,
    // and each wave stages its own panel rows.
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll 1
    for (int q = 0; q < C::NPAN; ++q) {
        const int l = TRANS ? q : C::NPAN - 1 - q;
        const int c0 = l * IB;
        stage_store_rows<NB, IB>(sm, S, 0, false, c0);
        // The top rows first, then the next panel's prefetch.
        gdouble *tp = top + (size_t)c0 * ldtop + col0;
        double tv[C::EPT];
        load_top<NB, IB>(tv, tp, ldtop, WS);
        const int ln = q + 1 < C::NPAN ? (TRANS ? l + 1 : l - 1) : l;
        stage_load_rows<NB, IB>(S, tik, ln * IB, 0, Ti + ln * IB * IB);
        if constexpr (PREC == PREC_FP64) apply_panel<NB, IB, TRANS>(sm, X, 0, tp, ldtop, CB, tv);
        else apply_panel_mx<NB, IB, PREC>(sm, X, 0, tp, ldtop, tv);
    }
    store_strip<NB, IB>(X, x, ldx, col0, CB, 0);
}

// Inner panel l alone of the block reflector of tile vt applied to one
// strip (32 columns at col0) of x: H_l^T (TRANS) or H_l.  With `diag`, vt
// is a diagonal tile (V unit lower triangular from row l ib, the rows above
// untouched); otherwise the coupled TS form, whose ib top rows are rows
// [l ib, (l+1) ib) of `top`.  S holds the panel and its T as
// apply_panel_stage loaded them (the caller may issue that load early: the
// factor does not change).  Loads the strip, applies the panel and stores
// back the rows it changed, so that consecutive panels may run on
// different workgroups.
template <int NB, int IB>
__device__ __forceinline__ void apply_panel_stage(Stage<NB, IB> &S, const gdouble *vt, const gdouble *Tg, int l, bool diag)
{
    const int c0 = l * IB;
    stage_load_rows<NB, IB>(S, vt, c0, diag ? c0 : 0, Tg + l * IB * IB);
}

template <int NB, int IB, bool TRANS>
__device__ __forceinline__ void apply_one_panel(Smem<NB, IB> &sm, const Stage<NB, IB> &S, int l, bool diag,
                                                gdouble *top, int ldtop, gdouble *x, int ldx, int col0)
{
    using C = Cfg<NB, IB>;
    const int c0 = l * IB, r0 = diag ? c0 : 0;
    Strip<NB, IB> X;
    load_strip<NB, IB>(X, x, ldx, col0, CB);
    gdouble *tp = diag ? nullptr : top + (size_t)c0 * ldtop + col0;
    double tv[C::EPT] = {};
    if (!diag) load_top<NB, IB>(tv, tp, ldtop, WS);
    stage_store_rows<NB, IB>(sm, S, r0, diag, c0);
    apply_panel<NB, IB, TRANS>(sm, X, r0, tp, ldtop, CB, tv);
    // Only the rows the panel changed go back: the rows above a diagonal
    // panel may meanwhile be updated by another panel's workgroup.
    store_strip<NB, IB>(X, x, ldx, col0, CB, r0);
}

// DLARFB: strip s of A_kj <- Q_kk^T A_kj (in the split modes a strip is as
// wide as the SSRFB tasks', taken 32 columns at a time).
template <int NB, int IB, int PREC>
__device__ __forceinline__ void task_larfb(Smem<NB, IB> &sm, const MatDev &M, int k, int j, int s)
{
    constexpr int SUB = NB / strips_of<NB, PREC>() / WS;
#pragma unroll 1
    for (int u = 0; u < SUB; ++u) {
        if (u > 0) __syncthreads();
        apply_diag_strip<NB, IB, true, PREC>(sm, tile_ptr(M, NB, k, k), tblock_ptr(M, NB, IB, k, k),
                                             tile_ptr(M, NB, k, j), NB, (s * SUB + u) * WS);
    }
}

// DSSRFB: strip s of [A_kj; A_ij] <- Q_ik^T [A_kj; A_ij].
template <int NB, int IB, int PREC>
__device__ __forceinline__ void task_ssrfb(Smem<NB, IB> &sm, const MatDev &M, int k, int i, int j, int s)
{
    if constexpr (PREC == PREC_FP64)
        apply_ts_strip<NB, IB, true, PREC>(sm, tile_ptr(M, NB, i, k), tblock_ptr(M, NB, IB, k, i), tile_ptr(M, NB, k, j),
                                           NB, tile_ptr(M, NB, i, j), NB, s * WS);
    else
        task_ssrfb_cols<NB, IB, PREC>(sm, M, k, i, j, s);
}

// PUPD(k, i, l, s): one strip of a panel task's trailing update as a task of
// its own.  The block reflector of inner panel l of tile (i, k) (V read back
// from the tile, T_l from its T blocks) is applied to strip s of the same
// tile, rows from l ib on, for the diagonal tile (GEQRT, i == k), and for
// i > k (TSQRT) to the pair [R rows of panel l in strip s; strip s of A_ik].
// Same operands and the same product code as the panel task's own trailing
// update, so the result does not depend on which of the two ran it.
template <int NB, int IB, int PREC>
__device__ __forceinline__ void task_pupd(Smem<NB, IB> &sm, const MatDev &M, int k, int i, int l, int s)
{
    using C = Cfg<NB, IB>;
    const bool diag = i == k;
    gdouble *tik = tile_ptr(M, NB, i, k);
    const int c0 = l * IB, r0 = diag ? c0 : 0, col0 = s * WS;
    Stage<NB, IB> S;
    stage_load_rows<NB, IB>(S, tik, c0, r0, tblock_ptr(M, NB, IB, k, i) + l * IB * IB);
    Strip<NB, IB> X;
    load_strip<NB, IB>(X, tik, NB, col0, CB);
    gdouble *top = diag ? nullptr : tile_ptr(M, NB, k, k) + (size_t)c0 * NB + col0;
    double tv[C::EPT] = {};
    if (!diag) load_top<NB, IB>(tv, top, NB, WS);
    stage_store_rows<NB, IB>(sm, S, r0, diag, c0);
    if constexpr (PREC == PREC_FP64) apply_panel<NB, IB>(sm, X, r0, top, NB, CB, tv);
    else apply_panel_mx<NB, IB, PREC>(sm, X, r0, top, NB, tv);
    store_strip<NB, IB>(X, tik, NB, col0, CB, r0);
}

// Workers come in two roles: ROLE_PANEL runs GEQRT and TSQRT (queue
// levels 0-1), ROLE_UPDATE runs LARFB, SSRFB and PUPD (levels 2..NLEVEL-1).  The
// persistent kernel gives the panel role to its lowest workgroup indices,
// which the dispatcher makes resident first.
enum { ROLE_PANEL = 0, ROLE_UPDATE = 1 };

// With SPLIT a panel task is one inner panel of its tile kernel (the grid
// has nb / ib panel tasks per tile), else the whole tile kernel.
template <int NB, int IB, int ROLE, int PREC, bool SPLIT>
__device__ __forceinline__ void run_task(Smem<NB, IB> &sm, const MatDev &M, const Task &t)
{
    // One panel per strip: the panel tasks leave their trailing updates to
    // PUPD tasks (the grid has them exactly then).
    constexpr int NSX = strips_of<NB, PREC>();
    constexpr bool PU = SPLIT && Cfg<NB, IB>::NPAN == NSX && Cfg<NB, IB>::NPAN > 1;
    if constexpr (ROLE == ROLE_PANEL) {
        if constexpr (SPLIT) {
            if (t.type == GEQRT) geqrt_panel<NB, IB, PREC>(sm, M, t.k, t.l, false, false, !PU);
            else tsqrt_panel<NB, IB, PREC>(sm, M, t.k, t.i, t.l, false, false, !PU);
        } else {
            if (t.type == GEQRT) task_geqrt<NB, IB, PREC>(sm, M, t.k);
            else task_tsqrt<NB, IB, PREC>(sm, M, t.k, t.i);
        }
    } else {
        if (t.type == LARFB) task_larfb<NB, IB, PREC>(sm, M, t.k, t.j, t.s);
        else if (PU && t.type == PUPD) task_pupd<NB, IB, PREC>(sm, M, t.k, t.i, t.l, t.s);
        else task_ssrfb<NB, IB, PREC>(sm, M, t.k, t.i, t.j, t.s);
    }
}

// ------------------------------------------------ serial (Algorithm 2) kernels

// One launch per group of independent tasks in Algorithm 2's loop order:
// GEQRT(k) / TSQRT(k, i): one workgroup; LARFB(k, .) / SSRFB(k, i, .):
// one workgroup per (j, strip).
template <int NB, int IB, int TYPE, int PREC>
__global__ __launch_bounds__(2 * NB) void k_serial(MatDev M, int k, int i, const int *status)
{
    __shared__ Smem<NB, IB> sm;
    if (*status != 0) return;
    constexpr int NS = strips_of<NB, PREC>();
    const int j = k + 1 + blockIdx.x / NS, s = blockIdx.x % NS;
    if constexpr (TYPE == GEQRT) task_geqrt<NB, IB, PREC>(sm, M, k);
    else if constexpr (TYPE == TSQRT) task_tsqrt<NB, IB, PREC>(sm, M, k, i);
    else if constexpr (TYPE == LARFB) task_larfb<NB, IB, PREC>(sm, M, k, j, s);
    else task_ssrfb<NB, IB, PREC>(sm, M, k, i, j, s);
}

// ------------------------------------------------------- DAG scheduler
//
// Memory ordering.  A task's results are published by one agent-scope
// release fence (after a workgroup barrier that orders every wave's stores
// before it) ahead of its successor releases, and every task starts with an
// agent-scope acquire fence.  The counter decrement that finds a successor
// ready acquires (so that whatever it publishes next carries every
// predecessor's results) but needs no release of its own after the fence;
// a queue slot is written with release and read relaxed (the popper's
// acquire fence completes the pair); the queue heads and the completion
// count order no data.  Each release or acquire on an atomic costs a cache
// write-back or invalidation, hence only these.

__device__ __forceinline__ int32_t ld_rlx_i(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_rlx(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void push_task(const SchedDev &S, int queue, int64_t gid)
{
    const uint32_t slot = __hip_atomic_fetch_add(&S.qtail[queue * QSTRIDE], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&S.qslot[S.qoff[queue] + slot], (int32_t)(gid + 1), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Non-blocking pop: -1 when the queue has nothing claimable right now.
__device__ __forceinline__ int64_t pop_task(const SchedDev &S, int queue)
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        const uint32_t t = ld_rlx(&S.qtail[queue * QSTRIDE]);
        const uint32_t h = ld_rlx(&S.qhead[queue * QSTRIDE]);
        if (h >= t) return -1;
        const int32_t v = ld_rlx_i(&S.qslot[S.qoff[queue] + h]);
        if (v == 0) return -1;   // pushed, but its slot not written yet
        uint32_t expect = h;
        if (__hip_atomic_compare_exchange_strong(&S.qhead[queue * QSTRIDE], &expect, h + 1, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return (int64_t)v - 1;
    }
    return -1;
}

// XCD this workgroup runs on (hardware register XCC_ID).
__device__ __forceinline__ int xcd_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (NXQ - 1); }

__device__ __forceinline__ int find_mat(const SchedDev &S, int64_t gid)
{
    int lo = 0, hi = S.nmat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (S.mats[mid].task_base <= gid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdULL;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ULL;
    x ^= x >> 33;
    return x;
}


// One pass over the queues a worker serves: the panel worker its two
// levels; an update worker the update levels in priority order, its own
// XCD's queue first and, when `steal`, the other XCDs' queues after it.
template <int ROLE>
__device__ __forceinline__ int64_t pop_any(const SchedDev &S, int xcd, bool steal, uint64_t shuffle_rng)
{
    if constexpr (ROLE == ROLE_PANEL) {
        const int first = (int)(shuffle_rng & 1);
        int64_t gid = pop_task(S, queue_index(first, 0));
        if (gid < 0) gid = pop_task(S, queue_index(first ^ 1, 0));
        return gid;
    } else {
        constexpr int NLV = NLEVEL - 2;
        const int start = (int)(shuffle_rng % NLV);
        for (int q = 0; q < NLV; ++q) {
            const int64_t gid = pop_task(S, queue_index(2 + (start + q) % NLV, xcd));
            if (gid >= 0) return gid;
        }
        if (steal) {
            for (int q = 0; q < NLV; ++q)
                for (int d = 1; d < NXQ; ++d) {
                    const int64_t gid = pop_task(S, queue_index(2 + (start + q) % NLV, (xcd + d) % NXQ));
                    if (gid >= 0) return gid;
                }
        }
        return -1;
    }
}

template <int NB, int IB, int ROLE, int PREC, bool SPLIT>
__device__ __forceinline__ void worker_loop(Smem<NB, IB> &sm, const SchedDev &S)
{
    __shared__ int64_t s_gid, s_next;
    __shared__ int s_next_queue;
    __shared__ int s_exit;
    __shared__ uint64_t s_tpop, s_trun;
    const int tid = tidx();
    uint64_t rng = mix64(S.seed ^ (0x9e3779b97f4a7c15ULL * (blockIdx.x + 1)));
    const int xcd = xcd_id();
    // Idle polling goes to a few memory lines that every worker shares, so
    // it is kept sparse: update workers back off to about 7 us between
    // polls and look at other XCDs' queues every eighth round; the few
    // panel workers of a single matrix poll every few hundred cycles.
    const int cap = ROLE == ROLE_PANEL ? (S.npanel <= 8 ? 2 : 5) : 7;
    if (tid == 0) s_next = -1;
    for (;;) {
        if (tid == 0) {
            int64_t gid = s_next;
            int ex = 0;
            s_next = -1;
            // A kept update below the lookahead level yields to a lookahead
            // update waiting in this XCD's queue (the kept one is queued).
            if constexpr (ROLE == ROLE_UPDATE) {
                if (gid >= 0 && s_next_queue >= queue_index(3, 0)) {
                    const int64_t la = pop_task(S, queue_index(2, xcd));
                    if (la >= 0) {
                        push_task(S, s_next_queue, gid);
                        gid = la;
                    }
                }
            }
            if (gid < 0) {
                // Poll the queues with exponential back-off, look at the
                // completion counter and the status word only every few
                // rounds; every idle round counts towards the watchdog.
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
                    gid = pop_any<ROLE>(S, xcd, ROLE == ROLE_UPDATE && (round & 7) == 7, pick);
                    if (gid >= 0) break;
                    if ((round & 3) == 0) {
                        if (__hip_atomic_load(S.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                            ex = 1;
                            break;
                        }
                        const uint32_t d = ld_rlx(S.done);
                        if (d >= S.total_tasks) {
                            ex = 1;
                            break;
                        }
                        if (d != seen) {
                            seen = d;
                            idle = 0;
                        }
                    }
                    if (++idle > S.spin_limit) {
                        __hip_atomic_fetch_or(S.status, STATUS_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ex = 1;
                        break;
                    }
                    backoff = backoff < cap ? backoff + 1 : cap;
                    for (int z = 0; z < (1 << backoff); ++z) __builtin_amdgcn_s_sleep(2);
                }
            }
            s_gid = gid;
            s_exit = ex;
            s_tpop = wall_clock64();
        }
        __syncthreads();
        if (s_exit) break;
        const int64_t gid = s_gid;
        // Acquire: one wave invalidates the (shared) L1 and L2 lines, the
        // barrier holds the others back until it has.
        if (tid < 64) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        const int mi = find_mat(S, gid);
        const MatDev &M = S.mats[mi];
        // Strips and panels per tile are compile-time constants here (the
        // host sets S.ns = nb / 32 and S.np to match the kernel), which
        // keeps the id arithmetic to shifts.
        const Grid g = make_grid(M.p, M.q, strips_of<NB, PREC>(), SPLIT ? Cfg<NB, IB>::NPAN : 1);
        const Task t = decode(g, gid - M.task_base);
        const uint64_t t0 = wall_clock64();
        run_task<NB, IB, ROLE, PREC, SPLIT>(sm, M, t);
        // Release: every wave waits for its own stores, then wave 0 writes
        // the L2 back and releases the successors (in program order after
        // its fence).  Of the successors this task makes ready, the first
        // one of this worker's role is kept and run next without a trip
        // through the queues (a TSQRT chain, or a strip's chain of updates,
        // stays on one workgroup); the others are queued.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (tid == 0) s_trun = wall_clock64();
        if (tid < 64) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const int ns = nsucc(g, t);
            bool kept = false;
            for (int base = 0; base < ns; base += 64) {
                const int n = base + tid;
                bool ready = false, mine = false;
                int64_t sgid = -1;
                int queue = 0;
                if (n < ns && !(S.drop_edge >= 0 && gid == S.drop_edge && n == 0)) {
                    const int64_t sl = succ(g, t, n);
                    const int32_t old = __hip_atomic_fetch_add(&S.counters[M.task_base + sl], -1, __ATOMIC_ACQUIRE,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                    if (old == 1) {
                        const Task nt = decode(g, sl);
                        ready = true;
                        mine = (nt.type == GEQRT || nt.type == TSQRT) == (ROLE == ROLE_PANEL);
                        sgid = M.task_base + sl;
                        queue = queue_of(nt, S.ns, mi);
                    }
                }
                const uint64_t cand = __ballot(ready && mine);
                const int keeper = (!kept && cand != 0) ? __ffsll((unsigned long long)cand) - 1 : -1;
                if (ready) {
                    if (tid == keeper) {
                        s_next = sgid;
                        s_next_queue = queue;
                    }
                    else push_task(S, queue, sgid);
                }
                kept = kept || keeper >= 0;
            }
        }
        if (tid == 0) {
            if (S.trace != nullptr) {
                const uint32_t e = __hip_atomic_fetch_add(S.trace_count, 1u, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                if (e < S.trace_cap) {
                    int64_t *ev = S.trace + (size_t)e * TRACE_WORDS;
                    ev[0] = t.type; ev[1] = t.k; ev[2] = t.i; ev[3] = t.type == PUPD ? t.l : t.j;
                    ev[4] = t.type <= TSQRT ? t.l : t.s;
                    ev[5] = ((int64_t)mi << 20) | (ROLE << 16) | blockIdx.x;
                    ev[6] = (int64_t)s_tpop;
                    ev[7] = (int64_t)t0;
                    ev[8] = (int64_t)s_trun;
                    ev[9] = (int64_t)wall_clock64();
                }
            }
            __hip_atomic_fetch_add(S.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// The persistent workers; SPLIT: the grid has one panel task per inner
// panel (S.np == nb / ib), else one per tile kernel (S.np == 1).  Separate
// kernels, so that each keeps its panel code with compile-time loop bounds.
template <int NB, int IB, int PREC, bool SPLIT>
__global__ __launch_bounds__(2 * NB) void k_worker(SchedDev S)
{
    __shared__ Smem<NB, IB> sm;
    if ((int)blockIdx.x < S.npanel) worker_loop<NB, IB, ROLE_PANEL, PREC, SPLIT>(sm, S);
    else worker_loop<NB, IB, ROLE_UPDATE, PREC, SPLIT>(sm, S);
}

// Host side of the kernels above for one arithmetic (PREC): the serial
// Algorithm 2 driver, the persistent scheduler launch and its occupancy.
template <int NB, int IB, int PREC>
static hipError_t serial_impl(const MatDev &M, const int *status, hipStream_t st)
{
    constexpr int NS = strips_of<NB, PREC>();
    static_assert(NS == strips_per_tile(NB, PREC), "host and device agree on the strips per tile");
    const int p = M.p, q = M.q, kmax = p < q ? p : q;
    const dim3 blk(Cfg<NB, IB>::NT);
    for (int k = 0; k < kmax; ++k) {
        hipLaunchKernelGGL((k_serial<NB, IB, GEQRT, PREC>), dim3(1), blk, 0, st, M, k, k, status);
        if (q - k - 1 > 0)
            hipLaunchKernelGGL((k_serial<NB, IB, LARFB, PREC>), dim3((q - k - 1) * NS), blk, 0, st, M, k, k,
                               status);
        for (int i = k + 1; i < p; ++i) {
            hipLaunchKernelGGL((k_serial<NB, IB, TSQRT, PREC>), dim3(1), blk, 0, st, M, k, i, status);
            if (q - k - 1 > 0)
                hipLaunchKernelGGL((k_serial<NB, IB, SSRFB, PREC>), dim3((q - k - 1) * NS), blk, 0, st, M, k, i,
                                   status);
        }
    }
    return hipGetLastError();
}

template <int NB, int IB, int PREC>
static hipError_t worker_impl(const SchedDev &S, int workers, hipStream_t st)
{
    if (S.np == Cfg<NB, IB>::NPAN && S.np > 1)
        hipLaunchKernelGGL((k_worker<NB, IB, PREC, true>), dim3(workers), dim3(Cfg<NB, IB>::NT), 0, st, S);
    else if (S.np == 1)
        hipLaunchKernelGGL((k_worker<NB, IB, PREC, false>), dim3(workers), dim3(Cfg<NB, IB>::NT), 0, st, S);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Workgroups per CU of both worker kernels (the smaller, should they differ).
template <int NB, int IB, int PREC>
static int worker_occupancy_impl()
{
    int a = 0, b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_worker<NB, IB, PREC, false>, Cfg<NB, IB>::NT, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_worker<NB, IB, PREC, true>, Cfg<NB, IB>::NT, 0) !=
            hipSuccess)
        return 1;
    a = a < b ? a : b;
    return a > 0 ? a : 1;
}

}  // namespace tq
