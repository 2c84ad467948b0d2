// Tile kernels of the tiled QR (Section 3.2.1, Algorithm 2) for gfx950, and
// the persistent DAG scheduler that runs them (Section 4).
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
    static constexpr int NSLOT = NW < 4 ? NW : 4;   // LDS slots of the cross-wave reduction
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
struct Smem {
    using C = Cfg<NB, IB>;
    double P[(NB + IB) * C::LDP];    // panel / V: rows 0..nb-1 tile rows, nb.. head rows
    double Wp[C::NSLOT * IB * WS];   // per-wave partial products
    double Wa[IB * WS];              // reduced W (or the Gram matrix V^T V)
    double Wb[IB * WS];              // T^T W
    double Tl[IB * IB];              // T of the current inner panel
    double tau[IB];
    double xb[2][NB];                // reflector broadcast (double-buffered by column parity)
    double sc[2][2];                 // tau of the broadcast reflector
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ gdouble *tile_ptr(const MatDev &M, int nb, int i, int j)
{
    return (gdouble *)(M.tiles + ((size_t)j * M.p + i) * (size_t)nb * nb);
}

__device__ __forceinline__ gdouble *tblock_ptr(const MatDev &M, int nb, int ib, int k, int i)
{
    return (gdouble *)(M.T + ((size_t)k * M.p + i) * (size_t)ib * nb);
}

// Stage <- columns [c0, c0 + ib) of rows [r0, nb) of a row-major tile
// (rows above r0 left zero) and the ib x ib T block at Tg.
template <int NB, int IB>
__device__ __forceinline__ void stage_load(Stage<NB, IB> &S, const gdouble *tile, int c0, int r0,
                                           const gdouble *Tg)
{
    using C = Cfg<NB, IB>;
    constexpr int H = IB / 2;
#pragma unroll
    for (int u = 0; u < C::VPT; ++u) {
        const int e = threadIdx.x + u * C::NT, r = e / H, c2 = e % H;
        S.v[u] = r >= r0 ? *reinterpret_cast<const gv2d *>(tile + (size_t)r * NB + c0 + 2 * c2)
                         : v2d{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < C::TPT; ++u) {
        const int e = threadIdx.x + u * C::NT;
        S.t[u] = e < IB * IB / 2 ? reinterpret_cast<const gv2d *>(Tg)[e] : v2d{0.0, 0.0};
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
        const int e = threadIdx.x + u * C::NT, r = e / H, c = 2 * (e % H);
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
        const int e = threadIdx.x + u * C::NT;
        if (e < IB * IB / 2) reinterpret_cast<v2d *>(sm.Tl)[e] = S.t[u];
    }
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

template <int NB, int IB>
__device__ __forceinline__ void store_strip(const Strip<NB, IB> &X, gdouble *tile, int ld, int col0, int cbn,
                                            int rlo)
{
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = wave_id() * 32;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        if (rowbase + rb * 16 < rlo) continue;
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

// Per-wave partial accumulators (BA x BB blocks of 16 x 16 in accumulator
// layout, row stride ld) -> sm.Wp slots 0..NSLOT-1.  With 8 waves the upper
// four first store, then the lower four add theirs (slot q = P_{q+4} + P_q),
// which halves the LDS the reduction needs; the caller sums the slots in
// order.  Ends with a barrier.
template <int NB, int IB, int BA, int BB>
__device__ __forceinline__ void waves_to_slots(Smem<NB, IB> &sm, const d4 (&acc)[BA][BB], int ld)
{
    using C = Cfg<NB, IB>;
    constexpr int SLOT = IB * WS;
    const int w = wave_id(), n = lane_id() & 15, g = lane_id() >> 4;
    if (C::NW > C::NSLOT) {
        if (w >= C::NSLOT) {
#pragma unroll
            for (int a = 0; a < BA; ++a)
#pragma unroll
                for (int b = 0; b < BB; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        sm.Wp[(w - C::NSLOT) * SLOT + (a * 16 + 4 * r + g) * ld + b * 16 + n] = acc[a][b][r];
        }
        __syncthreads();
        if (w < C::NSLOT) {
#pragma unroll
            for (int a = 0; a < BA; ++a)
#pragma unroll
                for (int b = 0; b < BB; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        double *d = &sm.Wp[w * SLOT + (a * 16 + 4 * r + g) * ld + b * 16 + n];
                        *d = *d + acc[a][b][r];
                    }
        }
    } else {
#pragma unroll
        for (int a = 0; a < BA; ++a)
#pragma unroll
            for (int b = 0; b < BB; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    sm.Wp[w * SLOT + (a * 16 + 4 * r + g) * ld + b * 16 + n] = acc[a][b][r];
    }
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

// Apply the block reflector of one inner panel, held in LDS (sm.P rows
// 0..nb-1 = V, rows below `rlo` ignored; sm.Tl = T), to a strip X:
//   W = [top +] V^T X;  W <- T^T W;  [top -= W;]  X -= V W
// (with TRANS == false, W <- T W: the reflector itself instead of its
// transpose).
// `top` (may be NULL) points at the ib x (16 cbn) block of the coupled upper
// tile (the R rows the TS form also updates), row stride ldtop.
// Three workgroup barriers; the products V^T X, T^T W and V W run on MFMA.
template <int NB, int IB, bool TRANS = true>
__device__ void apply_panel(Smem<NB, IB> &sm, Strip<NB, IB> &X, int rlo, gdouble *top, int ldtop, int cbn)
{
    using C = Cfg<NB, IB>;
    const int tid = threadIdx.x, w = wave_id();
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = w * 32;
    const int ncol = cbn * 16;

    double tv[C::EPT];
    if (top != nullptr) {
#pragma unroll
        for (int u = 0; u < C::EPT; ++u) {
            const int e = tid + u * C::NT, kr = e / WS, c = e % WS;
            tv[u] = c < ncol ? top[(size_t)kr * ldtop + c] : 0.0;
        }
    }

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
                for (int cb = 0; cb < CB; ++cb) Wacc[a][cb] = mfma(va, X.v[rb][cb][r], Wacc[a][cb]);
            }
        }
    }
    waves_to_slots<NB, IB, C::IBB, CB>(sm, Wacc, WS);
#pragma unroll
    for (int u = 0; u < C::EPT; ++u) {
        const int e = tid + u * C::NT, c = e % WS;
        double s = sum_slots<NB, IB>(sm, e);
        if (top != nullptr && c < ncol) s = tv[u] + s;
        sm.Wa[e] = s;
    }
    __syncthreads();
    // T^T W: one 16 x 16 output block per wave.
    for (int blk = w; blk < C::IBB * CB; blk += C::NW) {
        const int a = blk / CB, cb = blk % CB;
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < IB / 4; ++kc)
            acc = mfma(TRANS ? sm.Tl[(4 * kc + g) * IB + a * 16 + n] : sm.Tl[(a * 16 + n) * IB + 4 * kc + g],
                       sm.Wa[(4 * kc + g) * WS + cb * 16 + n], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = a * 16 + 4 * r + g, c = cb * 16 + n;
            sm.Wb[i * WS + c] = acc[r];
            if (top != nullptr && c < ncol) top[(size_t)i * ldtop + c] -= acc[r];
        }
    }
    __syncthreads();
    // X -= V (T^T W)
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb) {
        if (rowbase + rb * 16 < rlo) continue;
#pragma unroll
        for (int kc = 0; kc < IB / 4; ++kc) {
            const double va = sm.P[(rowbase + rb * 16 + n) * C::LDP + 4 * kc + g];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const double wb = -sm.Wb[(4 * kc + g) * WS + cb * 16 + n];
                X.v[rb][cb] = mfma(va, wb, X.v[rb][cb]);
            }
        }
    }
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
// later column applies it.
template <int NB, int IB>
__device__ void panel_factor(Smem<NB, IB> &sm, int c0, bool ts)
{
    using C = Cfg<NB, IB>;
    constexpr int RG = C::RG, RPT = C::RPT, LDP = C::LDP;
    static_assert(64 % RG == 0, "the threads of a column share one wave");
    const int tid = threadIdx.x, c = tid / RG, rg = tid % RG;
    double pr[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) pr[i] = sm.P[(rg + i * RG) * LDP + c];
#pragma unroll 1
    for (int j = 0; j < IB; ++j) {
        const int hrow = ts ? NB + j : c0 + j;
        const int tlo = ts ? 0 : c0 + j + 1;
        double *xb = sm.xb[j & 1];
        double *sc = sm.sc[j & 1];
        if (c == j) {
            double alpha;
            if (ts) {
                alpha = sm.P[hrow * LDP + j];
            } else {
                double h = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; ++i)
                    if (rg + i * RG == hrow) h = pr[i];
                alpha = group_sum<RG>(h);   // only the owner contributes
            }
            double part = 0.0;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const double x = rg + i * RG >= tlo ? pr[i] : 0.0;
                part += x * x;
            }
            const double sig = group_sum<RG>(part);
            double xnorm, h;
            if (sig <= 1.0e300 && (sig >= 2.2250738585072014e-308 || sig == 0.0)) {
                // Nothing over- or underflowed (a zero sum with nonzero
                // entries is caught by the scaled pass below).
                xnorm = sqrt(sig);
                h = fabs(alpha) < 1.0e150 ? sqrt(alpha * alpha + sig) : hypot(alpha, xnorm);
            } else {
                xnorm = -1.0;
                h = 0.0;
            }
            if (xnorm < 0.0 || (sig == 0.0 && group_max<RG>(part) != 0.0)) {
                // Redo the norm scaled by the largest magnitude.
                double mx = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; ++i)
                    if (rg + i * RG >= tlo) mx = fmax(mx, fabs(pr[i]));
                const double mxa = group_max<RG>(mx);
                double p2 = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const double t = rg + i * RG >= tlo ? pr[i] / mxa : 0.0;
                    p2 += t * t;
                }
                xnorm = mxa * sqrt(group_sum<RG>(p2));
                h = hypot(alpha, xnorm);
            }
            double tau = 0.0;
            if (xnorm != 0.0) {
                const double beta = alpha >= 0.0 ? -h : h;
                tau = (beta - alpha) / beta;
                const double scal = 1.0 / (alpha - beta);
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int r = rg + i * RG;
                    if (r >= tlo) {
                        pr[i] = pr[i] * scal;
                        xb[r] = pr[i];
                    }
                    if (!ts && r == hrow) pr[i] = beta;
                }
                if (ts && rg == 0) sm.P[hrow * LDP + j] = beta;
            }
            if (rg == 0) {
                sc[0] = tau;
                sm.tau[j] = tau;
            }
        }
        __syncthreads();
        const double tau = sc[0];
        if (c > j && tau != 0.0) {
            double part = 0.0;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int r = rg + i * RG;
                if (r >= tlo) part += xb[r] * pr[i];
            }
            const double dot = group_sum<RG>(part);
            double hc;
            if (ts) {
                hc = sm.P[hrow * LDP + c];
            } else {
                double h = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; ++i)
                    if (rg + i * RG == hrow) h = pr[i];
                hc = group_sum<RG>(h);   // only the owner contributes
            }
            const double tw = tau * (hc + dot);
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int r = rg + i * RG;
                if (r >= tlo) pr[i] -= xb[r] * tw;
                if (!ts && r == hrow) pr[i] = hc - tw;
            }
            if (ts && rg == 0) sm.P[hrow * LDP + c] = hc - tw;
        }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int r = rg + i * RG;
        if (ts || r >= c0) sm.P[r * LDP + c] = pr[i];
    }
    __syncthreads();
}

// T of the panel in sm.P (rows >= rlo; V with its unit diagonal explicit):
// G = V^T V on MFMA, then column by column (compact WY, forward)
//   T[j][j] = tau_j,  T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j].
// Lane i builds row i of T in registers: its entries only depend on the
// row's earlier entries, and with the loops unrolled each new entry waits
// for one multiply-add after the previous one.  Leaves T in sm.Tl and writes
// it to Tg (row-major ib x ib).
template <int NB, int IB>
__device__ void build_t(Smem<NB, IB> &sm, int rlo, gdouble *Tg)
{
    using C = Cfg<NB, IB>;
    const int tid = threadIdx.x, w = wave_id();
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
    for (int e = tid; e < IB * IB; e += C::NT) sm.Wa[e] = sum_slots<NB, IB>(sm, e);
    __syncthreads();
    if (tid < IB) {
        const int i = tid;
        double trow[IB];
#pragma unroll
        for (int kk = 0; kk < IB; ++kk) trow[kk] = kk == i ? sm.tau[kk] : 0.0;
#pragma unroll
        for (int j = 1; j < IB; ++j) {
            double s = 0.0;
#pragma unroll
            for (int kk = 0; kk < j; ++kk) s += trow[kk] * sm.Wa[kk * IB + j];
            if (i < j) trow[j] = -sm.tau[j] * s;
        }
#pragma unroll
        for (int kk = 0; kk < IB; ++kk) sm.Tl[i * IB + kk] = trow[kk];
    }
    __syncthreads();
    for (int e = tid; e < IB * IB; e += C::NT) Tg[e] = sm.Tl[e];
}

// ------------------------------------------------------------ tile kernels

// DGEQRT(A_kk) -> (V_kk, R_kk, T_kk).
template <int NB, int IB>
__device__ void task_geqrt(Smem<NB, IB> &sm, const MatDev &M, int k)
{
    using C = Cfg<NB, IB>;
    gdouble *tkk = tile_ptr(M, NB, k, k);
    gdouble *Tk = tblock_ptr(M, NB, IB, k, k);
    Stage<NB, IB> S;
#pragma unroll 1
    for (int l = 0; l < C::NPAN; ++l) {
        const int c0 = l * IB;
        stage_load<NB, IB>(S, tkk, c0, c0, Tk);
        stage_store<NB, IB>(sm, S, c0, false, c0);
        __syncthreads();
        panel_factor<NB, IB>(sm, c0, false);
        // Write R and V back; keep V with explicit unit diagonal in LDS.
        constexpr int H = IB / 2;
#pragma unroll
        for (int u = 0; u < C::VPT; ++u) {
            const int e = threadIdx.x + u * C::NT, r = e / H, cc = 2 * (e % H);
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
#pragma unroll 1
        for (int col0 = c0 + IB; col0 < NB; col0 += WS) {
            const int cbn = min(CB, (NB - col0) / 16);
            Strip<NB, IB> X;
            load_strip<NB, IB>(X, tkk, NB, col0, cbn);
            apply_panel<NB, IB>(sm, X, c0, nullptr, 0, cbn);
            store_strip<NB, IB>(X, tkk, NB, col0, cbn, c0);
        }
        __syncthreads();
    }
}

// DTSQRT(R_kk, A_ik) -> (R_kk, V_ik, T_ik).
template <int NB, int IB>
__device__ void task_tsqrt(Smem<NB, IB> &sm, const MatDev &M, int k, int i)
{
    using C = Cfg<NB, IB>;
    gdouble *tkk = tile_ptr(M, NB, k, k);
    gdouble *tik = tile_ptr(M, NB, i, k);
    gdouble *Ti = tblock_ptr(M, NB, IB, k, i);
    Stage<NB, IB> S;
    constexpr int H = IB / 2;
#pragma unroll 1
    for (int l = 0; l < C::NPAN; ++l) {
        const int c0 = l * IB;
        stage_load<NB, IB>(S, tik, c0, 0, Ti);
        for (int e = threadIdx.x; e < IB * IB; e += C::NT) {
            const int r = e / IB, c = e % IB;
            sm.P[(NB + r) * C::LDP + c] = r <= c ? tkk[(size_t)(c0 + r) * NB + c0 + c] : 0.0;
        }
        stage_store<NB, IB>(sm, S, 0, false, c0);
        __syncthreads();
        panel_factor<NB, IB>(sm, c0, true);
        for (int e = threadIdx.x; e < IB * IB; e += C::NT) {
            const int r = e / IB, c = e % IB;
            if (r <= c) tkk[(size_t)(c0 + r) * NB + c0 + c] = sm.P[(NB + r) * C::LDP + c];
        }
#pragma unroll
        for (int u = 0; u < C::VPT; ++u) {
            const int e = threadIdx.x + u * C::NT, r = e / H, cc = 2 * (e % H);
            *reinterpret_cast<gv2d *>(tik + (size_t)r * NB + c0 + cc) =
                *reinterpret_cast<v2d *>(&sm.P[r * C::LDP + cc]);
        }
        build_t<NB, IB>(sm, 0, Ti + l * IB * IB);
        __syncthreads();
#pragma unroll 1
        for (int col0 = c0 + IB; col0 < NB; col0 += WS) {
            const int cbn = min(CB, (NB - col0) / 16);
            Strip<NB, IB> X;
            load_strip<NB, IB>(X, tik, NB, col0, cbn);
            apply_panel<NB, IB>(sm, X, 0, tkk + (size_t)c0 * NB + col0, NB, cbn);
            store_strip<NB, IB>(X, tik, NB, col0, cbn, 0);
        }
        __syncthreads();
    }
}

// One strip (32 columns at col0, row stride ldx) of X <- Q_kk^T X (TRANS)
// or Q_kk X, Q_kk the block reflector of the diagonal tile tkk with T
// blocks Tk.  Q_kk = H_0 ... H_{t-1} over the inner panels, so Q_kk^T runs
// the panels forward with T^T and Q_kk backward with T.
template <int NB, int IB, bool TRANS>
__device__ void apply_diag_strip(Smem<NB, IB> &sm, const gdouble *tkk, const gdouble *Tk, gdouble *x, int ldx,
                                 int col0)
{
    using C = Cfg<NB, IB>;
    Stage<NB, IB> S;
    const int l0 = TRANS ? 0 : C::NPAN - 1;
    stage_load<NB, IB>(S, tkk, l0 * IB, l0 * IB, Tk + l0 * IB * IB);
    Strip<NB, IB> X;
    load_strip<NB, IB>(X, x, ldx, col0, CB);
#pragma unroll 1
    for (int q = 0; q < C::NPAN; ++q) {
        const int l = TRANS ? q : C::NPAN - 1 - q;
        const int c0 = l * IB;
        stage_store<NB, IB>(sm, S, c0, true, c0);
        __syncthreads();
        if (q + 1 < C::NPAN) {
            const int ln = TRANS ? l + 1 : l - 1;
            stage_load<NB, IB>(S, tkk, ln * IB, ln * IB, Tk + ln * IB * IB);
        }
        apply_panel<NB, IB, TRANS>(sm, X, c0, nullptr, 0, CB);
        __syncthreads();
    }
    store_strip<NB, IB>(X, x, ldx, col0, CB, 0);
}

// One strip of [top; X] <- Q_ik^T [top; X] (TRANS) or Q_ik [top; X], Q_ik
// the coupled block reflector of tile tik (reflectors [e; V2]) with T blocks
// Ti; `top` is the whole upper tile (its rows c0.. are the ones each inner
// panel touches).
template <int NB, int IB, bool TRANS>
__device__ void apply_ts_strip(Smem<NB, IB> &sm, const gdouble *tik, const gdouble *Ti, gdouble *top, int ldtop,
                               gdouble *x, int ldx, int col0)
{
    using C = Cfg<NB, IB>;
    Stage<NB, IB> S;
    const int l0 = TRANS ? 0 : C::NPAN - 1;
    stage_load<NB, IB>(S, tik, l0 * IB, 0, Ti + l0 * IB * IB);
    Strip<NB, IB> X;
    load_strip<NB, IB>(X, x, ldx, col0, CB);
#pragma unroll 1
    for (int q = 0; q < C::NPAN; ++q) {
        const int l = TRANS ? q : C::NPAN - 1 - q;
        const int c0 = l * IB;
        stage_store<NB, IB>(sm, S, 0, false, c0);
        __syncthreads();
        if (q + 1 < C::NPAN) {
            const int ln = TRANS ? l + 1 : l - 1;
            stage_load<NB, IB>(S, tik, ln * IB, 0, Ti + ln * IB * IB);
        }
        apply_panel<NB, IB, TRANS>(sm, X, 0, top + (size_t)c0 * ldtop + col0, ldtop, CB);
        __syncthreads();
    }
    store_strip<NB, IB>(X, x, ldx, col0, CB, 0);
}

// DLARFB: strip s of A_kj <- Q_kk^T A_kj.
template <int NB, int IB>
__device__ void task_larfb(Smem<NB, IB> &sm, const MatDev &M, int k, int j, int s)
{
    apply_diag_strip<NB, IB, true>(sm, tile_ptr(M, NB, k, k), tblock_ptr(M, NB, IB, k, k), tile_ptr(M, NB, k, j), NB,
                                   s * WS);
}

// DSSRFB: strip s of [A_kj; A_ij] <- Q_ik^T [A_kj; A_ij].
template <int NB, int IB>
__device__ void task_ssrfb(Smem<NB, IB> &sm, const MatDev &M, int k, int i, int j, int s)
{
    apply_ts_strip<NB, IB, true>(sm, tile_ptr(M, NB, i, k), tblock_ptr(M, NB, IB, k, i), tile_ptr(M, NB, k, j), NB,
                                 tile_ptr(M, NB, i, j), NB, s * WS);
}

// Workers come in two roles: ROLE_PANEL runs GEQRT and TSQRT (queue
// levels 0-1), ROLE_UPDATE runs LARFB and SSRFB (levels 2..NLEVEL-1).  The
// persistent kernel gives the panel role to its lowest workgroup indices,
// which the dispatcher makes resident first.
enum { ROLE_PANEL = 0, ROLE_UPDATE = 1 };

template <int NB, int IB, int ROLE>
__device__ __forceinline__ void run_task(Smem<NB, IB> &sm, const MatDev &M, const Task &t)
{
    if constexpr (ROLE == ROLE_PANEL) {
        if (t.type == GEQRT) task_geqrt<NB, IB>(sm, M, t.k);
        else task_tsqrt<NB, IB>(sm, M, t.k, t.i);
    } else {
        if (t.type == LARFB) task_larfb<NB, IB>(sm, M, t.k, t.j, t.s);
        else task_ssrfb<NB, IB>(sm, M, t.k, t.i, t.j, t.s);
    }
}

// ------------------------------------------------ serial (Algorithm 2) kernels

// One launch per group of independent tasks in Algorithm 2's loop order:
// GEQRT(k) / TSQRT(k, i): one workgroup; LARFB(k, .) / SSRFB(k, i, .):
// one workgroup per (j, strip).
template <int NB, int IB, int TYPE>
__global__ __launch_bounds__(2 * NB) void k_serial(MatDev M, int k, int i, const int *status)
{
    __shared__ Smem<NB, IB> sm;
    if (*status != 0) return;
    constexpr int NS = Cfg<NB, IB>::NS;
    const int j = k + 1 + blockIdx.x / NS, s = blockIdx.x % NS;
    if constexpr (TYPE == GEQRT) task_geqrt<NB, IB>(sm, M, k);
    else if constexpr (TYPE == TSQRT) task_tsqrt<NB, IB>(sm, M, k, i);
    else if constexpr (TYPE == LARFB) task_larfb<NB, IB>(sm, M, k, j, s);
    else task_ssrfb<NB, IB>(sm, M, k, i, j, s);
}

// ------------------------------------------------------- DAG scheduler

__device__ __forceinline__ int32_t ld_acq(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_rlx(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void push_task(const SchedDev &S, int queue, int64_t gid)
{
    const uint32_t slot = __hip_atomic_fetch_add(&S.qtail[queue * 32], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&S.qslot[S.qoff[queue] + slot], (int32_t)(gid + 1), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Non-blocking pop: -1 when the queue has nothing claimable right now.
__device__ __forceinline__ int64_t pop_task(const SchedDev &S, int queue)
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        const uint32_t t = ld_rlx(&S.qtail[queue * 32]);
        const uint32_t h = ld_rlx(&S.qhead[queue * 32]);
        if (h >= t) return -1;
        const int32_t v = ld_acq(&S.qslot[S.qoff[queue] + h]);
        if (v == 0) return -1;
        uint32_t expect = h;
        if (__hip_atomic_compare_exchange_strong(&S.qhead[queue * 32], &expect, h + 1, __ATOMIC_ACQ_REL,
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

// Counters <- in-degrees, queues cleared, GEQRT(0) of every matrix queued.
__global__ void k_sched_init(SchedDev S)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t gid = tid0; gid < S.total_ids; gid += stride) {
        const int mi = find_mat(S, gid);
        const MatDev &M = S.mats[mi];
        const Grid g = make_grid(M.p, M.q, S.ns);
        const Task t = decode(g, gid - M.task_base);
        S.counters[gid] = valid(g, t) ? indegree(g, t) : -1;
    }
    for (int64_t e = tid0; e < S.qslot_total; e += stride) S.qslot[e] = 0;
    for (int64_t e = tid0; e < NQUEUE * 32; e += stride) {
        S.qhead[e] = 0;
        S.qtail[e] = 0;
    }
    if (tid0 == 0) {
        *S.done = 0;
        *S.trace_count = 0;
    }
}

__global__ void k_sched_seed(SchedDev S)
{
    // Runs after k_sched_init (stream order): queue every GEQRT(0).
    // Every matrix in the list is non-empty (the host drops empty ones).
    for (int mi = threadIdx.x; mi < S.nmat; mi += blockDim.x)
        S.qslot[S.qoff[queue_index(0, 0)] + mi] = (int32_t)(S.mats[mi].task_base + 1);
    __syncthreads();
    if (threadIdx.x == 0) S.qtail[queue_index(0, 0) * 32] = (uint32_t)S.nmat;
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

template <int NB, int IB, int ROLE>
__device__ __forceinline__ void worker_loop(Smem<NB, IB> &sm, const SchedDev &S)
{
    __shared__ int64_t s_gid;
    __shared__ int s_exit;
    const int tid = threadIdx.x;
    uint64_t rng = mix64(S.seed ^ (0x9e3779b97f4a7c15ULL * (blockIdx.x + 1)));
    const int xcd = xcd_id();
    for (;;) {
        if (tid == 0) {
            // Idle loop: poll the queues with exponential back-off, look at
            // the completion counter and the status word only every few
            // rounds; every idle round counts towards the watchdog.
            int64_t gid = -1;
            int ex = 0;
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
                gid = pop_any<ROLE>(S, xcd, ROLE == ROLE_UPDATE && (round & 3) == 3, pick);
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
                const int cap = ROLE == ROLE_PANEL ? 2 : 5;
                backoff = backoff < cap ? backoff + 1 : cap;
                for (int z = 0; z < (1 << backoff); ++z) __builtin_amdgcn_s_sleep(2);
            }
            s_gid = gid;
            s_exit = ex;
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
        const Grid g = make_grid(M.p, M.q, S.ns);
        const Task t = decode(g, gid - M.task_base);
        const uint64_t t0 = wall_clock64();
        run_task<NB, IB, ROLE>(sm, M, t);
        // Release: every wave waits for its own stores, then wave 0 writes
        // the L2 back and releases the successors (in program order after
        // its fence).
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (tid < 64) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const int ns = tid < 64 ? nsucc(g, t) : 0;
        for (int n = tid; n < ns; n += 64) {
            if (S.drop_edge >= 0 && gid == S.drop_edge && n == 0) continue;
            const int64_t sl = succ(g, t, n);
            const int32_t old = __hip_atomic_fetch_add(&S.counters[M.task_base + sl], -1, __ATOMIC_ACQ_REL,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            if (old == 1) push_task(S, queue_of(decode(g, sl), S.ns, mi), M.task_base + sl);
        }
        if (tid == 0) {
            if (S.trace != nullptr) {
                const uint32_t e = __hip_atomic_fetch_add(S.trace_count, 1u, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                if (e < S.trace_cap) {
                    int64_t *ev = S.trace + (size_t)e * 8;
                    ev[0] = t.type; ev[1] = t.k; ev[2] = t.i; ev[3] = t.j; ev[4] = t.s;
                    ev[5] = ((int64_t)mi << 20) | (ROLE << 16) | blockIdx.x;
                    ev[6] = (int64_t)t0;
                    ev[7] = (int64_t)wall_clock64();
                }
            }
            __hip_atomic_fetch_add(S.done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

template <int NB, int IB>
__global__ __launch_bounds__(2 * NB) void k_worker(SchedDev S)
{
    __shared__ Smem<NB, IB> sm;
    if ((int)blockIdx.x < S.npanel) worker_loop<NB, IB, ROLE_PANEL>(sm, S);
    else worker_loop<NB, IB, ROLE_UPDATE>(sm, S);
}

// -------------------------------------------------- applying Q and Q^T

// B <- Q^T B (TRANS) or Q B for Q of a finished factorisation, B held in
// row blocks of nb rows (row-major, leading dimension D.ldb, a multiple of
// the strip width).  Q^T applies, for k = 0, 1, ..: Q_kk^T to block k, then
// Q_ik^T to blocks (k, i) for i = k+1, k+2, ..  (the order in which the
// factorisation applied them to A); Q applies the transposes in reverse.
// Workgroup w runs step k (k = w for Q^T, kmax-1-w for Q) over its row
// blocks in that order; before touching block i it waits until the step
// that precedes it in the product has finished block i (progress flags in
// D.prog).  That neighbour always has the lower workgroup index, so it was
// dispatched first and the waits make progress; every wait is bounded.
template <int NB, int IB, bool TRANS>
__global__ __launch_bounds__(2 * NB) void k_apply(ApplyDev D)
{
    __shared__ Smem<NB, IB> sm;
    __shared__ int s_abort;
    const int tid = threadIdx.x;
    const int kmax = D.kmax, p = D.M.p;
    const int k = TRANS ? (int)blockIdx.x : kmax - 1 - (int)blockIdx.x;
    const gdouble *tkk = tile_ptr(D.M, NB, k, k);
    gdouble *Bk = (gdouble *)(D.B + (size_t)k * NB * D.ldb);
    const int nrow = p - k;   // blocks k .. p-1
    if (*D.status != 0) return;   // input rejected (non-finite factor)
    for (int q = 0; q < nrow; ++q) {
        // Q^T: k, k+1, .., p-1.   Q: p-1, .., k+1, then k.
        const int r = TRANS ? k + q : (q + 1 < nrow ? p - 1 - q : k);
        const bool wait = TRANS ? k > 0 : (k + 1 < kmax && r != k);
        if (tid == 0) {
            int abort = 0;
            if (wait) {
                const int *flag = &D.prog[TRANS ? k - 1 : k + 1];
                int64_t spins = 0;
                for (;;) {
                    const int v = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (TRANS ? v >= r : v <= r) break;
                    if (__hip_atomic_load(D.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        ++spins > D.spin_limit) {
                        __hip_atomic_fetch_or(D.status, STATUS_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        abort = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            s_abort = abort;
        }
        __syncthreads();
        if (s_abort) return;
        gdouble *Br = (gdouble *)(D.B + (size_t)r * NB * D.ldb);
#pragma unroll 1
        for (int st = 0; st < D.nstrip; ++st) {
            if (r == k)
                apply_diag_strip<NB, IB, TRANS>(sm, tkk, tblock_ptr(D.M, NB, IB, k, k), Bk, D.ldb, st * WS);
            else
                apply_ts_strip<NB, IB, TRANS>(sm, tile_ptr(D.M, NB, r, k), tblock_ptr(D.M, NB, IB, k, r), Bk, D.ldb,
                                              Br, D.ldb, st * WS);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(&D.prog[k], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Progress flags before an apply: Q^T steps start at k-1 (nothing done),
// Q steps at p (nothing done, rows are taken in descending order).
__global__ void k_apply_init(int *prog, int kmax, int p, int trans)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < kmax; k += gridDim.x * blockDim.x)
        prog[k] = trans ? k - 1 : p;
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

// Column-major (A, lda) -> zero-padded row-major tiles, 64 x 64 blocks via
// an LDS transpose.  Flags NaN/Inf in *status.
__global__ __launch_bounds__(256) void k_cm2tile(const double *A, int64_t lda, int64_t m, int64_t n,
                                                 double *tiles, int nb, int p, int q, int *status)
{
    __shared__ double buf[64][65];
    const int sub = nb / 64;
    const int64_t blk = blockIdx.x;
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

// Tiles -> column-major (A, lda), entries inside m x n only.  Skipped when
// the status flags an error so that A is left as the caller gave it.
__global__ __launch_bounds__(256) void k_tile2cm(double *A, int64_t lda, int64_t m, int64_t n,
                                                 const double *tiles, int nb, int p, int q,
                                                 const int *status)
{
    if (*status != 0) return;
    __shared__ double buf[64][65];
    const int sub = nb / 64;
    const int64_t blk = blockIdx.x;
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

template <int NB, int IB>
static hipError_t serial_impl(const MatDev &M, const int *status, hipStream_t st)
{
    constexpr int NS = Cfg<NB, IB>::NS;
    const int p = M.p, q = M.q, kmax = p < q ? p : q;
    const dim3 blk(Cfg<NB, IB>::NT);
    for (int k = 0; k < kmax; ++k) {
        hipLaunchKernelGGL((k_serial<NB, IB, GEQRT>), dim3(1), blk, 0, st, M, k, k, status);
        if (q - k - 1 > 0)
            hipLaunchKernelGGL((k_serial<NB, IB, LARFB>), dim3((q - k - 1) * NS), blk, 0, st, M, k, k, status);
        for (int i = k + 1; i < p; ++i) {
            hipLaunchKernelGGL((k_serial<NB, IB, TSQRT>), dim3(1), blk, 0, st, M, k, i, status);
            if (q - k - 1 > 0)
                hipLaunchKernelGGL((k_serial<NB, IB, SSRFB>), dim3((q - k - 1) * NS), blk, 0, st, M, k, i, status);
        }
    }
    return hipGetLastError();
}

template <int NB, int IB>
static hipError_t worker_impl(const SchedDev &S, int workers, hipStream_t st)
{
    hipLaunchKernelGGL((k_worker<NB, IB>), dim3(workers), dim3(Cfg<NB, IB>::NT), 0, st, S);
    return hipGetLastError();
}

template <int NB, int IB>
static int worker_occupancy_impl()
{
    int a = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_worker<NB, IB>, Cfg<NB, IB>::NT, 0) != hipSuccess)
        return 1;
    return a > 0 ? a : 1;
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

hipError_t launch_factor_serial(int nb, int ib, const MatDev &M, const int *status, hipStream_t st)
{
#define TQ_CALL(NB, IB) return serial_impl<NB, IB>(M, status, st)
    TQ_DISPATCH(nb, ib, TQ_CALL);
#undef TQ_CALL
}

template <int NB, int IB>
static hipError_t apply_impl(const ApplyDev &D, bool trans, hipStream_t st)
{
    hipLaunchKernelGGL(k_apply_init, dim3(1), dim3(256), 0, st, D.prog, D.kmax, D.M.p, trans ? 1 : 0);
    if (trans)
        hipLaunchKernelGGL((k_apply<NB, IB, true>), dim3(D.kmax), dim3(Cfg<NB, IB>::NT), 0, st, D);
    else
        hipLaunchKernelGGL((k_apply<NB, IB, false>), dim3(D.kmax), dim3(Cfg<NB, IB>::NT), 0, st, D);
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

hipError_t launch_worker(int nb, int ib, const SchedDev &S, int workers, hipStream_t st)
{
#define TQ_CALL(NB, IB) return worker_impl<NB, IB>(S, workers, st)
    TQ_DISPATCH(nb, ib, TQ_CALL);
#undef TQ_CALL
}

int worker_occupancy(int nb, int ib)
{
#define TQ_CALL(NB, IB) return worker_occupancy_impl<NB, IB>()
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
