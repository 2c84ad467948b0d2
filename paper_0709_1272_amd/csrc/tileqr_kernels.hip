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
// Work unit.  Every task runs on one workgroup of 256 threads (4 wave64s).
// The GEMM-shaped parts use v_mfma_f64_16x16x4_f64.  For this instruction
// lane L (n = L % 16, g = L / 16) supplies A[n][g] and B[g][n] and holds
// D[4 r + g][n] in accumulator element r (r = 0..3).  A tile strip of
// 32 columns is held in accumulators, wave w owning rows
// [w nb/4, (w+1) nb/4): element r of row block rb is row
// w nb/4 + 16 rb + 4 r + g, column 16 cb + n.  The same registers then serve
// directly as the B operand of the product V^T X (rows as the contracted
// index: K-chunk r covers rows 16 rb + 4 r .. + 3).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tileqr_dag.h"
#include "tileqr_internal.h"

namespace tq {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;   // threads per workgroup
constexpr int WS = 32;    // strip width (columns) of the GEMM-shaped kernels
constexpr int CB = WS / 16;

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int NB, int IB>
struct Cfg {
    static constexpr int RB = NB / 64;       // 16-row blocks per wave
    static constexpr int IBB = IB / 16;      // 16-wide blocks of the ib dimension
    static constexpr int NPAN = NB / IB;     // inner panels per tile
    static constexpr int LDP = IB + 1;       // LDS row stride of the panel buffer
    static constexpr int RG = NT / IB;       // row groups of the panel factorisation
    static constexpr int RPT = NB / RG;      // panel rows per thread
    static constexpr int NS = NB / WS;       // strips per tile
    static_assert(NB % 64 == 0 && IB % 16 == 0 && NB % IB == 0, "blocking");
};

// A 32-column strip of a tile in accumulator layout (see the file header).
template <int NB, int IB>
struct Strip {
    d4 v[Cfg<NB, IB>::RB][CB];
};

template <int NB, int IB>
struct Smem {
    using C = Cfg<NB, IB>;
    double P[(NB + IB) * C::LDP];    // panel / V: rows 0..nb-1 tile rows, nb.. head rows
    double Wp[4 * IB * WS];          // per-wave partial products
    double Wa[IB * WS];              // reduced W (or the Gram matrix V^T V)
    double Wb[IB * WS];              // T^T W
    double Tl[IB * IB];              // T of the current inner panel
    double tau[IB];
    double red[(2 + IB) * C::RG];    // panel reductions: sum of squares, max, dots
};

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

__device__ __forceinline__ double *tile_ptr(const MatDev &M, int nb, int i, int j)
{
    return M.tiles + ((size_t)j * M.p + i) * (size_t)nb * nb;
}

__device__ __forceinline__ double *tblock_ptr(const MatDev &M, int nb, int ib, int k, int i)
{
    return M.T + ((size_t)k * M.p + i) * (size_t)ib * nb;
}

// X (accumulator layout) <- strip of a row-major tile: columns
// [col0, col0 + 16 cbn), rows of every row block.
template <int NB, int IB>
__device__ __forceinline__ void load_strip(Strip<NB, IB> &X, const double *tile, int ld,
                                           int col0, int cbn)
{
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = wave_id() * (NB / 4);
#pragma unroll
    for (int rb = 0; rb < Cfg<NB, IB>::RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rowbase + rb * 16 + 4 * r + g;
                X.v[rb][cb][r] = cb < cbn ? tile[(size_t)row * ld + col0 + cb * 16 + n] : 0.0;
            }
}

template <int NB, int IB>
__device__ __forceinline__ void store_strip(const Strip<NB, IB> &X, double *tile, int ld,
                                            int col0, int cbn, int rlo)
{
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = wave_id() * (NB / 4);
#pragma unroll
    for (int rb = 0; rb < Cfg<NB, IB>::RB; ++rb) {
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

// Apply the block reflector of one inner panel, held in LDS (sm.P rows
// 0..nb-1 = V, rows below `rlo` ignored; sm.Tl = T), to a strip X:
//   W = [top +] V^T X;  W <- T^T W;  [top -= W;]  X -= V W.
// `top` (may be NULL) points at the ib x (16 cbn) block of the coupled upper
// tile (the R rows the TS form also updates), row stride ldtop.
template <int NB, int IB>
__device__ void apply_panel(Smem<NB, IB> &sm, Strip<NB, IB> &X, int rlo, double *top,
                            int ldtop, int cbn)
{
    using C = Cfg<NB, IB>;
    const int tid = threadIdx.x, w = wave_id();
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = w * (NB / 4);

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
#pragma unroll
    for (int a = 0; a < C::IBB; ++a)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sm.Wp[w * IB * WS + (a * 16 + 4 * r + g) * WS + cb * 16 + n] = Wacc[a][cb][r];
    __syncthreads();
    const int ncol = cbn * 16;
    for (int e = tid; e < IB * WS; e += NT) {
        const int kr = e / WS, c = e % WS;
        double s = ((sm.Wp[e] + sm.Wp[IB * WS + e]) + sm.Wp[2 * IB * WS + e]) + sm.Wp[3 * IB * WS + e];
        if (top != nullptr && c < ncol) s = top[(size_t)kr * ldtop + c] + s;
        sm.Wa[e] = s;
    }
    __syncthreads();
    for (int e = tid; e < IB * WS; e += NT) {
        const int i = e / WS, c = e % WS;
        double s = 0.0;
        for (int kk = 0; kk <= i; ++kk) s += sm.Tl[kk * IB + i] * sm.Wa[kk * WS + c];
        sm.Wb[e] = s;
        if (top != nullptr && c < ncol) top[(size_t)i * ldtop + c] -= s;
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

// Householder factorisation of the ib columns held in sm.P (Section 3.2.1:
// DGEQRT's panel when ts == false, DTSQRT's when ts == true).
//   GEQRT: column j has its head (diagonal) at P row c0 + j and its tail in
//          P rows c0 + j + 1 .. nb - 1.
//   TSQRT: column j has its head at P row nb + j (row j of the triangle R)
//          and its tail in P rows 0 .. nb - 1 (the square tile); the rest of
//          R is untouched by this reflector.
// Reflector: beta = -sign(alpha) ||[alpha; x]|| (sign(0) = +1),
// tau = (beta - alpha) / beta, v = x / (alpha - beta); tau = 0 when x = 0.
// Each thread owns column c = tid % ib and rows rg, rg + RG, ... of the tail.
template <int NB, int IB>
__device__ void panel_factor(Smem<NB, IB> &sm, int c0, bool ts)
{
    using C = Cfg<NB, IB>;
    constexpr int RG = C::RG, RPT = C::RPT, LDP = C::LDP;
    const int tid = threadIdx.x, c = tid % IB, rg = tid / IB;
    double *red_ss = sm.red, *red_mx = sm.red + RG, *red_dot = sm.red + 2 * RG;
    for (int j = 0; j < IB; ++j) {
        const int hrow = ts ? NB + j : c0 + j;
        const int tlo = ts ? 0 : c0 + j + 1;
        const double alpha = sm.P[hrow * LDP + j];
        double xr[RPT];
        double hc = 0.0;
        if (c >= j) {
            double part = 0.0, mx = 0.0;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int r = rg + i * RG;
                const double x = r >= tlo ? sm.P[r * LDP + j] : 0.0;
                xr[i] = x;
                if (c == j) {
                    part += x * x;
                    mx = fmax(mx, fabs(x));
                } else if (r >= tlo) {
                    part += x * sm.P[r * LDP + c];
                }
            }
            if (c == j) {
                red_ss[rg] = part;
                red_mx[rg] = mx;
            } else {
                red_dot[rg * IB + c] = part;
                hc = sm.P[hrow * LDP + c];
            }
        }
        __syncthreads();
        double sig = 0.0, mxa = 0.0;
        for (int q = 0; q < RG; ++q) {
            sig += red_ss[q];
            mxa = fmax(mxa, red_mx[q]);
        }
        double xnorm;
        if (!(sig <= 1.0e300) || (sig < 2.2250738585072014e-308 && mxa > 0.0)) {
            // Sum of squares overflowed or underflowed: recompute it scaled
            // by the largest magnitude (block-uniform branch).
            __syncthreads();
            if (c == j) {
                double part = 0.0;
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const double t = xr[i] / mxa;
                    part += t * t;
                }
                red_ss[rg] = part;
            }
            __syncthreads();
            double s2 = 0.0;
            for (int q = 0; q < RG; ++q) s2 += red_ss[q];
            xnorm = mxa * sqrt(s2);
        } else {
            xnorm = sqrt(sig);
        }
        if (xnorm != 0.0) {
            const double h = hypot(alpha, xnorm);
            const double beta = alpha >= 0.0 ? -h : h;
            const double tau = (beta - alpha) / beta;
            const double scal = 1.0 / (alpha - beta);
            if (c == j) {
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int r = rg + i * RG;
                    if (r >= tlo) sm.P[r * LDP + j] = xr[i] * scal;
                }
                if (rg == 0) {
                    sm.P[hrow * LDP + j] = beta;
                    sm.tau[j] = tau;
                }
            } else if (c > j) {
                double dot = 0.0;
                for (int q = 0; q < RG; ++q) dot += red_dot[q * IB + c];
                const double wv = hc + scal * dot;
                const double tw = tau * wv;
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int r = rg + i * RG;
                    if (r >= tlo) sm.P[r * LDP + c] -= (xr[i] * scal) * tw;
                }
                if (rg == 0) sm.P[hrow * LDP + c] = hc - tw;
            }
        } else if (tid == 0) {
            sm.tau[j] = 0.0;
        }
        __syncthreads();
    }
}

// T of the panel in sm.P (rows >= rlo; V with its unit diagonal explicit):
// G = V^T V on MFMA, then column by column (compact WY, forward)
//   T[j][j] = tau_j,  T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j].
// Leaves T in sm.Tl and writes it to Tg (row-major ib x ib).
template <int NB, int IB>
__device__ void build_t(Smem<NB, IB> &sm, int rlo, double *Tg)
{
    using C = Cfg<NB, IB>;
    const int tid = threadIdx.x, w = wave_id();
    const int n = lane_id() & 15, g = lane_id() >> 4, rowbase = w * (NB / 4);
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
#pragma unroll
    for (int a = 0; a < C::IBB; ++a)
#pragma unroll
        for (int b = 0; b < C::IBB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sm.Wp[w * IB * IB + (a * 16 + 4 * r + g) * IB + b * 16 + n] = G[a][b][r];
    __syncthreads();
    for (int e = tid; e < IB * IB; e += NT)
        sm.Wa[e] = ((sm.Wp[e] + sm.Wp[IB * IB + e]) + sm.Wp[2 * IB * IB + e]) + sm.Wp[3 * IB * IB + e];
    __syncthreads();
    if (tid < IB) {
        const int i = tid;
        for (int j = 0; j < IB; ++j) {
            double v;
            if (i < j) {
                double s = 0.0;
                for (int kk = i; kk < j; ++kk) s += sm.Tl[i * IB + kk] * sm.Wa[kk * IB + j];
                v = -sm.tau[j] * s;
            } else {
                v = i == j ? sm.tau[j] : 0.0;
            }
            sm.Tl[i * IB + j] = v;
        }
    }
    __syncthreads();
    for (int e = tid; e < IB * IB; e += NT) Tg[e] = sm.Tl[e];
}

// V of inner panel l of the diagonal tile into sm.P rows c0..nb-1 with the
// unit diagonal and the zeros above it made explicit.
template <int NB, int IB>
__device__ void load_v_diag(Smem<NB, IB> &sm, const double *tkk, int c0)
{
    using C = Cfg<NB, IB>;
    for (int e = threadIdx.x; e < (NB - c0) * IB; e += NT) {
        const int r = c0 + e / IB, c = e % IB;
        const int d = r - c0;
        double v = tkk[(size_t)r * NB + c0 + c];
        if (d < c) v = 0.0;
        else if (d == c) v = 1.0;
        sm.P[r * C::LDP + c] = v;
    }
}

template <int NB, int IB>
__device__ void load_t(Smem<NB, IB> &sm, const double *Tg)
{
    for (int e = threadIdx.x; e < IB * IB; e += NT) sm.Tl[e] = Tg[e];
}

// ------------------------------------------------------------ tile kernels

// DGEQRT(A_kk) -> (V_kk, R_kk, T_kk).
template <int NB, int IB>
__device__ void task_geqrt(Smem<NB, IB> &sm, const MatDev &M, int k)
{
    using C = Cfg<NB, IB>;
    double *tkk = tile_ptr(M, NB, k, k);
    double *Tk = tblock_ptr(M, NB, IB, k, k);
    for (int l = 0; l < C::NPAN; ++l) {
        const int c0 = l * IB;
        for (int e = threadIdx.x; e < (NB - c0) * IB; e += NT) {
            const int r = c0 + e / IB, c = e % IB;
            sm.P[r * C::LDP + c] = tkk[(size_t)r * NB + c0 + c];
        }
        __syncthreads();
        panel_factor<NB, IB>(sm, c0, false);
        // Write R and V back; keep V with explicit unit diagonal in LDS.
        for (int e = threadIdx.x; e < (NB - c0) * IB; e += NT) {
            const int r = c0 + e / IB, c = e % IB;
            const int d = r - c0;
            const double v = sm.P[r * C::LDP + c];
            tkk[(size_t)r * NB + c0 + c] = v;
            if (d <= c) sm.P[r * C::LDP + c] = d == c ? 1.0 : 0.0;
        }
        __syncthreads();
        build_t<NB, IB>(sm, c0, Tk + l * IB * IB);
        __syncthreads();
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
    double *tkk = tile_ptr(M, NB, k, k);
    double *tik = tile_ptr(M, NB, i, k);
    double *Ti = tblock_ptr(M, NB, IB, k, i);
    for (int l = 0; l < C::NPAN; ++l) {
        const int c0 = l * IB;
        for (int e = threadIdx.x; e < IB * IB; e += NT) {
            const int r = e / IB, c = e % IB;
            sm.P[(NB + r) * C::LDP + c] = r <= c ? tkk[(size_t)(c0 + r) * NB + c0 + c] : 0.0;
        }
        for (int e = threadIdx.x; e < NB * IB; e += NT) {
            const int r = e / IB, c = e % IB;
            sm.P[r * C::LDP + c] = tik[(size_t)r * NB + c0 + c];
        }
        __syncthreads();
        panel_factor<NB, IB>(sm, c0, true);
        for (int e = threadIdx.x; e < IB * IB; e += NT) {
            const int r = e / IB, c = e % IB;
            if (r <= c) tkk[(size_t)(c0 + r) * NB + c0 + c] = sm.P[(NB + r) * C::LDP + c];
        }
        for (int e = threadIdx.x; e < NB * IB; e += NT) {
            const int r = e / IB, c = e % IB;
            tik[(size_t)r * NB + c0 + c] = sm.P[r * C::LDP + c];
        }
        build_t<NB, IB>(sm, 0, Ti + l * IB * IB);
        __syncthreads();
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

// DLARFB: strip s of A_kj <- Q_kk^T A_kj.
template <int NB, int IB>
__device__ void task_larfb(Smem<NB, IB> &sm, const MatDev &M, int k, int j, int s)
{
    using C = Cfg<NB, IB>;
    const double *tkk = tile_ptr(M, NB, k, k);
    double *tkj = tile_ptr(M, NB, k, j);
    const double *Tk = tblock_ptr(M, NB, IB, k, k);
    const int col0 = s * WS;
    Strip<NB, IB> X;
    load_strip<NB, IB>(X, tkj, NB, col0, CB);
    for (int l = 0; l < C::NPAN; ++l) {
        const int c0 = l * IB;
        load_v_diag<NB, IB>(sm, tkk, c0);
        load_t<NB, IB>(sm, Tk + l * IB * IB);
        __syncthreads();
        apply_panel<NB, IB>(sm, X, c0, nullptr, 0, CB);
        __syncthreads();
    }
    store_strip<NB, IB>(X, tkj, NB, col0, CB, 0);
}

// DSSRFB: strip s of [A_kj; A_ij] <- Q_ik^T [A_kj; A_ij].
template <int NB, int IB>
__device__ void task_ssrfb(Smem<NB, IB> &sm, const MatDev &M, int k, int i, int j, int s)
{
    using C = Cfg<NB, IB>;
    const double *tik = tile_ptr(M, NB, i, k);
    double *tkj = tile_ptr(M, NB, k, j);
    double *tij = tile_ptr(M, NB, i, j);
    const double *Ti = tblock_ptr(M, NB, IB, k, i);
    const int col0 = s * WS;
    Strip<NB, IB> X;
    load_strip<NB, IB>(X, tij, NB, col0, CB);
    for (int l = 0; l < C::NPAN; ++l) {
        const int c0 = l * IB;
        for (int e = threadIdx.x; e < NB * IB; e += NT) {
            const int r = e / IB, c = e % IB;
            sm.P[r * C::LDP + c] = tik[(size_t)r * NB + c0 + c];
        }
        load_t<NB, IB>(sm, Ti + l * IB * IB);
        __syncthreads();
        apply_panel<NB, IB>(sm, X, 0, tkj + (size_t)c0 * NB + col0, NB, CB);
        __syncthreads();
    }
    store_strip<NB, IB>(X, tij, NB, col0, CB, 0);
}

template <int NB, int IB>
__device__ void run_task(Smem<NB, IB> &sm, const MatDev &M, const Task &t)
{
    switch (t.type) {
    case GEQRT: task_geqrt<NB, IB>(sm, M, t.k); break;
    case TSQRT: task_tsqrt<NB, IB>(sm, M, t.k, t.i); break;
    case LARFB: task_larfb<NB, IB>(sm, M, t.k, t.j, t.s); break;
    default: task_ssrfb<NB, IB>(sm, M, t.k, t.i, t.j, t.s); break;
    }
}

// ------------------------------------------------ serial (Algorithm 2) kernels

// One launch per group of independent tasks in Algorithm 2's loop order:
// GEQRT(k) / TSQRT(k, i): one workgroup; LARFB(k, .) / SSRFB(k, i, .):
// one workgroup per (j, strip).
template <int NB, int IB>
__global__ __launch_bounds__(NT) void k_serial(MatDev M, int type, int k, int i, const int *status)
{
    __shared__ Smem<NB, IB> sm;
    if (*status != 0) return;
    constexpr int NS = Cfg<NB, IB>::NS;
    Task t;
    t.type = type;
    t.k = k;
    t.i = i;
    t.j = k + 1 + blockIdx.x / NS;
    t.s = blockIdx.x % NS;
    run_task<NB, IB>(sm, M, t);
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

__device__ __forceinline__ void push_task(const SchedDev &S, int level, int64_t gid)
{
    const uint32_t slot = __hip_atomic_fetch_add(&S.qtail[level * 32], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&S.qslot[S.qoff[level] + slot], (int32_t)(gid + 1), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Non-blocking pop: -1 when the queue has nothing claimable right now.
__device__ __forceinline__ int64_t pop_task(const SchedDev &S, int level)
{
    for (int attempt = 0; attempt < 4; ++attempt) {
        const uint32_t h = ld_rlx(&S.qhead[level * 32]);
        const uint32_t t = ld_rlx(&S.qtail[level * 32]);
        if (h >= t) return -1;
        const int32_t v = ld_acq(&S.qslot[S.qoff[level] + h]);
        if (v == 0) return -1;
        uint32_t expect = h;
        if (__hip_atomic_compare_exchange_strong(&S.qhead[level * 32], &expect, h + 1, __ATOMIC_ACQ_REL,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return (int64_t)v - 1;
    }
    return -1;
}

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
    if (tid0 < 4 * 32) {
        S.qhead[tid0] = 0;
        S.qtail[tid0] = 0;
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
        S.qslot[S.qoff[0] + mi] = (int32_t)(S.mats[mi].task_base + 1);
    __syncthreads();
    if (threadIdx.x == 0) S.qtail[0] = (uint32_t)S.nmat;
}

template <int NB, int IB>
__global__ __launch_bounds__(NT) void k_worker(SchedDev S)
{
    __shared__ Smem<NB, IB> sm;
    __shared__ int64_t s_gid;
    __shared__ int s_exit;
    const int tid = threadIdx.x;
    uint64_t rng = mix64(S.seed ^ (0x9e3779b97f4a7c15ULL * (blockIdx.x + 1)));
    for (;;) {
        if (tid == 0) {
            int64_t gid = -1;
            int ex = 0;
            int64_t idle = 0;
            uint32_t seen = ld_rlx(S.done);
            for (;;) {
                if (__hip_atomic_load(S.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    ex = 1;
                    break;
                }
                if (S.shuffle) {
                    rng = mix64(rng + 1);
                    for (int z = 0; z < (int)(rng & 7); ++z) __builtin_amdgcn_s_sleep(1);
                    const int start = (int)((rng >> 8) & 3);
                    for (int q = 0; q < 4 && gid < 0; ++q) gid = pop_task(S, (start + q) & 3);
                } else {
                    for (int q = 0; q < 4 && gid < 0; ++q) gid = pop_task(S, q);
                }
                if (gid >= 0) break;
                const uint32_t d = ld_rlx(S.done);
                if (d >= S.total_tasks) { ex = 1; break; }
                if (d != seen) {
                    seen = d;
                    idle = 0;
                } else if (++idle > S.spin_limit) {
                    __hip_atomic_fetch_or(S.status, STATUS_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ex = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            s_gid = gid;
            s_exit = ex;
        }
        __syncthreads();
        if (s_exit) break;
        const int64_t gid = s_gid;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int mi = find_mat(S, gid);
        const MatDev &M = S.mats[mi];
        const Grid g = make_grid(M.p, M.q, S.ns);
        const Task t = decode(g, gid - M.task_base);
        const uint64_t t0 = wall_clock64();
        run_task<NB, IB>(sm, M, t);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        const int ns = nsucc(g, t);
        for (int n = tid; n < ns; n += NT) {
            if (S.drop_edge >= 0 && gid == S.drop_edge && n == 0) continue;
            const int64_t sl = succ(g, t, n);
            const int32_t old = __hip_atomic_fetch_add(&S.counters[M.task_base + sl], -1, __ATOMIC_ACQ_REL,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            if (old == 1) push_task(S, decode(g, sl).type, M.task_base + sl);
        }
        if (tid == 0) {
            if (S.trace != nullptr) {
                const uint32_t e = __hip_atomic_fetch_add(S.trace_count, 1u, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                if (e < S.trace_cap) {
                    int64_t *ev = S.trace + (size_t)e * 8;
                    ev[0] = t.type; ev[1] = t.k; ev[2] = t.i; ev[3] = t.j; ev[4] = t.s;
                    ev[5] = mi * 65536 + blockIdx.x;
                    ev[6] = (int64_t)t0;
                    ev[7] = (int64_t)wall_clock64();
                }
            }
            __hip_atomic_fetch_add(S.done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
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
    for (int k = 0; k < kmax; ++k) {
        hipLaunchKernelGGL((k_serial<NB, IB>), dim3(1), dim3(NT), 0, st, M, (int)GEQRT, k, k, status);
        if (q - k - 1 > 0)
            hipLaunchKernelGGL((k_serial<NB, IB>), dim3((q - k - 1) * NS), dim3(NT), 0, st, M, (int)LARFB, k,
                               k, status);
        for (int i = k + 1; i < p; ++i) {
            hipLaunchKernelGGL((k_serial<NB, IB>), dim3(1), dim3(NT), 0, st, M, (int)TSQRT, k, i, status);
            if (q - k - 1 > 0)
                hipLaunchKernelGGL((k_serial<NB, IB>), dim3((q - k - 1) * NS), dim3(NT), 0, st, M, (int)SSRFB,
                                   k, i, status);
        }
    }
    return hipGetLastError();
}

template <int NB, int IB>
static hipError_t worker_impl(const SchedDev &S, int workers, hipStream_t st)
{
    hipLaunchKernelGGL((k_worker<NB, IB>), dim3(workers), dim3(NT), 0, st, S);
    return hipGetLastError();
}

template <int NB, int IB>
static int worker_occupancy_impl()
{
    int nblk = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, k_worker<NB, IB>, NT, 0) != hipSuccess) return 1;
    return nblk > 0 ? nblk : 1;
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
