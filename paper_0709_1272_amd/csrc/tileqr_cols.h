// Split-precision SSRFB by reflector blocks of up to four inner panels.
// Included by tileqr_tile.h after the split-precision helpers.
//
// DSSRFB (Section 3.2.1) applies the coupled block reflector of TSQRT(k, i)
// to the tile pair [A_kj; A_ij].  Inner blocking (Section 3.2.3) applies it
// one group of s reflectors at a time; here a group is a "half" of up to
// HP = 4 inner panels of 32 (s = 128 at nb = 256, s = nb below), whose
// T_h = [[T_a, -T_a (V_a^T V_b) T_b], [0, T_b]] (recursively over the
// panels) is formed once per TS tile by the last TSQRT panel.  Per half:
//   W = A_kj[half rows] + V_h^T A_ij      (K = nb)
//   W' = T_h^T W;  A_kj[half rows] -= W'
//   A_ij -= V_h W'                       (K = s)
// so the strip of A_ij is split into narrow parts once per half, not once
// per inner panel, and each product is a block of MFMAs with few
// workgroup barriers between the phases.  The paper's cost 4b^3 + s b^2
// (Section 3.2.3) grows by the larger s: 4.5 b^3 at b = 256, s = 128.
//
// The operands of the three products are split into narrow parts
// (x = x0 + x1 [+ x2], each part the rounded remainder, formed in FP32 from
// x rounded to FP32) and run on the 16x16x32 narrow MFMAs with FP32
// accumulation.  V is split once, by the TSQRT panel that forms it, into the
// exact register images the MFMAs take (one 16-byte vector of 8 narrow
// values per lane), in two layouts: one for V^T X (a lane takes 8 rows of
// one column) and one for V W (8 columns of one row); T_h^T likewise.
//
// Lane layout of v_mfma_f32_16x16x32_{bf16,f16} (lane L = 16 g + n): A[n][8g+e]
// and B[8g+e][n] in element e, D[4g+r][n] in element r.  The K index of every
// product is permuted the same way on both operands: position 8g + e stands
// for row (or column) 16 (e / 4) + 4 g + e % 4 of its 32-block, which is where
// the D layout leaves rows 4 g + r of two 16-row blocks, so results feed the
// next product without a shuffle.
#pragma once

namespace tq {

typedef uint32_t u4 __attribute__((ext_vector_type(4)));
typedef uint32_t u2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) u4 gu4;

// LDS bytes the split update needs (parts: 3 at most).
template <int NB>
struct SxLds {
    using C = SxCfg<NB>;
    static constexpr int XS = C::NCH * C::NCB * 3 * 64 * 16;   // X images
    static constexpr int WS = C::HP * C::NCB * 3 * 64 * 16;    // W or W' images
    static constexpr int XSC = C::NCH * C::WSX * 8;            // inverse X scales per chunk and column
    static constexpr int WMAX = C::NW * C::WSX * 8;            // column maxima per wave
    static constexpr int BYTES = XS + WS + XSC + WMAX;
    // T_h build in the TSQRT task: Gram blocks, T_h blocks, Y scratch (FP32).
    static constexpr int BUILD = (C::NPAIR + C::NTB + C::HP) * 1024 * 4 + 16 * 8;
};

// Strips per tile of the LARFB / SSRFB tasks: 32 columns in FP64, the
// split update's strip width in the split modes.
template <int NB, int PREC>
__host__ __device__ constexpr int strips_of()
{
    return PREC == PREC_FP64 ? NB / WS : SxCfg<NB>::NSX;
}

template <int NB, int PREC>
__device__ __forceinline__ gu4 *sx_tile(const MatDev &M, int k, int i)
{
    using L = SxLayout<NB, Narrow<PREC>::NPART>;
    return (gu4 *)M.vsplit + ((size_t)k * M.p + i) * L::TILE;
}

// Scale applied to V's parts: |v| <= 1 for every reflector entry
// (|alpha - beta| >= |x_i|), so a fixed power of two keeps the FP16 parts
// out of the subnormal range.
template <int PREC>
__device__ __forceinline__ constexpr double v_scale()
{
    return PREC == PREC_FP16X2 ? 4096.0 : 1.0;
}

// Power-of-two scale s (and 1 / s) that brings m > 0 into [2^14, 2^15).
__device__ __forceinline__ void pow2_scale(double m, double &s, double &inv)
{
    int ex = 0;
    if (m > 0.0) (void)frexp(m, &ex);
    ex = ex < -1000 ? -1000 : (ex > 1000 ? 1000 : ex);
    s = ldexp(1.0, 15 - ex);
    inv = ldexp(1.0, ex - 15);
}

// The narrow parts of x[e] * scale, formed in FP32: f = RN_f32(x s), then
// part q = RN_narrow(f), f <- f - part q (exact in FP32).
template <int PREC>
__device__ __forceinline__ void split8_f32(const double (&x)[8], double scale, Parts<PREC> &P)
{
    using E = typename Narrow<PREC>::elem;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        float f = (float)(x[e] * scale);
#pragma unroll
        for (int q = 0; q < Narrow<PREC>::NPART; ++q) {
            const E h = (E)f;
            P.p[q][e] = h;
            f = f - (float)h;
        }
    }
}

template <int PREC>
__device__ __forceinline__ u4 as_u4(const typename Narrow<PREC>::vec &v)
{
    return __builtin_bit_cast(u4, v);
}

template <int PREC>
__device__ __forceinline__ typename Narrow<PREC>::vec from_u4(u4 v)
{
    return __builtin_bit_cast(typename Narrow<PREC>::vec, v);
}

template <int PREC>
__device__ __forceinline__ void load_parts(Parts<PREC> &A, const gu4 *src)
{
#pragma unroll
    for (int q = 0; q < Narrow<PREC>::NPART; ++q) A.p[q] = from_u4<PREC>(src[q * 64]);
}

template <int PREC>
__device__ __forceinline__ void load_parts_lds(Parts<PREC> &A, const u4 *src)
{
#pragma unroll
    for (int q = 0; q < Narrow<PREC>::NPART; ++q) A.p[q] = from_u4<PREC>(src[q * 64]);
}

// Largest |value| of a 16-column block column over a wave: the lane's own
// entries and those of the three other lanes of its column.
template <int CNT>
__device__ __forceinline__ double column_max(const double *v)
{
    double m = 0.0;
#pragma unroll
    for (int e = 0; e < CNT; ++e) m = fmax(m, fabs(v[e]));
    m = fmax(m, __shfl_xor(m, 16));
    m = fmax(m, __shfl_xor(m, 32));
    return m;
}

// Writes the V images of inner panel l of TS tile (i, k): V (rows 0..nb-1,
// columns 0..ib-1 of sm.P, FP64), complete in LDS (the caller has passed a
// barrier since it was formed).
template <int NB, int IB, int PREC>
__device__ __forceinline__ void write_vsplit(const Smem<NB, IB> &sm, gu4 *dst)
{
    static_assert(IB == 32, "split images take ib = 32");
    using C = Cfg<NB, IB>;
    using X = SxCfg<NB>;
    constexpr int P = Narrow<PREC>::NPART;
    using L = SxLayout<NB, P>;
    constexpr double VS = v_scale<PREC>();
    const int tid = threadIdx.x;
    // V^T X images: chunk c, block a, lane (n, g), element e = V[32c + 16(e/4) + 4g + e%4][16a + n].
    constexpr int NVTX = X::NCH * 2 * 64;
#pragma unroll
    for (int u = 0; u < NVTX / C::NT; ++u) {
        const int v = tid + u * C::NT, ln = v & 63, ca = v >> 6, c = ca >> 1, a = ca & 1;
        const int nn = ln & 15, gg = ln >> 4;
        double xv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) xv[e] = sm.P[(32 * c + 16 * (e >> 2) + 4 * gg + (e & 3)) * C::LDP + 16 * a + nn];
        Parts<PREC> Pt;
        split8_f32<PREC>(xv, VS, Pt);
#pragma unroll
        for (int q = 0; q < P; ++q) dst[(ca * P + q) * 64 + ln] = as_u4<PREC>(Pt.p[q]);
    }
    // V W images: row block rb, lane (n, g), element e = V[16 rb + n][16(e/4) + 4g + e%4].
    constexpr int NVW = X::NRB * 64;
#pragma unroll
    for (int u = 0; u < NVW / C::NT; ++u) {
        const int v = tid + u * C::NT, ln = v & 63, rb = v >> 6;
        const int nn = ln & 15, gg = ln >> 4;
        double xv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) xv[e] = sm.P[(16 * rb + nn) * C::LDP + 16 * (e >> 2) + 4 * gg + (e & 3)];
        Parts<PREC> Pt;
        split8_f32<PREC>(xv, VS, Pt);
#pragma unroll
        for (int q = 0; q < P; ++q) dst[L::VTX_SZ + (rb * P + q) * 64 + ln] = as_u4<PREC>(Pt.p[q]);
    }
}

// After the last inner panel of TS tile (i, k) (every panel's V images and
// T_l in memory): for each reflector block h, T_h in FP32 by the column
// recurrence T_{0:m+1} = [[T_{0:m}, -T_{0:m} G_{0:m,m} T_m], [0, T_m]] with
// the Gram blocks G_lm = V_l^T V_m (from the V images on the narrow MFMAs),
// then the T_h^T images with one power-of-two scale per 16-column block of
// T_h.  Uses the workgroup's LDS (nothing else live) and ends with a barrier.
template <int NB, int IB, int PREC>
__device__ __forceinline__ void build_th(Smem<NB, IB> &sm, const MatDev &M, int k, int i)
{
    using C = SxCfg<NB>;
    constexpr int P = Narrow<PREC>::NPART;
    using L = SxLayout<NB, P>;
    static_assert(SxLds<NB>::BUILD <= (int)sizeof(Smem<NB, IB>), "T_h build fits in LDS");
    constexpr int NT = 64 * C::NW;
    constexpr double VS = v_scale<PREC>();
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, n = lane & 15, g = lane >> 4;
    float *Gs = reinterpret_cast<float *>(&sm);       // [pair][32][32]
    float *Tb = Gs + C::NPAIR * 1024;                   // [block (l <= m)][32][32]
    float *Ys = Tb + C::NTB * 1024;                     // [l][32][32]
    double *sinv = reinterpret_cast<double *>(Ys + C::HP * 1024);   // [16]
    gu4 *base = sx_tile<NB, PREC>(M, k, i);
    const gdouble *Ti = tblock_ptr(M, NB, IB, k, i);
    // Block index of T_h[l][m] (l <= m) and pair index of G[l][m] (l < m).
    auto tb = [](int l, int m) { return m * (m + 1) / 2 + l; };
    auto pr = [](int l, int m) { return m * (m - 1) / 2 + l; };
#pragma unroll 1
    for (int h = 0; h < C::NH; ++h) {
        const int l0 = h * C::HP;
        __syncthreads();
        // Gram blocks: 16 x 16 tiles (pair, a, a'), K over the tile's chunks.
#pragma unroll 1
        for (int it = w; it < C::NPAIR * 4; it += C::NW) {
            const int pi = it >> 2, a = (it >> 1) & 1, a2 = it & 1;
            int m = 1;
            while (m * (m + 1) / 2 <= pi) ++m;
            const int l = pi - m * (m - 1) / 2;
            const gu4 *vl = base + (size_t)(l0 + l) * L::PANEL, *vm = base + (size_t)(l0 + m) * L::PANEL;
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
            for (int c = 0; c < C::NCH; ++c) {
                Parts<PREC> A, B;
                load_parts<PREC>(A, vl + ((c * 2 + a) * P) * 64 + lane);
                load_parts<PREC>(B, vm + ((c * 2 + a2) * P) * 64 + lane);
                acc += split_product<PREC>(A, B);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Gs[pi * 1024 + (16 * a + 4 * g + r) * 32 + 16 * a2 + n] = acc[r] * (float)(1.0 / (VS * VS));
        }
        // Diagonal blocks T_l (upper triangular, from memory).
        for (int e = tid; e < C::HP * 1024; e += NT) {
            const int l = e >> 10, r = (e >> 5) & 31, c = e & 31;
            Tb[tb(l, l) * 1024 + r * 32 + c] = r <= c ? (float)Ti[(size_t)(l0 + l) * 1024 + r * 32 + c] : 0.f;
        }
        __syncthreads();
#pragma unroll 1
        for (int m = 1; m < C::HP; ++m) {
            // Y_l = G_lm T_m (l < m).
            for (int e = tid; e < m * 1024; e += NT) {
                const int l = e >> 10, r = (e >> 5) & 31, c = e & 31;
                const float *gr = Gs + pr(l, m) * 1024 + r * 32;
                const float *tm = Tb + tb(m, m) * 1024;
                float s = 0.f;
                for (int q = 0; q <= c; ++q) s += gr[q] * tm[q * 32 + c];
                Ys[l * 1024 + r * 32 + c] = s;
            }
            __syncthreads();
            // T_h[l][m] = -sum_{l' = l .. m-1} T_h[l][l'] Y_l'.
            for (int e = tid; e < m * 1024; e += NT) {
                const int l = e >> 10, r = (e >> 5) & 31, c = e & 31;
                float s = 0.f;
                for (int lp = l; lp < m; ++lp) {
                    const float *tr = Tb + tb(l, lp) * 1024 + r * 32;
                    const float *yc = Ys + lp * 1024 + c;
                    for (int q = lp == l ? r : 0; q < 32; ++q) s += tr[q] * yc[q * 32];
                }
                Tb[tb(l, m) * 1024 + r * 32 + c] = -s;
            }
            __syncthreads();
        }
        // One scale per 16-column block rb of T_h (rows 0 .. 32 (rb / 2) + 31).
        if (tid < 64 * ((C::HRB + 3) / 4)) {
            // wave-sized groups of 16 lanes per block: lane n of group rb.
            const int rb = tid >> 4, cn = tid & 15;
            float mx = 0.f;
            if (rb < C::HRB) {
                const int mblk = rb >> 1, c = 16 * (rb & 1) + cn;
                for (int l = 0; l <= mblk; ++l)
                    for (int r = 0; r < 32; ++r) mx = fmaxf(mx, fabsf(Tb[tb(l, mblk) * 1024 + r * 32 + c]));
            }
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 16));
            if (rb < C::HRB && cn == 0) {
                double s, inv;
                pow2_scale((double)mx, s, inv);
                sinv[rb] = inv;
            }
        }
        __syncthreads();
        gu4 *th = base + (size_t)C::NP * L::PANEL + (size_t)h * L::HALF;
        // Images: row block rb, chunk kc <= rb / 2, lane (n, g), element
        // e = T_h[32 kc + 16(e/4) + 4g + e%4][16 rb + n] (times the block's scale).
        for (int v = tid; v < C::HRB * C::HP * 64; v += NT) {
            const int ln = v & 63, blk = v >> 6, rb = blk / C::HP, kc = blk % C::HP;
            if (kc > rb / 2) continue;
            const int nn = ln & 15, gg = ln >> 4, mblk = rb >> 1, c = 16 * (rb & 1) + nn;
            const double s = 1.0 / sinv[rb];
            double xv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) xv[e] = (double)Tb[tb(kc, mblk) * 1024 + (16 * (e >> 2) + 4 * gg + (e & 3)) * 32 + c];
            Parts<PREC> Pt;
            split8_f32<PREC>(xv, s, Pt);
#pragma unroll
            for (int q = 0; q < P; ++q) th[((rb * C::HP + kc) * P + q) * 64 + ln] = as_u4<PREC>(Pt.p[q]);
        }
        if (tid < C::HRB) reinterpret_cast<gdouble *>(th + L::TH_IMG)[tid] = sinv[tid];
    }
    __syncthreads();
}

// DSSRFB(k, i, j, s) in a split precision: strip s (64 columns) of
// [A_kj; A_ij] <- Q_ik^T [A_kj; A_ij], one reflector block of up to four
// inner panels at a time, with the images TSQRT(k, i) wrote.  Wave w keeps
// rows 32 w .. 32 w + 31 of the strip of A_ij (chunk w) in FP64 registers
// for the whole task, and per block the rows RPW w .. of W.
template <int NB, int IB, int PREC>
__device__ __forceinline__ void task_ssrfb_mx(Smem<NB, IB> &sm, const MatDev &M, int k, int i, int j, int s)
{
    using C = SxCfg<NB>;
    constexpr int P = Narrow<PREC>::NPART;
    using L = SxLayout<NB, P>;
    using LD = SxLds<NB>;
    static_assert(IB == 32, "split images take ib = 32");
    static_assert(LD::BYTES <= (int)sizeof(Smem<NB, IB>), "the split update fits in LDS");
    constexpr double VINV = 1.0 / v_scale<PREC>();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
    const int col0 = s * C::WSX;
    gdouble *X = tile_ptr(M, NB, i, j);
    gdouble *top = tile_ptr(M, NB, k, j);
    const gu4 *img = sx_tile<NB, PREC>(M, k, i);
    char *raw = reinterpret_cast<char *>(&sm);
    u4 *XS = reinterpret_cast<u4 *>(raw);                          // [c][cb][q][lane]
    u4 *WSm = reinterpret_cast<u4 *>(raw + LD::XS);                // [kc][cb][q][lane]
    double *xsc = reinterpret_cast<double *>(raw + LD::XS + LD::WS);   // [c][64]
    double *wmax = xsc + C::NCH * C::WSX;                          // [w][64]

    // The wave's rows of A_ij: row blocks 2w, 2w + 1, element r of lane
    // (n, g) is row 16 rb + 4g + r, column col0 + 16 cb + n.
    double x[2][C::NCB][4];
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int cb = 0; cb < C::NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) x[jj][cb][r] = X[(size_t)(32 * w + 16 * jj + 4 * g + r) * NB + col0 + 16 * cb + n];

#pragma unroll 1
    for (int h = 0; h < C::NH; ++h) {
        // X images of chunk w, one scale per column over the chunk's rows.
#pragma unroll
        for (int cb = 0; cb < C::NCB; ++cb) {
            double xv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) xv[e] = x[e >> 2][cb][e & 3];
            double sc, inv;
            pow2_scale(column_max<8>(xv), sc, inv);
            Parts<PREC> Pt;
            split8_f32<PREC>(xv, sc, Pt);
#pragma unroll
            for (int q = 0; q < P; ++q) XS[((w * C::NCB + cb) * P + q) * 64 + lane] = as_u4<PREC>(Pt.p[q]);
            if (g == 0) xsc[w * C::WSX + 16 * cb + n] = inv * VINV;
        }
        // W = top rows + V_h^T X for the wave's row blocks of this block
        // (local rb = RPW w + jj: panel HP h + rb / 2, block rb % 2).
        double W[C::RPW][C::NCB][4];
#pragma unroll
        for (int jj = 0; jj < C::RPW; ++jj) {
            const int row = 16 * (C::HRB * h + C::RPW * w + jj);
#pragma unroll
            for (int cb = 0; cb < C::NCB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) W[jj][cb][r] = top[(size_t)(row + 4 * g + r) * NB + col0 + 16 * cb + n];
        }
        __syncthreads();
#pragma unroll 1
        for (int c = 0; c < C::NCH; ++c) {
            Parts<PREC> Bx[C::NCB];
#pragma unroll
            for (int cb = 0; cb < C::NCB; ++cb) load_parts_lds<PREC>(Bx[cb], XS + ((c * C::NCB + cb) * P) * 64 + lane);
            double u[C::NCB];
#pragma unroll
            for (int cb = 0; cb < C::NCB; ++cb) u[cb] = xsc[c * C::WSX + 16 * cb + n];
#pragma unroll
            for (int jj = 0; jj < C::RPW; ++jj) {
                const int rb = C::RPW * w + jj;
                Parts<PREC> Av;
                load_parts<PREC>(Av, img + (size_t)(C::HP * h + rb / 2) * L::PANEL + ((c * 2 + (rb & 1)) * P) * 64 + lane);
#pragma unroll
                for (int cb = 0; cb < C::NCB; ++cb) {
                    const f4 d = split_product<PREC>(Av, Bx[cb]);
#pragma unroll
                    for (int r = 0; r < 4; ++r) W[jj][cb][r] += (double)d[r] * u[cb];
                }
            }
        }
        // Column maxima of W over the block's rows (all waves).
#pragma unroll
        for (int cb = 0; cb < C::NCB; ++cb) {
            double m = 0.0;
#pragma unroll
            for (int jj = 0; jj < C::RPW; ++jj)
#pragma unroll
                for (int r = 0; r < 4; ++r) m = fmax(m, fabs(W[jj][cb][r]));
            m = fmax(m, __shfl_xor(m, 16));
            m = fmax(m, __shfl_xor(m, 32));
            if (g == 0) wmax[w * C::WSX + 16 * cb + n] = m;
        }
        __syncthreads();
        double wsi[C::NCB];
#pragma unroll
        for (int cb = 0; cb < C::NCB; ++cb) {
            double m = 0.0;
#pragma unroll
            for (int ww = 0; ww < C::NW; ++ww) m = fmax(m, wmax[ww * C::WSX + 16 * cb + n]);
            double sc, inv;
            pow2_scale(m, sc, inv);
            wsi[cb] = inv;
            // The wave's rows are elements 4 (rb % 2) .. of chunk rb / 2.
#pragma unroll
            for (int jj = 0; jj < C::RPW; ++jj) {
                const int rb = C::RPW * w + jj;
                double xv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) xv[e] = W[jj][cb][e & 3];
                Parts<PREC> Pt;
                split8_f32<PREC>(xv, sc, Pt);
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const u4 v = as_u4<PREC>(Pt.p[q]);
                    u2 *dst = reinterpret_cast<u2 *>(WSm + (((rb >> 1) * C::NCB + cb) * P + q) * 64 + lane) + (rb & 1);
                    *dst = (u2){v.x, v.y};
                }
            }
        }
        __syncthreads();
        // W' = T_h^T W for the wave's row blocks; the top rows take -W'.
        const gu4 *th = img + (size_t)C::NP * L::PANEL + (size_t)h * L::HALF;
        const gdouble *thsc = reinterpret_cast<const gdouble *>(th + L::TH_IMG);
        double Wp[C::RPW][C::NCB][4];
#pragma unroll
        for (int jj = 0; jj < C::RPW; ++jj) {
            const int rb = C::RPW * w + jj;
            f4 acc[C::NCB];
#pragma unroll
            for (int cb = 0; cb < C::NCB; ++cb) acc[cb] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
            for (int kc = 0; kc <= rb / 2; ++kc) {
                Parts<PREC> At;
                load_parts<PREC>(At, th + ((rb * C::HP + kc) * P) * 64 + lane);
#pragma unroll
                for (int cb = 0; cb < C::NCB; ++cb) {
                    Parts<PREC> Bw;
                    load_parts_lds<PREC>(Bw, WSm + ((kc * C::NCB + cb) * P) * 64 + lane);
                    acc[cb] += split_product<PREC>(At, Bw);
                }
            }
            const double tsi = thsc[rb];
            const int row = 16 * (C::HRB * h + rb);
#pragma unroll
            for (int cb = 0; cb < C::NCB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    Wp[jj][cb][r] = (double)acc[cb][r] * (tsi * wsi[cb]);
                    gdouble *tp = top + (size_t)(row + 4 * g + r) * NB + col0 + 16 * cb + n;
                    *tp = *tp - Wp[jj][cb][r];
                }
        }
        // Column maxima of W' (every wave is past its reads of W's images).
#pragma unroll
        for (int cb = 0; cb < C::NCB; ++cb) {
            double m = 0.0;
#pragma unroll
            for (int jj = 0; jj < C::RPW; ++jj)
#pragma unroll
                for (int r = 0; r < 4; ++r) m = fmax(m, fabs(Wp[jj][cb][r]));
            m = fmax(m, __shfl_xor(m, 16));
            m = fmax(m, __shfl_xor(m, 32));
            if (g == 0) wmax[w * C::WSX + 16 * cb + n] = m;
        }
        __syncthreads();
        double wpi[C::NCB];
#pragma unroll
        for (int cb = 0; cb < C::NCB; ++cb) {
            double m = 0.0;
#pragma unroll
            for (int ww = 0; ww < C::NW; ++ww) m = fmax(m, wmax[ww * C::WSX + 16 * cb + n]);
            double sc, inv;
            pow2_scale(m, sc, inv);
            wpi[cb] = inv * VINV;
#pragma unroll
            for (int jj = 0; jj < C::RPW; ++jj) {
                const int rb = C::RPW * w + jj;
                double xv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) xv[e] = Wp[jj][cb][e & 3];
                Parts<PREC> Pt;
                split8_f32<PREC>(xv, sc, Pt);
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const u4 v = as_u4<PREC>(Pt.p[q]);
                    u2 *dst = reinterpret_cast<u2 *>(WSm + (((rb >> 1) * C::NCB + cb) * P + q) * 64 + lane) + (rb & 1);
                    *dst = (u2){v.x, v.y};
                }
            }
        }
        __syncthreads();
        // X -= V_h W' for the wave's rows (chunk w), K over the block's panels.
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            f4 acc[C::NCB];
#pragma unroll
            for (int cb = 0; cb < C::NCB; ++cb) acc[cb] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
            for (int kc = 0; kc < C::HP; ++kc) {
                Parts<PREC> Av;
                load_parts<PREC>(Av, img + (size_t)(C::HP * h + kc) * L::PANEL + L::VTX_SZ + ((2 * w + jj) * P) * 64 + lane);
#pragma unroll
                for (int cb = 0; cb < C::NCB; ++cb) {
                    Parts<PREC> Bw;
                    load_parts_lds<PREC>(Bw, WSm + ((kc * C::NCB + cb) * P) * 64 + lane);
                    acc[cb] += split_product<PREC>(Av, Bw);
                }
            }
#pragma unroll
            for (int cb = 0; cb < C::NCB; ++cb)
#pragma unroll
                for (int r = 0; r < 4; ++r) x[jj][cb][r] -= (double)acc[cb][r] * wpi[cb];
        }
        // No barrier: the next block's first writes (X images, W column
        // maxima) go to memory every wave finished reading before the
        // barriers above.
    }
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
#pragma unroll
        for (int cb = 0; cb < C::NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) X[(size_t)(32 * w + 16 * jj + 4 * g + r) * NB + col0 + 16 * cb + n] = x[jj][cb][r];
}

}  // namespace tq
