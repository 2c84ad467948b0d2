// Split-precision SSRFB by column blocks, with reflectors split once.
// Included by tileqr_tile.h after the split-precision helpers.
//
// DSSRFB (Section 3.2.1) applies the coupled block reflector of TSQRT(k, i)
// to the tile pair [A_kj; A_ij], one inner panel of ib = 32 reflectors at a
// time (Section 3.2.3):
//   W = A_kj[panel rows] + V_l^T A_ij;  W <- T_l^T W;
//   A_kj[panel rows] -= W;  A_ij -= V_l W.
// Here a task takes a strip of WSX columns, and each wave owns a block of
// 16 columns over RPW rows of A_ij, held in FP64 registers for the whole
// task.  V_l^T A_ij then needs no reduction across waves except between the
// two row halves of a tile of 256 rows (one exchange through LDS), so an
// inner panel costs one exchange and two barriers around the staging of the
// next panel instead of three barriers and a slot reduction per 32 columns.
//
// The operands of the three products are split into narrow parts
// (x = x0 + x1 [+ x2], each part the rounded remainder, formed in FP32 from
// x rounded to FP32) and run on the 16x16x32 narrow MFMAs with FP32
// accumulation per 32-row chunk and FP64 accumulation across chunks.  V and
// T are split once, by the TSQRT panel that forms them, into the exact
// register images the MFMAs take (one 16-byte vector of 8 narrow values per
// lane), in two layouts for V: one for V^T X (a lane takes 8 rows of one
// column) and one for V W (8 columns of one row).  The update task stages a
// panel's images in LDS with plain 16-byte copies, prefetched one panel
// ahead into registers.
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
typedef __attribute__((address_space(1))) u4 gu4;

// Geometry of the column-block update for tile size NB.
template <int NB>
struct ColCfg {
    static constexpr int NW = NB / 32;             // waves of the workgroup
    static constexpr int RH = NB >= 256 ? 2 : 1;   // row halves of a tile
    static constexpr int NCB = NW / RH;            // 16-column blocks per strip
    static constexpr int WSX = 16 * NCB;           // strip width (64 for nb 128, 256; 32 for nb 64)
    static constexpr int NSX = NB / WSX;           // strips per tile
    static constexpr int RPW = NB / RH;            // rows per wave
    static constexpr int RBW = RPW / 16;           // 16-row blocks per wave
    static constexpr int CHW = RPW / 32;           // 32-row chunks per wave
};

// Split images of one inner panel of one TS tile, in 16-byte vectors, in
// two regions: A (the images the products before the coupled-row update
// read) and B (those of the product after it), staged into LDS at
// different points of the panel.
template <int NB, int P>
struct VsLayout {
    static constexpr int VTX = 0;                                // A: [chunk c][block a][part][lane]
    static constexpr int TT = VTX + (NB / 32) * 2 * P * 64;      // A: [block a][part][lane]
    static constexpr int HDR = TT + 2 * P * 64;                  // A: {1 / V scale, 1 / T scale}
    static constexpr int ASIZE = (HDR + 1 + 7) / 8 * 8;
    static constexpr int VW = ASIZE;                             // B: [row block][part][lane]
    static constexpr int BSIZE = (NB / 16) * P * 64;
    static constexpr int SIZE = VW + BSIZE;
};

// Strips per tile of the LARFB / SSRFB tasks: 32 columns in FP64, the
// column-block width in the split modes.
template <int NB, int PREC>
__host__ __device__ constexpr int strips_of()
{
    return PREC == PREC_FP64 ? NB / WS : ColCfg<NB>::NSX;
}

template <int NB, int IB, int PREC>
__device__ __forceinline__ gu4 *vsplit_ptr(const MatDev &M, int k, int i, int l)
{
    using L = VsLayout<NB, Narrow<PREC>::NPART>;
    return (gu4 *)M.vsplit + (((size_t)k * M.p + i) * (NB / IB) + l) * L::SIZE;
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
__device__ __forceinline__ typename Narrow<PREC>::vec from_u4(const u4 &v)
{
    return __builtin_bit_cast(typename Narrow<PREC>::vec, v);
}

// Writes the split images of inner panel l of TS tile (i, k): V (rows 0..nb-1,
// columns 0..ib-1 of sm.P, FP64) and T (sm.Tl, row-major ib x ib), both
// complete in LDS (the caller has passed a barrier since they were formed).
// Every thread writes V vectors; wave 0 also writes T's and the header.
template <int NB, int IB, int PREC>
__device__ __forceinline__ void write_vsplit(const Smem<NB, IB> &sm, gu4 *dst)
{
    static_assert(IB == 32, "split images take ib = 32");
    using C = Cfg<NB, IB>;
    constexpr int P = Narrow<PREC>::NPART;
    using L = VsLayout<NB, P>;
    // |v| <= 1 for every reflector entry (|alpha - beta| >= |x_i|): a fixed
    // scale keeps the FP16 parts out of the subnormal range.
    constexpr double VS = PREC == PREC_FP16X2 ? 4096.0 : 1.0;
    const int tid = tidx(), lane = lane_id(), n = lane & 15, g = lane >> 4;
    // V^T X images: chunk c, block a, lane (n, g), element e = V[32c + 16(e/4) + 4g + e%4][16a + n].
    constexpr int NVTX = (NB / 32) * 2 * 64;
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
        for (int q = 0; q < P; ++q) dst[L::VTX + (ca * P + q) * 64 + ln] = as_u4<PREC>(Pt.p[q]);
    }
    // V W images: row block rb, lane (n, g), element e = V[16 rb + n][16(e/4) + 4g + e%4].
    constexpr int NVW = (NB / 16) * 64;
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
        for (int q = 0; q < P; ++q) dst[L::VW + (rb * P + q) * 64 + ln] = as_u4<PREC>(Pt.p[q]);
    }
    if (wave_id() == 0) {
        // T images for T^T W: block a, element e = T[16(e/4) + 4g + e%4][16a + n],
        // T scaled by a power of two from its largest entry.
        double mx = 0.0;
#pragma unroll
        for (int u = 0; u < IB * IB / 64; ++u) mx = fmax(mx, fabs(sm.Tl[lane + 64 * u]));
        mx = group_max<64>(mx);
        double ts, tinv;
        pow2_scale(mx, ts, tinv);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            double xv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) xv[e] = sm.Tl[(16 * (e >> 2) + 4 * g + (e & 3)) * IB + 16 * a + n];
            Parts<PREC> Pt;
            split8_f32<PREC>(xv, ts, Pt);
#pragma unroll
            for (int q = 0; q < P; ++q) dst[L::TT + (a * P + q) * 64 + lane] = as_u4<PREC>(Pt.p[q]);
        }
        if (lane == 0) {
            const v2d hdr = {1.0 / VS, tinv};
            dst[L::HDR] = __builtin_bit_cast(u4, hdr);
        }
    }
}

// Column scale of a wave's 16-column block: the largest |value| of the
// lane's own entries and of the three other lanes of its column.
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

// Staging of COUNT vectors of a panel's images: global -> registers (every
// thread the same number of loads, indexes clamped) and registers -> LDS.
template <int NB, int COUNT>
struct VsStage {
    static constexpr int NT = 2 * NB;
    static constexpr int SPT = (COUNT + NT - 1) / NT;
    u4 v[SPT];
};

template <int NB, int COUNT>
__device__ __forceinline__ void vs_load(VsStage<NB, COUNT> &S, const gu4 *src)
{
#pragma unroll
    for (int u = 0; u < VsStage<NB, COUNT>::SPT; ++u) {
        const int e = tidx() + u * VsStage<NB, COUNT>::NT;
        S.v[u] = src[e < COUNT ? e : COUNT - 1];
    }
}

template <int NB, int COUNT>
__device__ __forceinline__ void vs_store(u4 *lv, const VsStage<NB, COUNT> &S)
{
#pragma unroll
    for (int u = 0; u < VsStage<NB, COUNT>::SPT; ++u) {
        const int e = tidx() + u * VsStage<NB, COUNT>::NT;
        if (e < COUNT) lv[e] = S.v[u];
    }
}

// DSSRFB(k, i, j, s) in a split precision: strip s (ColCfg::WSX columns) of
// [A_kj; A_ij] <- Q_ik^T [A_kj; A_ij], with the split images of V_ik and T_ik
// that the TSQRT(k, i) panels wrote.
template <int NB, int IB, int PREC>
__device__ __forceinline__ void task_ssrfb_cols(Smem<NB, IB> &sm, const MatDev &M, int k, int i, int j, int s)
{
    using C = ColCfg<NB>;
    constexpr int P = Narrow<PREC>::NPART;
    constexpr int NPAN = NB / IB;
    using L = VsLayout<NB, P>;
    static_assert(IB == 32, "split images take ib = 32");
    static_assert(L::SIZE * 16 + (C::RH == 2 ? C::NW * 8 * 64 * 8 : 0) <= (int)sizeof(Smem<NB, IB>),
                  "panel images and the exchange slots fit in the workgroup's LDS");
    const int w = wave_id(), lane = lane_id(), n = lane & 15, g = lane >> 4;
    const int cb = w % C::NCB, h = w / C::NCB;
    const int col = s * C::WSX + 16 * cb + n;
    const int row0 = h * C::RPW;
    gdouble *X = tile_ptr(M, NB, i, j);
    gdouble *top = tile_ptr(M, NB, k, j);
    const gu4 *vs0 = vsplit_ptr<NB, IB, PREC>(M, k, i, 0);
    u4 *lv = reinterpret_cast<u4 *>(&sm);
    double *slots = reinterpret_cast<double *>(lv + L::SIZE);

    double x[C::RBW][4];
#pragma unroll
    for (int rb = 0; rb < C::RBW; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[rb][r] = X[(size_t)(row0 + 16 * rb + 4 * g + r) * NB + col];
    double tv[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) tv[a][r] = top[(size_t)(16 * a + 4 * g + r) * NB + col];
    // Region A of a panel is staged once every wave has read the previous
    // panel's (after T^T W), region B once every wave is done with V W; the
    // register copies of the two are never live at the same time.
    VsStage<NB, L::ASIZE> SA;
    VsStage<NB, L::BSIZE> SB;
    vs_load<NB, L::ASIZE>(SA, vs0);
    vs_load<NB, L::BSIZE>(SB, vs0 + L::VW);
    vs_store<NB, L::ASIZE>(lv, SA);
    vs_store<NB, L::BSIZE>(lv + L::VW, SB);
    vs_load<NB, L::ASIZE>(SA, vs0 + (NPAN > 1 ? 1 : 0) * L::SIZE);
    __syncthreads();

#pragma unroll 1
    for (int l = 0; l < NPAN; ++l) {
        const v2d hdr = __builtin_bit_cast(v2d, lv[L::HDR]);
        const double vinv = hdr.x, tinv = hdr.y;
        // W = V_l^T X over this wave's rows, FP32 per 32-row chunk, FP64 across.
        double xs, xinv;
        pow2_scale(column_max<C::RBW * 4>(&x[0][0]), xs, xinv);
        const double ux = xinv * vinv;
        double W[2][4] = {};
#pragma unroll
        for (int cc = 0; cc < C::CHW; ++cc) {
            const int c = h * C::CHW + cc;
            double xv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) xv[e] = x[2 * cc + (e >> 2)][e & 3];
            Parts<PREC> Bx;
            split8_f32<PREC>(xv, xs, Bx);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                Parts<PREC> Av;
#pragma unroll
                for (int q = 0; q < P; ++q) Av.p[q] = from_u4<PREC>(lv[L::VTX + ((c * 2 + a) * P + q) * 64 + lane]);
                const f4 d = split_product<PREC>(Av, Bx);
#pragma unroll
                for (int r = 0; r < 4; ++r) W[a][r] += (double)d[r] * ux;
            }
        }
        // The two row halves' partial sums, added in the same order by both.
        if constexpr (C::RH == 2) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) slots[(w * 8 + 4 * a + r) * 64 + lane] = W[a][r];
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    W[a][r] = slots[(cb * 8 + 4 * a + r) * 64 + lane] + slots[((cb + C::NCB) * 8 + 4 * a + r) * 64 + lane];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) W[a][r] = tv[a][r] + W[a][r];
        // W' = T_l^T W.
        double ws, winv;
        pow2_scale(column_max<8>(&W[0][0]), ws, winv);
        double Wp[2][4];
        {
            double wv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) wv[e] = W[e >> 2][e & 3];
            Parts<PREC> Bw;
            split8_f32<PREC>(wv, ws, Bw);
            const double ut = winv * tinv;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                Parts<PREC> At;
#pragma unroll
                for (int q = 0; q < P; ++q) At.p[q] = from_u4<PREC>(lv[L::TT + (a * P + q) * 64 + lane]);
                const f4 d = split_product<PREC>(At, Bw);
#pragma unroll
                for (int r = 0; r < 4; ++r) Wp[a][r] = (double)d[r] * ut;
            }
        }
        // Every wave has read region A of this panel: stage the next one's
        // (after the last panel a repeat of its own, so that every iteration
        // issues the same loads) and prefetch the next region B.
        __syncthreads();
        const int l1 = l + 1 < NPAN ? l + 1 : l;
        vs_store<NB, L::ASIZE>(lv, SA);
        vs_load<NB, L::BSIZE>(SB, vs0 + (size_t)l1 * L::SIZE + L::VW);
        // The coupled rows of A_kj: each row half writes one 16-row block.
#pragma unroll
        for (int a = 0; a < 2; ++a)
            if (C::RH == 1 || a == h)
#pragma unroll
                for (int r = 0; r < 4; ++r) top[(size_t)(32 * l + 16 * a + 4 * g + r) * NB + col] = tv[a][r] - Wp[a][r];
        // The next panel's coupled rows (a reload of these after the last).
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) tv[a][r] = top[(size_t)(32 * l1 + 16 * a + 4 * g + r) * NB + col];
        // X -= V_l W'.
        {
            double ws2, winv2;
            pow2_scale(column_max<8>(&Wp[0][0]), ws2, winv2);
            double wv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) wv[e] = Wp[e >> 2][e & 3];
            Parts<PREC> Bw;
            split8_f32<PREC>(wv, ws2, Bw);
            const double uw = winv2 * vinv;
#pragma unroll
            for (int rbw = 0; rbw < C::RBW; ++rbw) {
                const int rb = h * C::RBW + rbw;
                Parts<PREC> Av;
#pragma unroll
                for (int q = 0; q < P; ++q) Av.p[q] = from_u4<PREC>(lv[L::VW + (rb * P + q) * 64 + lane]);
                const f4 d = split_product<PREC>(Av, Bw);
#pragma unroll
                for (int r = 0; r < 4; ++r) x[rbw][r] = x[rbw][r] - (double)d[r] * uw;
            }
        }
        // Region B of the next panel once every wave is done with V W, then
        // the prefetch of region A of the one after.
        __syncthreads();
        vs_store<NB, L::BSIZE>(lv + L::VW, SB);
        const int l2 = l + 2 < NPAN ? l + 2 : NPAN - 1;
        vs_load<NB, L::ASIZE>(SA, vs0 + (size_t)l2 * L::SIZE);
        __syncthreads();
    }
#pragma unroll
    for (int rb = 0; rb < C::RBW; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) X[(size_t)(row0 + 16 * rb + 4 * g + r) * NB + col] = x[rb][r];
}

}  // namespace tq
