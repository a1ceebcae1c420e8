// Stages of the paper's own network (Sec. 3.5): per level one 3x3 conv and
// one 1x1 conv (each + ReLU), average pooling, skip merged by a sum, no
// level-0 skip, a 1x1 output conv and a sigmoid.
//
// One kernel per stage: halo tile -> LDS (with the sum skip
// up(y_{l+1}) + x_l formed in the prologue), the 3x3 as MFMA implicit GEMM
// (as in conv_kernels.h), then the 1x1 as a second MFMA GEMM taken straight
// from the accumulator registers: a 16x16 accumulator holds, per lane, four
// consecutive output channels of one pixel, which is exactly the B-operand
// layout of v_mfma_f32_16x16x16_{bf16,f16} (K = 16 channels per MFMA), and
// per-element for v_mfma_f32_16x16x4_f32.  Nothing of the 3x3 output
// touches memory.  Epilogues: store; 2x2 average pool (with or without the
// full-resolution skip store); the output 1x1 + sigmoid; the output 1x1 to
// four channels of the space-to-depth form (Sec. 3.5), whose depth-to-space
// head k_d2s_out then forms the full-resolution visibility.  The first
// encoder stage of that form reads its input through space-to-depth in the
// halo load, so the rearranged input never exists in memory.
#include <hip/hip_runtime.h>

#include "conv_kernels.h"
#include "conv_up.h"

namespace nsm {
namespace {
using namespace ck;

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

template <Dt D>
__device__ __forceinline__ f32x4 mfma_1x1(const uint2& wa, const f32x4& act, f32x4 acc) {
    using T = typename DT<D>::T;
    if constexpr (D == Dt::F32) {
        (void)wa;
        return acc;   // float32 path handled per element by the caller
    } else {
        T b4[4] = {from_f<T>(act[0]), from_f<T>(act[1]), from_f<T>(act[2]), from_f<T>(act[3])};
        if constexpr (D == Dt::BF16 || D == Dt::F8) {
            bf16x4 a, b;
            __builtin_memcpy(&a, &wa, 8);
            __builtin_memcpy(&b, b4, 8);
            return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        } else {
            f16x4 a, b;
            __builtin_memcpy(&a, &wa, 8);
            __builtin_memcpy(&b, b4, 8);
            return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, acc, 0, 0, 0);
        }
    }
}

// LDS elements of one stage tile: the halo tile's block-major planes, then
// the low-resolution rows (16-byte aligned).
template <Dt D, int CS, int CU, bool SUM, int C1, int TH>
struct PTile {
    using G = Geo<D, CS, (SUM ? 0 : CU), C1>;
    static constexpr int PS = plane_stride<D>((TH + 2) * (kTW + 2));
    static constexpr int LOW_OFF = (G::BPT * PS + 7) / 8 * 8;
    static constexpr int ELEMS = LOW_OFF + LowTile<D, CU, TH>::SIZE;
};

// One TH x 32 output tile at (x0, y0) of image n: the whole stage for it.
template <Dt D, bool IN_F32, int CS, int CU, bool SUM, int C1, int C2, PMode MODE, int TH, bool S2D>
__device__ __forceinline__ void pconv_tile(const PConvArgs& a, int x0, int y0, int n, typename DT<D>::T* tile,
                                           typename DT<D>::T* lowt) {
    using T = typename DT<D>::T;
    using G = Geo<D, CS, (SUM ? 0 : CU), C1>;
    constexpr int EPB = G::EPB, NKG = G::NKG, NF = G::NF, BPT = G::BPT, NB = G::NB;
    constexpr int NF2 = (C2 + 15) / 16;
    constexpr int WP = kTW + 2, NPIX = (TH + 2) * WP;
    constexpr int PS = plane_stride<D>(NPIX);       // block-major LDS planes
    constexpr int RPW = TH / 4, MF = RPW * 2;
    constexpr bool POOL = MODE == PMode::PoolOnly || MODE == PMode::PoolSkip;
    static_assert(!POOL || RPW % 2 == 0, "pooling needs whole row pairs per wave");
    static_assert(C1 % 16 == 0, "the 1x1 reads whole 16-channel fragments");

    const int h = a.h, w = a.w;
    load_halo_tile<D, IN_F32, CS, CU, EPB, PS, TH, SUM, S2D>(tile, lowt, a.in, a.low, n, h, w, x0, y0);

    // the wave index is uniform in the wave: keep it in a scalar register
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int px = lane & 15, g = lane >> 4;
    const u32x4* wpk = reinterpret_cast<const u32x4*>(a.wpk);
    f32x4 acc[MF][NF];
#pragma unroll
    for (int m = 0; m < MF; ++m)
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[m][f] = f32x4{0.f, 0.f, 0.f, 0.f};
    // weight fragments are fetched PD k-groups ahead of their MFMAs
    constexpr int PD = NF <= 2 ? 2 : 1;
    u32x4 wbuf[PD + 1][NF];
    auto wload = [&](int q, u32x4 (&dst)[NF]) {
#pragma unroll
        for (int f = 0; f < NF; ++f) dst[f] = wpk[(f * NKG + q) * 64 + lane];
    };
#pragma unroll
    for (int q = 0; q < PD && q < NKG; ++q) wload(q, wbuf[q]);
#pragma unroll
    for (int q = 0; q < NKG; ++q) {
        if (q + PD < NKG) wload(q + PD, wbuf[(q + PD) % (PD + 1)]);
        const u32x4 (&wf)[NF] = wbuf[q % (PD + 1)];
        int b = 4 * q + g;
        if (b >= NB) b = NB - 1;
        const int tap = b / BPT, cb = b - tap * BPT;
        const int ky = tap / 3, kx = tap - ky * 3;
        const int base = cb * PS + (ky * WP + kx + px) * EPB;
#pragma unroll
        for (int m = 0; m < MF; ++m) {
            const int r = wave * RPW + (m >> 1), cf = m & 1;
            const u32x4 xb = *reinterpret_cast<const u32x4*>(&tile[base + (r * WP + cf * 16) * EPB]);
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[m][f] = mfma_kgroup<D>(wf[f], xb, acc[m][f]);
        }
    }
    // 3x3 bias + ReLU
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        float bb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) bb[e] = a.b1[f * 16 + 4 * g + e];
#pragma unroll
        for (int m = 0; m < MF; ++m)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[m][f][e] = fmaxf(acc[m][f][e] + bb[e], 0.0f);
    }
    // 1x1 on the accumulators: acc2[co2][px] = sum_co1 W1[co2][co1] * acc[co1][px]
    f32x4 acc2[MF][NF2];
#pragma unroll
    for (int m = 0; m < MF; ++m)
#pragma unroll
        for (int f2 = 0; f2 < NF2; ++f2) acc2[m][f2] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int f2 = 0; f2 < NF2; ++f2) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if constexpr (D == Dt::F32) {
                const f32x4 w4 = reinterpret_cast<const f32x4*>(a.w1pk)[(f2 * NF + f) * 64 + lane];
#pragma unroll
                for (int m = 0; m < MF; ++m)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc2[m][f2] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4[e], acc[m][f][e], acc2[m][f2], 0, 0, 0);
            } else {
                const uint2 w4 = reinterpret_cast<const uint2*>(a.w1pk)[(f2 * NF + f) * 64 + lane];
#pragma unroll
                for (int m = 0; m < MF; ++m) acc2[m][f2] = mfma_1x1<D>(w4, acc[m][f], acc2[m][f2]);
            }
        }
    }
#pragma unroll
    for (int f2 = 0; f2 < NF2; ++f2) {
        float bb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = f2 * 16 + 4 * g + e;
            bb[e] = co < C2 ? a.b2[co] : 0.0f;
        }
#pragma unroll
        for (int m = 0; m < MF; ++m)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc2[m][f2][e] = fmaxf(acc2[m][f2][e] + bb[e], 0.0f);
    }

    if constexpr (MODE == PMode::Head) {
        float hw[NF2][4];
#pragma unroll
        for (int f2 = 0; f2 < NF2; ++f2)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = f2 * 16 + 4 * g + e;
                hw[f2][e] = co < C2 ? a.head_w[co] : 0.0f;
            }
        const float hb = a.head_w[C2];
#pragma unroll
        for (int m = 0; m < MF; ++m) {
            const int y = y0 + wave * RPW + (m >> 1), x = x0 + (m & 1) * 16 + px;
            float s = 0.0f;
#pragma unroll
            for (int f2 = 0; f2 < NF2; ++f2)
#pragma unroll
                for (int e = 0; e < 4; ++e) s += hw[f2][e] * acc2[m][f2][e];
            s = sum_rows4(s);
            if (y < h && x < w && g == 0) {
                const size_t p = ((size_t)n * h + y) * w + x;
                const float logit = s + hb;
                a.vis[p] = 1.0f / (1.0f + __expf(-logit));
                if (a.logits) a.logits[p] = logit;
            }
        }
    } else if constexpr (MODE == PMode::D2S) {
        // out4[p][k] = sum_co W[k][co] y[p][co] + b[k]: per-lane partial sums over
        // this lane's channels, summed over the four lane groups; group g stores k = g
        float hw[4][NF2][4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int f2 = 0; f2 < NF2; ++f2)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int co = f2 * 16 + 4 * g + e;
                    hw[k][f2][e] = co < C2 ? a.head_w[k * C2 + co] : 0.0f;
                }
        const float hb = a.head_w[4 * C2 + g];
        float* out4 = reinterpret_cast<float*>(a.out);
#pragma unroll
        for (int m = 0; m < MF; ++m) {
            const int y = y0 + wave * RPW + (m >> 1), x = x0 + (m & 1) * 16 + px;
            float s[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float t = 0.0f;
#pragma unroll
                for (int f2 = 0; f2 < NF2; ++f2)
#pragma unroll
                    for (int e = 0; e < 4; ++e) t += hw[k][f2][e] * acc2[m][f2][e];
                t = sum_rows4(t);
                s[k] = t;
            }
            const float mine = g == 0 ? s[0] : (g == 1 ? s[1] : (g == 2 ? s[2] : s[3]));
            if (y < h && x < w) out4[(((size_t)n * h + y) * w + x) * 4 + g] = mine + hb;
        }
    } else {
        using S = typename ST<D>::S;
        if constexpr (MODE != PMode::PoolOnly) {
            S* out = reinterpret_cast<S*>(a.out);
#pragma unroll
            for (int m = 0; m < MF; ++m) {
                const int y = y0 + wave * RPW + (m >> 1), x = x0 + (m & 1) * 16 + px;
                if (y < h && x < w) {
                    const size_t p = ((size_t)n * h + y) * w + x;
#pragma unroll
                    for (int f2 = 0; f2 < NF2; ++f2) {
                        const int co = f2 * 16 + 4 * g;
                        if (co < C2) {
                            float v4[4] = {acc2[m][f2][0], acc2[m][f2][1], acc2[m][f2][2], acc2[m][f2][3]};
                            store4<S, C2>(out + p * C2 + co, co, v4);
                        }
                    }
                }
            }
        }
        if constexpr (POOL) {
            S* pooled = reinterpret_cast<S*>(a.pooled);
            const int hp = h >> 1, wp = w >> 1;
            // row pair pr of this wave = fragments 4 pr + cf (upper row) and 4 pr + 2 + cf
#pragma unroll
            for (int pr = 0; pr < RPW / 2; ++pr)
#pragma unroll
            for (int cf = 0; cf < 2; ++cf) {
                const int yp = (y0 >> 1) + wave * (RPW / 2) + pr, xp = ((x0 + cf * 16 + px) >> 1);
#pragma unroll
                for (int f2 = 0; f2 < NF2; ++f2) {
                    float av[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float v = acc2[4 * pr + cf][f2][e] + acc2[4 * pr + 2 + cf][f2][e];
                        av[e] = (v + __shfl_xor(v, 1)) * 0.25f;
                    }
                    const int co = f2 * 16 + 4 * g;
                    if ((px & 1) == 0 && yp < hp && xp < wp && co < C2) {
                        const size_t p = ((size_t)n * hp + yp) * wp + xp;
                        store4<S, C2>(pooled + p * C2 + co, co, av);
                    }
                }
            }
        }
    }
}

template <Dt D, bool IN_F32, int CS, int CU, bool SUM, int C1, int C2, PMode MODE, int TH, bool S2D>
__global__ void __launch_bounds__(kThreads) k_pconv(PConvArgs a) {
    using T = typename DT<D>::T;
    using PT = PTile<D, CS, CU, SUM, C1, TH>;
    __shared__ __attribute__((aligned(16))) T smem[PT::ELEMS];
    const int gx = gridDim.x, gy = gridDim.y;
    const int lt = xcd_remap(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    const int x0 = (lt % gx) * kTW, y0 = ((lt / gx) % gy) * TH, n = lt / (gx * gy);
    pconv_tile<D, IN_F32, CS, CU, SUM, C1, C2, MODE, TH, S2D>(a, x0, y0, n, smem, smem + PT::LOW_OFF);
}

// The full-resolution stage (input up(y_1) alone, 3x3 CU -> C1, 1x1 C1 -> C2,
// output 1x1 + sigmoid) with the bilinear x2 upsampling folded into four
// phase kernels over the low-resolution tile, as in the U-Net decoders
// (conv_up.h: same packing, same tile).  One launch: blocks [0, nb) take
// the border tiles (TH_G rows, the stage's general form, where the zero
// padding of up() applies), the rest the interior TH x 32 tiles.
template <Dt D, int CU, int C1, int TH, int TH_G>
struct PUp0 {
    using T = typename DT<D>::T;
    using G = UpGeo<D, 0, CU, C1>;
    using UT = UpTile<D, 0, CU, TH>;
    using PT = PTile<D, 0, CU, false, C1, TH_G>;
    static constexpr int ELEMS = UT::LOW > PT::ELEMS ? UT::LOW : PT::ELEMS;
};

template <Dt D, int CU, int C1, int C2, int TH, int TH_G>
__global__ void __launch_bounds__(kThreads) k_pconv_up0(PConvArgs a, const void* __restrict__ wup) {
    using T = typename DT<D>::T;
    using P = PUp0<D, CU, C1, TH, TH_G>;
    using G = typename P::G;
    using UT = typename P::UT;
    using PT = typename P::PT;
    constexpr int EPB = G::EPB, NF = G::NF, LPS = UT::LPS, RW = TH / 4;
    constexpr int NF2 = (C2 + 15) / 16;
    static_assert(TH % 8 == 0 && TH % TH_G == 0, "each wave needs rows of one parity in one half of the tile");
    __shared__ __attribute__((aligned(16))) T smem[P::ELEMS];
    const int h = a.h, w = a.w, hl = h >> 1, wl = w >> 1;
    const int nb = border_tiles_per_image(TH, TH_G, h, w) * a.n;
    const int b = blockIdx.x;
    if (b < nb) {
        int bx, by, bn;
        border_tile(b, TH, TH_G, h, w, &bx, &by, &bn);
        pconv_tile<D, false, 0, CU, false, C1, C2, PMode::Head, TH_G, false>(a, bx, by, bn, smem,
                                                                              smem + PT::LOW_OFF);
        return;
    }
    const int gx = (w + kTW - 1) / kTW - 2, gy = (h + TH - 1) / TH - 2;
    const int lt = xcd_remap(b - nb, gx * gy * a.n);
    const int x0 = (lt % gx + 1) * kTW, y0 = ((lt / gx) % gy + 1) * TH, n = lt / (gx * gy);
    T* lowt = smem;
    // low-resolution rows y0/2-1 .. y0/2+TH/2 and columns x0/2-1 .. x0/2+16 (in the image)
    {
        using S = typename ST<D>::S;
        constexpr int KL = UT::LC * G::BPT_U, BB = blk_bytes<D>();
        const S* lbase = reinterpret_cast<const S*>(a.low) + (((size_t)n * hl + (y0 >> 1) - 1) * wl + (x0 >> 1) - 1) * CU;
        const __amdgpu_buffer_rsrc_t lr = buf_rsrc(lbase);
        const int lrow = wl * CU * (int)sizeof(S);
        copy_rows1<UT::LR, KL>(
            [&](int r, int k) -> u32x4 {
                const int cb = k / UT::LC, c = k - cb * UT::LC;
                return load_blk<D>(lr, r * lrow + (c * G::BPT_U + cb) * BB, 0);
            },
            [&](int r, int k, const u32x4& v) {
                const int cb = k / UT::LC, c = k - cb * UT::LC;
                *reinterpret_cast<u32x4*>(&lowt[cb * LPS + (r * UT::LC + c) * EPB]) = v;
            },
            threadIdx.x);
    }
    __syncthreads();

    // waves: row parity py = wave & 1, rows RW * half .. of that parity; each
    // row is two 16-pixel fragments, the even and the odd columns
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int j = lane & 15, g = lane >> 4;
    const int py = wave & 1, half = wave >> 1, rb = RW * half;
    f32x4 acc[RW][2][NF];
#pragma unroll
    for (int m = 0; m < RW; ++m)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[m][p][f] = f32x4{0.f, 0.f, 0.f, 0.f};
    const __amdgpu_buffer_rsrc_t wr = buf_rsrc(wup);
    const int wl16 = lane * 16;
    const int wph = py * 2 * NF * G::NKG_U * 1024;        // this wave's row phase
#pragma unroll
    for (int q = 0; q < G::NKG_U; ++q) {
        u32x4 w0[NF], w1[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            w0[f] = buf_load16(wr, wl16, wph + (f * G::NKG_U + q) * 1024);
            w1[f] = buf_load16(wr, wl16, wph + ((NF + f) * G::NKG_U + q) * 1024);
        }
        int bk = 4 * q + g;
        if (bk >= G::NB_U) bk = G::NB_U - 1;
        const int t = bk / G::BPT_U, cb = bk - t * G::BPT_U;
        const int ty = t / 3, tx = t - ty * 3;
#pragma unroll
        for (int m = 0; m < RW; ++m) {
            const int r = rb + m + ty;
            const u32x4 xb = *reinterpret_cast<const u32x4*>(&lowt[cb * LPS + (r * UT::LC + j + tx) * EPB]);
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                acc[m][0][f] = mfma_kgroup<D>(w0[f], xb, acc[m][0][f]);
                acc[m][1][f] = mfma_kgroup<D>(w1[f], xb, acc[m][1][f]);
            }
        }
    }
    // 3x3 bias + ReLU, then the 1x1 on the accumulators, bias + ReLU
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        float bb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) bb[e] = a.b1[f * 16 + 4 * g + e];
#pragma unroll
        for (int m = 0; m < RW; ++m)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[m][p][f][e] = fmaxf(acc[m][p][f][e] + bb[e], 0.0f);
    }
    f32x4 acc2[RW][2][NF2];
#pragma unroll
    for (int m = 0; m < RW; ++m)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int f2 = 0; f2 < NF2; ++f2) acc2[m][p][f2] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int f2 = 0; f2 < NF2; ++f2) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if constexpr (D == Dt::F32) {
                const f32x4 w4 = reinterpret_cast<const f32x4*>(a.w1pk)[(f2 * NF + f) * 64 + lane];
#pragma unroll
                for (int m = 0; m < RW; ++m)
#pragma unroll
                    for (int p = 0; p < 2; ++p)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc2[m][p][f2] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(w4[e], acc[m][p][f][e], acc2[m][p][f2], 0, 0, 0);
            } else {
                const uint2 w4 = reinterpret_cast<const uint2*>(a.w1pk)[(f2 * NF + f) * 64 + lane];
#pragma unroll
                for (int m = 0; m < RW; ++m)
#pragma unroll
                    for (int p = 0; p < 2; ++p) acc2[m][p][f2] = mfma_1x1<D>(w4, acc[m][p][f], acc2[m][p][f2]);
            }
        }
    }
    float hw[NF2][4];
#pragma unroll
    for (int f2 = 0; f2 < NF2; ++f2) {
        float bb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = f2 * 16 + 4 * g + e;
            bb[e] = co < C2 ? a.b2[co] : 0.0f;
            hw[f2][e] = co < C2 ? a.head_w[co] : 0.0f;
        }
#pragma unroll
        for (int m = 0; m < RW; ++m)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc2[m][p][f2][e] = fmaxf(acc2[m][p][f2][e] + bb[e], 0.0f);
    }
    // output 1x1 + sigmoid: logit of pixel (row m, column 2j + p), complete in
    // every lane group after the cross-group sum; lane group g writes rows
    // m with m % 4 == g, two adjacent pixels per 8-byte store
    const float hb = a.head_w[C2];
    float s[RW][2];
#pragma unroll
    for (int m = 0; m < RW; ++m)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            float v = 0.0f;
#pragma unroll
            for (int f2 = 0; f2 < NF2; ++f2)
#pragma unroll
                for (int e = 0; e < 4; ++e) v += hw[f2][e] * acc2[m][p][f2][e];
            s[m][p] = sum_rows4(v) + hb;
        }
#pragma unroll
    for (int m0 = 0; m0 < RW; m0 += 4) {
        if (m0 + g < RW) {
            float l0 = s[m0][0], l1 = s[m0][1];
#pragma unroll
            for (int k = 1; k < 4; ++k)
                if (m0 + k < RW && g == k) { l0 = s[m0 + k][0]; l1 = s[m0 + k][1]; }
            const int y = y0 + py + 2 * (rb + m0 + g), x = x0 + 2 * j;
            const size_t pi = ((size_t)n * h + y) * w + x;
            *reinterpret_cast<float2*>(a.vis + pi) =
                make_float2(1.0f / (1.0f + __expf(-l0)), 1.0f / (1.0f + __expf(-l1)));
            if (a.logits) *reinterpret_cast<float2*>(a.logits + pi) = make_float2(l0, l1);
        }
    }
}

// Channel-split form of a wide stored stage (the 5-level network's
// bottleneck, 3x3 to 256 channels and 1x1 back to 128, at 1/16 of the image
// size: 64 x 128 pixels at 1024 x 2048).  The row-per-wave kernel above would
// run there as 64 blocks of one wave per CU.  Here a block is one row of 32
// pixels and its four waves split the 3x3's output channels: wave w computes
// fragments [w NF/4, (w+1) NF/4) of the 3x3 for both 16-pixel halves, applies
// bias and ReLU, and multiplies its channel slice by the matching columns of
// the 1x1.  The four partial 1x1 sums meet in LDS (the halo tile's memory,
// reused) and each wave finishes a quarter of the 1x1 outputs, adding the
// partials in a fixed order: 256 blocks at 64 x 128 pixels.
//
// Decoder stages with a summed skip (input = skip + bilinear x2 of the
// low-resolution tensor) use the same split with two-row tiles (CU > 0,
// SUM): the low-resolution rows of a one-row tile would not cover its halo.
// With MODE = PoolSkip (two-row tiles) the stage also writes the 2x2 average
// of its output, one pooled row per tile.
template <Dt D, int CS, int CU, bool SUM, int C1, int C2, int TH, PMode MODE = PMode::Store>
__global__ void __launch_bounds__(kThreads) k_pconv_cs(PConvArgs a) {
    using T = typename DT<D>::T;
    using S = typename ST<D>::S;
    using G = Geo<D, CS, (SUM ? 0 : CU), C1>;
    static_assert(CU == 0 || (SUM && CU == CS && TH % 2 == 0), "summed decoder stages use even tile rows");
    static_assert(MODE == PMode::Store || (MODE == PMode::PoolSkip && TH == 2), "pooling takes two-row tiles");
    constexpr int MF = 2 * TH;
    constexpr int EPB = G::EPB, NKG = G::NKG, NF = G::NF, BPT = G::BPT, NB = G::NB;
    constexpr int NFW = NF / 4, NF2 = C2 / 16, N2W = NF2 / 4;
    static_assert(NF % 4 == 0 && C2 % 64 == 0, "four waves split whole fragments");
    constexpr int WP = kTW + 2, NPIX = (TH + 2) * WP;
    constexpr int PS = plane_stride<D>(NPIX);
    constexpr int TILE_BYTES = BPT * PS * (int)sizeof(T);
    constexpr int RED_BYTES = 4 * MF * NF2 * 64 * 16;
    constexpr int SMEM = TILE_BYTES > RED_BYTES ? TILE_BYTES : RED_BYTES;
    __shared__ __attribute__((aligned(16))) unsigned char smem[SMEM];
    __shared__ __attribute__((aligned(16))) T lowt[LowTile<D, CU, TH>::SIZE];
    T* tile = reinterpret_cast<T*>(smem);

    const int h = a.h, w = a.w;
    const int gx = gridDim.x, gy = gridDim.y;
    const int lt = xcd_remap(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    const int x0 = (lt % gx) * kTW, y0 = ((lt / gx) % gy) * TH, n = lt / (gx * gy);
    load_halo_tile<D, false, CS, CU, EPB, PS, TH, SUM>(tile, lowt, a.in, a.low, n, h, w, x0, y0);

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int px = lane & 15, g = lane >> 4;
    const u32x4* wpk = reinterpret_cast<const u32x4*>(a.wpk);
    f32x4 acc[MF][NFW];
#pragma unroll
    for (int m = 0; m < MF; ++m)
#pragma unroll
        for (int f = 0; f < NFW; ++f) acc[m][f] = f32x4{0.f, 0.f, 0.f, 0.f};
    // one block per CU leaves no other wave to cover the weight loads: fetch
    // the fragments PD k-groups ahead of their MFMAs
    constexpr int PD = 4;
    u32x4 wbuf[PD + 1][NFW];
    auto wload = [&](int q, u32x4 (&dst)[NFW]) {
#pragma unroll
        for (int f = 0; f < NFW; ++f) dst[f] = wpk[((wave * NFW + f) * NKG + q) * 64 + lane];
    };
#pragma unroll
    for (int q = 0; q < PD && q < NKG; ++q) wload(q, wbuf[q]);
#pragma unroll
    for (int q = 0; q < NKG; ++q) {
        if (q + PD < NKG) wload(q + PD, wbuf[(q + PD) % (PD + 1)]);
        const u32x4 (&wf)[NFW] = wbuf[q % (PD + 1)];
        int b = 4 * q + g;
        if (b >= NB) b = NB - 1;
        const int tap = b / BPT, cb = b - tap * BPT;
        const int ky = tap / 3, kx = tap - ky * 3;
        const int base = cb * PS + (ky * WP + kx + px) * EPB;
#pragma unroll
        for (int m = 0; m < MF; ++m) {
            // fragment m: row m / 2 of the tile, 16-pixel half m % 2
            const u32x4 xb = *reinterpret_cast<const u32x4*>(&tile[base + ((m >> 1) * WP + (m & 1) * 16) * EPB]);
#pragma unroll
            for (int f = 0; f < NFW; ++f) acc[m][f] = mfma_kgroup<D>(wf[f], xb, acc[m][f]);
        }
    }
#pragma unroll
    for (int f = 0; f < NFW; ++f) {
        float bb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) bb[e] = a.b1[(wave * NFW + f) * 16 + 4 * g + e];
#pragma unroll
        for (int m = 0; m < MF; ++m)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[m][f][e] = fmaxf(acc[m][f][e] + bb[e], 0.0f);
    }
    // partial 1x1 over this wave's channel slice
    f32x4 acc2[MF][NF2];
#pragma unroll
    for (int m = 0; m < MF; ++m)
#pragma unroll
        for (int f2 = 0; f2 < NF2; ++f2) acc2[m][f2] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int f2 = 0; f2 < NF2; ++f2) {
#pragma unroll
        for (int f = 0; f < NFW; ++f) {
            const int fg = wave * NFW + f;
            if constexpr (D == Dt::F32) {
                const f32x4 w4 = reinterpret_cast<const f32x4*>(a.w1pk)[(f2 * NF + fg) * 64 + lane];
#pragma unroll
                for (int m = 0; m < MF; ++m)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc2[m][f2] = __builtin_amdgcn_mfma_f32_16x16x4f32(w4[e], acc[m][f][e], acc2[m][f2], 0, 0, 0);
            } else {
                const uint2 w4 = reinterpret_cast<const uint2*>(a.w1pk)[(f2 * NF + fg) * 64 + lane];
#pragma unroll
                for (int m = 0; m < MF; ++m) acc2[m][f2] = mfma_1x1<D>(w4, acc[m][f], acc2[m][f2]);
            }
        }
    }
    // the four partials meet in LDS; wave w finishes fragments [w N2W, (w+1) N2W)
    __syncthreads();                           // every wave is done reading the tile
    f32x4* red = reinterpret_cast<f32x4*>(smem);
#pragma unroll
    for (int m = 0; m < MF; ++m)
#pragma unroll
        for (int f2 = 0; f2 < NF2; ++f2) red[((wave * MF + m) * NF2 + f2) * 64 + lane] = acc2[m][f2];
    __syncthreads();
    S* out = reinterpret_cast<S*>(a.out);
#pragma unroll
    for (int k = 0; k < N2W; ++k) {
        const int f2 = wave * N2W + k, co = f2 * 16 + 4 * g;
        float bb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) bb[e] = a.b2[co + e];
        float val[MF][4];
#pragma unroll
        for (int m = 0; m < MF; ++m) {
            f32x4 v = red[((0 * MF + m) * NF2 + f2) * 64 + lane];
#pragma unroll
            for (int wv = 1; wv < 4; ++wv) v += red[((wv * MF + m) * NF2 + f2) * 64 + lane];
#pragma unroll
            for (int e = 0; e < 4; ++e) val[m][e] = fmaxf(v[e] + bb[e], 0.0f);
            const int y = y0 + (m >> 1), x = x0 + (m & 1) * 16 + px;
            if (y < h && x < w) {
                const size_t p = ((size_t)n * h + y) * w + x;
                store4<S, C2>(out + p * C2 + co, co, val[m]);
            }
        }
        if constexpr (MODE == PMode::PoolSkip) {
            // 2x2 average: the tile's two rows, then the neighbouring column (lane ^ 1)
            S* pooled = reinterpret_cast<S*>(a.pooled);
            const int hp = h >> 1, wp = w >> 1, yp = y0 >> 1;
#pragma unroll
            for (int cf = 0; cf < 2; ++cf) {
                const int xp = (x0 + cf * 16 + px) >> 1;
                float av[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float v = val[cf][e] + val[2 + cf][e];
                    av[e] = (v + __shfl_xor(v, 1)) * 0.25f;
                }
                if ((px & 1) == 0 && yp < hp && xp < wp) {
                    const size_t p = ((size_t)n * hp + yp) * wp + xp;
                    store4<S, C2>(pooled + p * C2 + co, co, av);
                }
            }
        }
    }
}

// Depth-to-space head of the space-to-depth form (Sec. 3.5).  One thread per
// low-resolution pixel (i, j) writes the 2x2 block (2i + dy, 2j + dx):
// logit = bilinear x2 of channel 0 (the taps of the decoder's upsampling:
// 0.25 / 0.75 towards the nearer low-res neighbour, clamped at the border,
// rows first) + channel 2 dy + dx for the three pixels other than (2i, 2j).
__global__ void __launch_bounds__(256) k_d2s_out(const float* __restrict__ y4, int n, int h, int w,
                                                  float* __restrict__ vis, float* __restrict__ logits) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)n * h * w;
    if (idx >= total) return;
    const int j = (int)(idx % w);
    const long long t = idx / w;
    const int i = (int)(t % h), f = (int)(t / h);
    const float4* img = reinterpret_cast<const float4*>(y4) + (size_t)f * h * w;
    const int im = max(i - 1, 0), ip = min(i + 1, h - 1);
    const int jm = max(j - 1, 0), jp = min(j + 1, w - 1);
    const float* c0 = reinterpret_cast<const float*>(img);
    auto ch0 = [&](int r, int c) { return c0[((size_t)r * w + c) * 4]; };
    const float4 me = img[(size_t)i * w + j];
    const int cols[3] = {jm, j, jp};
    float r0[3], r1[3];      // row-interpolated channel 0 at output rows 2i, 2i + 1
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float a = ch0(im, cols[q]), b = q == 1 ? me.x : ch0(i, cols[q]), c = ch0(ip, cols[q]);
        r0[q] = 0.25f * a + 0.75f * b;
        r1[q] = 0.75f * b + 0.25f * c;
    }
    float2 top, bot;
    top.x = 0.25f * r0[0] + 0.75f * r0[1];
    top.y = 0.75f * r0[1] + 0.25f * r0[2] + me.y;
    bot.x = 0.25f * r1[0] + 0.75f * r1[1] + me.z;
    bot.y = 0.75f * r1[1] + 0.25f * r1[2] + me.w;
    const int W = 2 * w;
    const size_t o = ((size_t)f * 2 * h + 2 * i) * W + 2 * j;
    float2 vt, vb;
    vt.x = 1.0f / (1.0f + __expf(-top.x));
    vt.y = 1.0f / (1.0f + __expf(-top.y));
    vb.x = 1.0f / (1.0f + __expf(-bot.x));
    vb.y = 1.0f / (1.0f + __expf(-bot.y));
    *reinterpret_cast<float2*>(vis + o) = vt;
    *reinterpret_cast<float2*>(vis + o + W) = vb;
    if (logits) {
        *reinterpret_cast<float2*>(logits + o) = top;
        *reinterpret_cast<float2*>(logits + o + W) = bot;
    }
}

// 1x1 weights [C2][C1] float32 -> [NF2][NF1][64 lanes][4] storage type:
// lane (co2 = l % 16, g = l / 16) element e holds W1[16 f2 + co2][16 f + 4 g + e].
template <Dt D, int C1, int C2>
__global__ void k_pack1x1(const float* __restrict__ w, void* __restrict__ out) {
    using T = typename DT<D>::T;
    constexpr int NF1 = C1 / 16, NF2 = (C2 + 15) / 16;
    constexpr int total = NF2 * NF1 * 64 * 4;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int e = idx & 3, lane = (idx >> 2) & 63, f = (idx >> 8) % NF1, f2 = (idx >> 8) / NF1;
    const int co2 = f2 * 16 + (lane & 15), co1 = f * 16 + 4 * (lane >> 4) + e;
    const float v = (co2 < C2) ? w[(size_t)co2 * C1 + co1] : 0.0f;
    reinterpret_cast<T*>(out)[idx] = from_f<T>(v);
}

// (cs, cu, sum, c1, c2, mode, float32 input, tile rows, space-to-depth input)
#define NSM_PSTAGES(X)                                        \
    X(4, 0, false, 16, 16, PoolOnly, true, 16, false)         \
    X(16, 0, false, 32, 32, PoolSkip, false, 8, false)        \
    X(16, 0, false, 32, 32, PoolSkip, true, 8, true)          \
    X(32, 0, false, 64, 64, PoolSkip, false, 8, false)        \
    X(64, 0, false, 128, 128, PoolSkip, false, 8, false)      \
    X(128, 0, false, 256, 128, Store, false, 4, false)        \
    X(32, 0, false, 64, 32, Store, false, 8, false)           \
    X(128, 128, true, 128, 64, Store, false, 4, false)        \
    X(64, 64, true, 64, 32, Store, false, 8, false)           \
    X(32, 32, true, 32, 16, Store, false, 8, false)           \
    X(32, 32, true, 32, 16, D2S, false, 8, false)             \
    X(0, 16, false, 16, 16, Head, false, 8, false)

template <Dt D> constexpr const char* pdt_suffix() {
    return D == Dt::F32 ? " f32" : (D == Dt::BF16 ? " bf16" : (D == Dt::F16 ? " f16" : " f8"));
}

#define NSM_PMATCH(CS_, CU_, SUM_, C1_, C2_, MODE_, F32_, S2D_)                                  \
    (st.cs == CS_ && st.cu == CU_ && st.sum == SUM_ && st.c1 == C1_ && st.c2 == C2_ &&          \
     st.mode == PMode::MODE_ && st.in_f32 == F32_ && st.s2d == S2D_)

template <Dt D>
bool ppack(const PStage& st, const float* w3, const float* w1, void* out, hipStream_t s, size_t* bytes,
           size_t* w1_off = nullptr, size_t* up_off = nullptr);

template <Dt D>
hipError_t plaunch(const PStage& st, const PConvArgs& a, hipStream_t s, bool* found) {
    // the 256-channel bottleneck runs in the channel-split form (same packed weights)
    if (st.cs == 128 && st.cu == 0 && !st.sum && st.c1 == 256 && st.c2 == 128 && st.mode == PMode::Store &&
        !st.in_f32 && !st.s2d) {
        *found = true;
        dim3 grid((a.w + kTW - 1) / kTW, a.h, a.n);
        TraceScope ts("pconv 128+0->256->128 Store split", pdt_suffix<D>(), s);
        k_pconv_cs<D, 128, 0, false, 256, 128, 1><<<grid, kThreads, 0, s>>>(a);
        return hipGetLastError();
    }
    // so does the level-3 decoder (128 + up 128 summed -> 128 -> 64), two rows per
    // block, in the 16-bit forms (in float32 its tile allows one block per CU,
    // and the row-tile kernel measured faster)
    if (D != Dt::F32 && st.cs == 128 && st.cu == 128 && st.sum && st.c1 == 128 && st.c2 == 64 &&
        st.mode == PMode::Store && !st.in_f32 && !st.s2d) {
        *found = true;
        dim3 grid((a.w + kTW - 1) / kTW, (a.h + 1) / 2, a.n);
        TraceScope ts("pconv 128+128->128->64 Store split", pdt_suffix<D>(), s);
        k_pconv_cs<D, 128, 128, true, 128, 64, 2><<<grid, kThreads, 0, s>>>(a);
        return hipGetLastError();
    }
    // and the level-3 encoder (64 -> 128 -> 128, pooled), two rows per block
    if (st.cs == 64 && st.cu == 0 && !st.sum && st.c1 == 128 && st.c2 == 128 && st.mode == PMode::PoolSkip &&
        !st.in_f32 && !st.s2d) {
        *found = true;
        dim3 grid((a.w + kTW - 1) / kTW, (a.h + 1) / 2, a.n);
        TraceScope ts("pconv 64+0->128->128 PoolSkip split", pdt_suffix<D>(), s);
        k_pconv_cs<D, 64, 0, false, 128, 128, 2, PMode::PoolSkip><<<grid, kThreads, 0, s>>>(a);
        return hipGetLastError();
    }
    // the full-resolution stage of up(y_1): phase form where the image has
    // interior tiles (16 rows), border tiles in its general form (8 rows)
    if (st.cs == 0 && st.cu == 16 && !st.sum && st.c1 == 16 && st.c2 == 16 && st.mode == PMode::Head &&
        !st.in_f32 && !st.s2d) {
        constexpr int THU = 16, THG = 8;
        const int gxt = (a.w + kTW - 1) / kTW, gyt = (a.h + THU - 1) / THU;
        if (gxt >= 3 && gyt >= 3) {
            *found = true;
            size_t up_off = 0;
            ppack<D>(st, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, &up_off);
            const void* wup = reinterpret_cast<const char*>(a.wpk) + up_off;
            const int blocks = border_tiles_per_image(THU, THG, a.h, a.w) * a.n + (gxt - 2) * (gyt - 2) * a.n;
            TraceScope ts("pconv 0+16->16->16 Head phase", pdt_suffix<D>(), s);
            k_pconv_up0<D, 16, 16, 16, THU, THG><<<blocks, kThreads, 0, s>>>(a, wup);
            return hipGetLastError();
        }
    }
#define NSM_PCASE(CS_, CU_, SUM_, C1_, C2_, MODE_, F32_, TH_, S2D_)                               \
    if (NSM_PMATCH(CS_, CU_, SUM_, C1_, C2_, MODE_, F32_, S2D_)) {                                \
        *found = true;                                                                            \
        if constexpr (C1_ >= 256) {     /* 256-wide stages run in the channel-split form */       \
            return hipErrorInvalidValue;                                                          \
        } else {                                                                                  \
            dim3 grid((a.w + kTW - 1) / kTW, (a.h + TH_ - 1) / TH_, a.n);                         \
            TraceScope ts(S2D_ ? "pconv s2d " #CS_ "->" #C1_ "->" #C2_ " " #MODE_                 \
                               : "pconv " #CS_ "+" #CU_ "->" #C1_ "->" #C2_ " " #MODE_,           \
                          pdt_suffix<D>(), s);                                                    \
            k_pconv<D, F32_, CS_, CU_, SUM_, C1_, C2_, PMode::MODE_, TH_, S2D_>                   \
                <<<grid, kThreads, 0, s>>>(a);                                                    \
            return hipGetLastError();                                                             \
        }                                                                                         \
    }
    NSM_PSTAGES(NSM_PCASE)
#undef NSM_PCASE
    *found = false;
    return hipErrorInvalidValue;
}

// Packed weights of a stage: the 3x3 pack, the 1x1 pack (256-byte aligned)
// and, for the full-resolution stage of up(y_1) alone, the phase-form pack
// of its 3x3 (conv_up.h, 256-byte aligned).
template <Dt D>
bool ppack(const PStage& st, const float* w3, const float* w1, void* out, hipStream_t s, size_t* bytes,
           size_t* w1_off, size_t* up_off) {
#define NSM_PPACK(CS_, CU_, SUM_, C1_, C2_, MODE_, F32_, TH_, S2D_)                               \
    if (NSM_PMATCH(CS_, CU_, SUM_, C1_, C2_, MODE_, F32_, S2D_)) {                                      \
        constexpr size_t b3 = packed_bytes<D, CS_, (SUM_ ? 0 : CU_), C1_>();                      \
        constexpr size_t b1 = (size_t)((C2_ + 15) / 16) * (C1_ / 16) * 64 * 4 * sizeof(typename DT<D>::T); \
        constexpr bool UP0 = CS_ == 0 && PMode::MODE_ == PMode::Head;                            \
        constexpr size_t o1 = (b3 + 255) & ~(size_t)255, ou = (o1 + b1 + 255) & ~(size_t)255;    \
        if (bytes) *bytes = UP0 ? ou + UpGeo<D, 0, (UP0 ? CU_ : 16), C1_>::BYTES : o1 + b1;      \
        if (w1_off) *w1_off = o1;                                                                 \
        if (up_off) *up_off = UP0 ? ou : 0;                                                       \
        if (out) {                                                                                \
            constexpr int n3 = (int)(b3 / 16 * DT<D>::EPB);                                       \
            k_pack<D, CS_, (SUM_ ? 0 : CU_), C1_><<<(n3 + 255) / 256, 256, 0, s>>>(w3, out);      \
            constexpr int n1 = (int)(b1 / sizeof(typename DT<D>::T));                             \
            k_pack1x1<D, C1_, C2_><<<(n1 + 255) / 256, 256, 0, s>>>(w1, reinterpret_cast<char*>(out) + o1); \
            if constexpr (UP0) {                                                                  \
                using GU = UpGeo<D, 0, CU_, C1_>;                                                 \
                constexpr int nu = (int)(4 * GU::PHASE_ELEMS);                                    \
                k_pack_up<D, 0, CU_, C1_><<<(nu + 255) / 256, 256, 0, s>>>(w3, reinterpret_cast<char*>(out) + ou); \
            }                                                                                     \
        }                                                                                         \
        return true;                                                                              \
    }
    NSM_PSTAGES(NSM_PPACK)
#undef NSM_PPACK
    return false;
}

}  // namespace

bool pconv_supported(const PStage& st) {
#define NSM_PSUP(CS_, CU_, SUM_, C1_, C2_, MODE_, F32_, TH_, S2D_) \
    if (NSM_PMATCH(CS_, CU_, SUM_, C1_, C2_, MODE_, F32_, S2D_)) return true;
    NSM_PSTAGES(NSM_PSUP)
#undef NSM_PSUP
    return false;
}

size_t pconv_packed_bytes(const PStage& st, Dt dt) {
    size_t b = 0;
    switch (dt) {
        case Dt::F32: ppack<Dt::F32>(st, nullptr, nullptr, nullptr, nullptr, &b); break;
        case Dt::BF16: ppack<Dt::BF16>(st, nullptr, nullptr, nullptr, nullptr, &b); break;
        case Dt::F16: ppack<Dt::F16>(st, nullptr, nullptr, nullptr, nullptr, &b); break;
        default: break;     // no 8-bit storage form of this network
    }
    return b;
}

hipError_t pconv_pack(const PStage& st, Dt dt, const float* w3, const float* w1, void* packed,
                      hipStream_t s) {
    bool ok = false;
    switch (dt) {
        case Dt::F32: ok = ppack<Dt::F32>(st, w3, w1, packed, s, nullptr); break;
        case Dt::BF16: ok = ppack<Dt::BF16>(st, w3, w1, packed, s, nullptr); break;
        case Dt::F16: ok = ppack<Dt::F16>(st, w3, w1, packed, s, nullptr); break;
        default: break;
    }
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}

size_t pconv_w1_offset(const PStage& st, Dt dt) {
    size_t o1 = 0;
    switch (dt) {
        case Dt::F32: ppack<Dt::F32>(st, nullptr, nullptr, nullptr, nullptr, nullptr, &o1); break;
        case Dt::BF16: ppack<Dt::BF16>(st, nullptr, nullptr, nullptr, nullptr, nullptr, &o1); break;
        case Dt::F16: ppack<Dt::F16>(st, nullptr, nullptr, nullptr, nullptr, nullptr, &o1); break;
        default: break;
    }
    return o1;
}

hipError_t d2s_forward(const float* y4, int n, int h, int w, float* vis, float* logits, hipStream_t s) {
    const long long total = (long long)n * h * w;
    if (total <= 0) return hipSuccess;
    TraceScope ts("d2s head", "", s);
    k_d2s_out<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(y4, n, h, w, vis, logits);
    return hipGetLastError();
}

hipError_t pconv_forward(const PStage& st, Dt dt, const PConvArgs& a, hipStream_t s) {
    bool found = false;
    hipError_t e = hipErrorInvalidValue;
    switch (dt) {
        case Dt::F32: e = plaunch<Dt::F32>(st, a, s, &found); break;
        case Dt::BF16: e = plaunch<Dt::BF16>(st, a, s, &found); break;
        case Dt::F16: e = plaunch<Dt::F16>(st, a, s, &found); break;
        default: break;
    }
    return found ? e : hipErrorInvalidValue;
}

}  // namespace nsm
