// Decoder stages with the bilinear x2 upsampling folded into the weights.
//
// A decoder stage (paper Sec. 3.5) convolves the concatenation [skip, up(low)]
// with a 3x3 kernel, where up() is bilinear x2 with half-pixel centres: row y
// of the upsampled image is 1/4 of low row (y-1)/2 and 3/4 of the next one
// for even y (the reverse for odd y), clamped to the low image.  Both maps are
// linear, so away from the image border the part of the stage that reads
// up(low) is itself a 3x3 convolution over the *low-resolution* tile, with a
// different kernel for each of the four output phases (y mod 2, x mod 2):
//
//   out(2i+py, 2j+px) = sum_{ty,tx} Wp[py][px][ty][tx] . low(i-1+ty, j-1+tx)
//   Wp[py][px][ty][tx] = sum_{ky,kx} C[py][ky][ty] C[px][kx][tx] W[ky][kx]
//
// with the 3x3 coupling tables C below (C[p][k][t] = the weight of low tap
// i-1+t in the upsampled row 2i+p+k-1).  Low taps that fall outside the low
// image are clamped when the low tile is staged, which is exactly what the
// clamped interpolation does.  What the phase form cannot express is the
// conv's zero padding of up() at rows -1 and H and columns -1 and W, so only
// tiles that stay clear of the first and last row and column use it; the
// border bands run the general kernel (conv_kernels.h).
//
// Gains on MI355X: no interpolation arithmetic at all (it was most of the
// vector ALU work of the general kernel), a low-resolution tile 4x smaller
// than the upsampled one, and every low-resolution operand read from LDS
// feeds the MFMAs of both x-phases.  The MFMA work per output pixel is
// unchanged (K = 9 * (CS + CU)).
//
// Tile: TH rows x 32 columns, 256 threads.  Wave w takes the rows of parity
// w & 1 in half w >> 1 of the tile, TH/4 rows; each row is two 16-pixel MFMA
// fragments, the even and the odd columns, so a fragment has one x-phase.
// The skip tile is stored split by column parity, so that the 16 pixels of a
// fragment (stride 2 in the image) are consecutive in LDS.  Both tiles are
// block-major (one 256-byte aligned plane per 16-byte channel block), as in
// the general kernel.
#pragma once
#include "conv_kernels.h"

namespace nsm {
namespace ck {

// C[p][k][t]: weight of low-resolution tap (i - 1 + t) in upsampled row
// 2i + p + k - 1 (rows of the 3x3 conv window k = 0, 1, 2).
__host__ __device__ constexpr double up_coupling(int p, int k, int t) {
    // upsampled row u = 2i + p + k - 1 = 2i + d, d in [-1, 2]
    // even u = 2m: 1/4 low(m-1) + 3/4 low(m); odd u = 2m+1: 3/4 low(m) + 1/4 low(m+1)
    const int d = p + k - 1;
    // d = -1: u = 2(i-1)+1 -> 3/4 low(i-1) + 1/4 low(i)
    // d =  0: u = 2i       -> 1/4 low(i-1) + 3/4 low(i)
    // d =  1: u = 2i+1     -> 3/4 low(i)   + 1/4 low(i+1)
    // d =  2: u = 2(i+1)   -> 1/4 low(i)   + 3/4 low(i+1)
    return d == -1 ? (t == 0 ? 0.75 : (t == 1 ? 0.25 : 0.0))
         : d == 0  ? (t == 0 ? 0.25 : (t == 1 ? 0.75 : 0.0))
         : d == 1  ? (t == 1 ? 0.75 : (t == 2 ? 0.25 : 0.0))
                   : (t == 1 ? 0.25 : (t == 2 ? 0.75 : 0.0));
}

template <Dt D, int CS, int CU, int CO>
struct UpGeo {
    static constexpr int EPB = DT<D>::EPB;
    static_assert(CS % EPB == 0 && CU % EPB == 0, "channels must fill whole 16-byte blocks");
    static constexpr int BPT_S = CS / EPB, BPT_U = CU / EPB;
    static constexpr int NB_S = 9 * BPT_S, NB_U = 9 * BPT_U;
    static constexpr int NKG_S = (NB_S + 3) / 4, NKG_U = (NB_U + 3) / 4;
    static constexpr int NF = (CO + 15) / 16;

    // packed weight elements: skip part, then 4 phases of the low-res part
    static constexpr size_t SKIP_ELEMS = (size_t)NF * NKG_S * 64 * EPB;
    static constexpr size_t PHASE_ELEMS = (size_t)NF * NKG_U * 64 * EPB;
    static constexpr size_t BYTES = (SKIP_ELEMS + 4 * PHASE_ELEMS) * sizeof(typename DT<D>::T);
};

// Tile geometry of the phase kernel.
template <Dt D, int CS, int CU, int TH>
struct UpTile {
    static constexpr int SR = TH + 2, SC = 17;          // skip tile: rows x (2 parity planes x 17)
    static constexpr int LR = TH / 2 + 2, LC = kTW / 2 + 2;
    static constexpr int SPS = plane_stride<D>(SR * 2 * SC), LPS = plane_stride<D>(LR * LC);
    static constexpr int SKIP = CS / DT<D>::EPB * SPS;
    static constexpr int LOW = CU / DT<D>::EPB * LPS;
};

// Pack the phase-form weights from OHWI float32 W[CO][3][3][CS+CU]:
// [NF][NKG_S][64][EPB] for the skip channels (k-block b = (tap, channel
// block) with tap = ky * 3 + kx), then for each phase py * 2 + px
// [NF][NKG_U][64][EPB] with k-block b = (low tap ty * 3 + tx, channel block).
// The phase kernels are formed in float64 and rounded once.
template <Dt D, int CS, int CU, int CO>
__global__ void k_pack_up(const float* __restrict__ w, void* __restrict__ out) {
    using T = typename DT<D>::T;
    using G = UpGeo<D, CS, CU, CO>;
    constexpr int EPB = G::EPB, CIN = CS + CU;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = G::SKIP_ELEMS + 4 * G::PHASE_ELEMS;
    if (idx >= total) return;
    const int e = (int)(idx % EPB);
    const int lane = (int)((idx / EPB) % 64);
    const int co_l = lane & 15, g = lane >> 4;
    double v = 0.0;
    bool skip_part = false;
    if constexpr (CS > 0) {       // stages of up() alone have no skip part
        if (idx < G::SKIP_ELEMS) {
            skip_part = true;
            const int q = (int)((idx / (EPB * 64)) % G::NKG_S);
            const int f = (int)(idx / ((size_t)EPB * 64 * G::NKG_S));
            const int co = f * 16 + co_l, b = 4 * q + g;
            if (b < G::NB_S && co < CO) {
                const int tap = b / G::BPT_S, cb = b % G::BPT_S;
                v = w[((size_t)co * 9 + tap) * CIN + cb * EPB + e];
            }
        }
    }
    if (!skip_part) {
        const size_t r = idx - G::SKIP_ELEMS;
        const int q = (int)((r / (EPB * 64)) % G::NKG_U);
        const int f = (int)((r / ((size_t)EPB * 64 * G::NKG_U)) % G::NF);
        const int ph = (int)(r / G::PHASE_ELEMS);
        const int py = ph >> 1, px = ph & 1;
        const int co = f * 16 + co_l, b = 4 * q + g;
        if (b < G::NB_U && co < CO) {
            const int t = b / G::BPT_U, cb = b % G::BPT_U;
            const int ty = t / 3, tx = t % 3;
            const int ch = CS + cb * EPB + e;
            for (int ky = 0; ky < 3; ++ky)
                for (int kx = 0; kx < 3; ++kx) {
                    const double c = up_coupling(py, ky, ty) * up_coupling(px, kx, tx);
                    if (c != 0.0) v += c * (double)w[((size_t)co * 9 + ky * 3 + kx) * CIN + ch];
                }
        }
    }
    reinterpret_cast<T*>(out)[idx] = from_f<T>((float)v);
}

// One launch covers the whole stage: blocks [0, nb) take the border tiles
// (the general kernel's TH_G x 32 tiles in the top and bottom bands and the
// first and last tile columns, border_tile()), the remaining blocks the
// interior TH x 32 tiles, none of whose pixels lies in the first or last row
// or column.  Border blocks come first so that their slower general path
// overlaps the phase-form blocks.  MODE is Store or Head.
template <Dt D, int CS, int CU, int CO, int TH, int TH_G>
constexpr int up_smem_elems() {
    using UT = UpTile<D, CS, CU, TH>;
    using GT = GenTile<D, CS, CU, CO, TH_G>;
    constexpr int LOW_OFF = (UT::SKIP + 7) / 8 * 8;
    return (LOW_OFF + UT::LOW) > GT::ELEMS ? (LOW_OFF + UT::LOW) : GT::ELEMS;
}

// Logical block b of a decoder stage (border tiles first, then interior).
template <Dt D, int CS, int CU, int CO, OutMode MODE, int TH, int TH_G>
__device__ __forceinline__ void up_block(const ConvArgs& a, const void* __restrict__ wup, int b,
                                         typename DT<D>::T* smem) {
    using T = typename DT<D>::T;
    using G = UpGeo<D, CS, CU, CO>;
    using UT = UpTile<D, CS, CU, TH>;
    using GT = GenTile<D, CS, CU, CO, TH_G>;
    constexpr int EPB = G::EPB, NF = G::NF, SPS = UpTile<D, CS, CU, TH>::SPS, LPS = UpTile<D, CS, CU, TH>::LPS;
    constexpr int RW = TH / 4;                  // rows per wave
    static_assert(TH % 8 == 0 && TH % TH_G == 0, "each wave needs rows of one parity in one half of the tile");
    static_assert(MODE == OutMode::Store || MODE == OutMode::Head, "decoder stages store or end in the head");
    constexpr int LOW_OFF = (UT::SKIP + 7) / 8 * 8;

    const int h = a.h, w = a.w, hl = h >> 1, wl = w >> 1;
    const int nb = border_tiles_per_image(TH, TH_G, h, w) * a.n;
    if (b < nb) {
        int bx, by, bn;
        border_tile(b, TH, TH_G, h, w, &bx, &by, &bn);
        conv_tile<D, false, CS, CU, CO, MODE, TH_G>(a, bx, by, bn, smem, smem + GT::LOW_OFF);
        return;
    }
    T* skip = smem;
    T* lowt = smem + LOW_OFF;
    const int gx = (w + kTW - 1) / kTW - 2, gy = (h + TH - 1) / TH - 2;
    const int lt = xcd_remap(b - nb, gx * gy * a.n);
    const int x0 = (lt % gx + 1) * kTW, y0 = ((lt / gx) % gy + 1) * TH, n = lt / (gx * gy);

    // ---------------- prologue: skip tile (split by column parity) and low tile
    // Interior tiles read only in-image pixels: skip rows y0-1 .. y0+TH and
    // columns x0-1 .. x0+32, low rows y0/2-1 .. y0/2+TH/2 and columns
    // x0/2-1 .. x0/2+16, all inside the image (and no clamping is needed).
    {
        using S = typename ST<D>::S;
        constexpr int KS = 34 * G::BPT_S, KL = UT::LC * G::BPT_U;   // blocks per tile row
        constexpr int BB = blk_bytes<D>();
        const S* sbase = reinterpret_cast<const S*>(a.in) + (((size_t)n * h + y0 - 1) * w + x0 - 1) * CS;
        const S* lbase = reinterpret_cast<const S*>(a.low) + (((size_t)n * hl + (y0 >> 1) - 1) * wl + (x0 >> 1) - 1) * CU;
        const __amdgpu_buffer_rsrc_t sr = buf_rsrc(sbase), lr = buf_rsrc(lbase);
        const int srow = w * CS * (int)sizeof(S), lrow = wl * CU * (int)sizeof(S);
        // chunk k = block k / (pixels per row) of pixel k % (pixels per row):
        // consecutive lanes store one block of consecutive pixels (no bank
        // conflicts), and a wave's loads still cover whole pixel runs
        auto skip_ld = [&](int r, int k) -> u32x4 {
            const int cb = k / 34, c = k - cb * 34;
            return load_blk<D>(sr, r * srow + (c * G::BPT_S + cb) * BB, 0);
        };
        auto skip_st = [&](int r, int k, const u32x4& v) {
            const int cb = k / 34, c = k - cb * 34;
            *reinterpret_cast<u32x4*>(&skip[cb * SPS + ((r * 2 + (c & 1)) * UT::SC + (c >> 1)) * EPB]) = v;
        };
        auto low_ld = [&](int r, int k) -> u32x4 {
            const int cb = k / UT::LC, c = k - cb * UT::LC;
            return load_blk<D>(lr, r * lrow + (c * G::BPT_U + cb) * BB, 0);
        };
        auto low_st = [&](int r, int k, const u32x4& v) {
            const int cb = k / UT::LC, c = k - cb * UT::LC;
            *reinterpret_cast<u32x4*>(&lowt[cb * LPS + (r * UT::LC + c) * EPB]) = v;
        };
        copy_rows2<UT::SR, KS, UT::LR, KL>(skip_ld, skip_st, low_ld, low_st, threadIdx.x);
    }
    __syncthreads();

    // ---------------- main loop
    // the wave index is uniform in the wave: keep it in a scalar register
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int j = lane & 15, g = lane >> 4;
    const int py = wave & 1, half = wave >> 1;
    // Stored stages with an even number of 16-channel fragments split the
    // output channels, not the rows, between the two waves of a row parity:
    // each wave streams half of the weights from L2 (the weight fragments,
    // not the MFMAs, fill the vector memory pipe) and reads twice the
    // activation fragments from LDS, which has the bandwidth to spare.
    constexpr bool SPLIT = MODE == OutMode::Store && NF % 2 == 0;
    constexpr int MR = SPLIT ? 2 * RW : RW;         // rows of parity py per wave
    constexpr int NFW = SPLIT ? NF / 2 : NF;        // 16-channel fragments per wave
    const int f0 = SPLIT ? half * NFW : 0;          // the wave's first fragment
    const int rb = SPLIT ? 0 : RW * half;           // the wave's first row of parity py
    f32x4 acc[MR][2][NFW];
#pragma unroll
    for (int m = 0; m < MR; ++m)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int f = 0; f < NFW; ++f) acc[m][p][f] = f32x4{0.f, 0.f, 0.f, 0.f};

    // skip channels: ordinary 3x3 taps over the full-resolution tile
    const __amdgpu_buffer_rsrc_t wr = buf_rsrc(wup);
    const int wl16 = lane * 16;
#pragma unroll
    for (int q = 0; q < G::NKG_S; ++q) {
        u32x4 wf[NFW];
#pragma unroll
        for (int f = 0; f < NFW; ++f) wf[f] = buf_load16(wr, wl16, ((f0 + f) * G::NKG_S + q) * 1024);
        int b = 4 * q + g;
        if (b >= G::NB_S) b = G::NB_S - 1;     // padding k: weights are zero there
        const int tap = b / G::BPT_S, cb = b - tap * G::BPT_S;
        const int ky = tap / 3, kx = tap - ky * 3;
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int row = py + 2 * (rb + m) + ky;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int c = p + kx;
                const u32x4 xb = *reinterpret_cast<const u32x4*>(
                    &skip[cb * SPS + ((row * 2 + (c & 1)) * UT::SC + j + (c >> 1)) * EPB]);
#pragma unroll
                for (int f = 0; f < NFW; ++f) acc[m][p][f] = mfma_kgroup<D>(wf[f], xb, acc[m][p][f]);
            }
        }
    }
    // upsampled channels: phase kernels over the low-resolution tile
    constexpr int WLO = NF * G::NKG_S * 1024;                  // byte offset of the phase packs
    const int wph = WLO + py * 2 * NF * G::NKG_U * 1024;        // this wave's row phase
#pragma unroll
    for (int q = 0; q < G::NKG_U; ++q) {
        u32x4 w0[NFW], w1[NFW];
#pragma unroll
        for (int f = 0; f < NFW; ++f) {
            w0[f] = buf_load16(wr, wl16, wph + ((f0 + f) * G::NKG_U + q) * 1024);
            w1[f] = buf_load16(wr, wl16, wph + ((NF + f0 + f) * G::NKG_U + q) * 1024);
        }
        int b = 4 * q + g;
        if (b >= G::NB_U) b = G::NB_U - 1;
        const int t = b / G::BPT_U, cb = b - t * G::BPT_U;
        const int ty = t / 3, tx = t - ty * 3;
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int r = rb + m + ty;
            const u32x4 xb = *reinterpret_cast<const u32x4*>(&lowt[cb * LPS + (r * UT::LC + j + tx) * EPB]);
#pragma unroll
            for (int f = 0; f < NFW; ++f) {
                acc[m][0][f] = mfma_kgroup<D>(w0[f], xb, acc[m][0][f]);
                acc[m][1][f] = mfma_kgroup<D>(w1[f], xb, acc[m][1][f]);
            }
        }
    }

    // ---------------- epilogue: bias + ReLU, then store or the 1x1 head
    float bias[NFW][4];
#pragma unroll
    for (int f = 0; f < NFW; ++f)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = (f0 + f) * 16 + 4 * g + e;
            bias[f][e] = (co < CO) ? a.bias[co] : 0.0f;
        }
#pragma unroll
    for (int m = 0; m < MR; ++m)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int f = 0; f < NFW; ++f)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[m][p][f][e] = fmaxf(acc[m][p][f][e] + bias[f][e], 0.0f);

    if constexpr (MODE == OutMode::Head) {
        float hw[NF][4];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = f * 16 + 4 * g + e;
                hw[f][e] = (co < CO) ? a.head_w[co] : 0.0f;
            }
        const float hb = a.head_w[CO];
        // s[m][p]: logit of pixel (row m, column 2j + p), complete in every
        // lane group after the two cross-group sums
        float s[RW][2];
#pragma unroll
        for (int m = 0; m < RW; ++m)
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                float v = 0.0f;
#pragma unroll
                for (int f = 0; f < NF; ++f)
#pragma unroll
                    for (int e = 0; e < 4; ++e) v += hw[f][e] * acc[m][p][f][e];
                v = sum_rows4(v);
                s[m][p] = v + hb;
            }
        // lane group g finishes rows m with m % 4 == g: one sigmoid per pixel
        // in the wave, and two adjacent pixels per 8-byte store
#pragma unroll
        for (int m0 = 0; m0 < RW; m0 += 4) {
            if (m0 + g < RW) {
                float l0 = s[m0][0], l1 = s[m0][1];
#pragma unroll
                for (int k = 1; k < 4; ++k)
                    if (m0 + k < RW && g == k) { l0 = s[m0 + k][0]; l1 = s[m0 + k][1]; }
                const int y = y0 + py + 2 * (RW * half + m0 + g), x = x0 + 2 * j;
                const size_t pi = ((size_t)n * h + y) * w + x;
                *reinterpret_cast<float2*>(a.vis + pi) = make_float2(sigmoid_fast(l0), sigmoid_fast(l1));
                if (a.logits) *reinterpret_cast<float2*>(a.logits + pi) = make_float2(l0, l1);
            }
        }
        if (a.act_out) {
#pragma unroll
            for (int m = 0; m < RW; ++m)
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const int y = y0 + py + 2 * (RW * half + m), x = x0 + 2 * j + p;
                    const size_t pi = ((size_t)n * h + y) * w + x;
#pragma unroll
                    for (int f = 0; f < NF; ++f) {
                        const int co = f * 16 + 4 * g;
                        if (co < CO) *reinterpret_cast<f32x4*>(a.act_out + pi * CO + co) = acc[m][p][f];
                    }
                }
        }
    } else {
        // interior tile: every pixel is in the image; offsets relative to the
        // tile's first pixel, the row step in a scalar register
        static_assert(CO % 16 == 0, "stored decoder stages fill whole 16-channel fragments");
        using S = typename ST<D>::S;
        constexpr int SZ = (int)sizeof(S);
        const __amdgpu_buffer_rsrc_t orc =
            buf_rsrc(reinterpret_cast<S*>(a.out) + (((size_t)n * h + y0) * w + x0) * CO);
        const int voff = (((py + 2 * rb) * w + 2 * j) * CO + 4 * g) * SZ;
        const int rstep = 2 * w * CO * SZ;
#pragma unroll
        for (int m = 0; m < MR; ++m)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int f = 0; f < NFW; ++f)
                    buf_store4<S>(orc, voff, m * rstep + (p * CO + (f0 + f) * 16) * SZ, acc[m][p][f]);
    }
}

template <Dt D, int CS, int CU, int CO, OutMode MODE, int TH, int TH_G>
__global__ void __launch_bounds__(kThreads) k_conv3x3_up(ConvArgs a, const void* __restrict__ wup) {
    using T = typename DT<D>::T;
    __shared__ __attribute__((aligned(16))) T smem[up_smem_elems<D, CS, CU, CO, TH, TH_G>()];
    up_block<D, CS, CU, CO, MODE, TH, TH_G>(a, wup, blockIdx.x, smem);
}

// Persistent form: a grid sized to the device's resident capacity walks the
// stage's logical blocks with a stride of the grid (same tiles, same bits).
template <Dt D, int CS, int CU, int CO, OutMode MODE, int TH, int TH_G>
__global__ void __launch_bounds__(kThreads) k_conv3x3_up_persist(ConvArgs a, const void* __restrict__ wup, int total) {
    using T = typename DT<D>::T;
    __shared__ __attribute__((aligned(16))) T smem[up_smem_elems<D, CS, CU, CO, TH, TH_G>()];
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        if (b != (int)blockIdx.x) __syncthreads();     // the previous block's LDS reads are done
        up_block<D, CS, CU, CO, MODE, TH, TH_G>(a, wup, b, smem);
    }
}

}  // namespace ck
}  // namespace nsm
