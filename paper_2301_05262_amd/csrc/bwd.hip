// Backward (adjoint) kernels of the shadow U-Net, float32 -- the
// differentiation form.  The paper trains its network with gradient descent
// (Sec. 3.3; supplemental Sec. 5); here every stage has a hand-written adjoint:
//
//   head       g = dvis * s * (1 - s) with s = sigmoid(logit); the 1x1 head's
//              weight / bias gradients and the gradient reaching the last
//              conv's pre-activation (through its ReLU: passes where > 0);
//   dgrad      input gradient of a 3x3 conv = a 3x3 conv of the output
//              gradient with the spatially flipped, channel-transposed
//              kernel (the forward conv kernel with a FLIP weight pack and a
//              linear epilogue);
//   wgrad      dW[co][tap][ci] = sum_p dz[p][co] * x[p + tap][ci] and
//              db[co] = sum_p dz[p][co]: an MFMA GEMM with the pixels as K;
//              every block owns a fixed run of tiles and writes its partial
//              sums, which a second kernel adds in block order -- no float
//              atomics, so the result is bitwise reproducible;
//   upsample   adjoint of the bilinear x2 upsampling written as a gather:
//              each low-res pixel sums the hi-res gradients that its taps
//              reached, with the same weights (clamping included);
//   max-pool   each window's gradient goes to its first maximum in the order
//              (0,0), (0,1), (1,0), (1,1); the skip gradient is added and
//              the encoder ReLU mask applied in the same pass.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "conv_kernels.h"

namespace nsm {
namespace {
using namespace ck;

constexpr int kHeadGrid = 1024;
constexpr int kWgradMaxGrid = 512;
constexpr int kWTH = 4;                          // wgrad tile rows (x 32 columns)

// ------------------------------------------------------------------- head
template <int C>
__global__ void __launch_bounds__(256) k_head_bwd(const float* __restrict__ vis,
                                                  const float* __restrict__ dvis,
                                                  const float* __restrict__ act,
                                                  const float* __restrict__ head_w, size_t npix,
                                                  float* __restrict__ dz, float* __restrict__ partial) {
    __shared__ float red[256];
    float acc[C + 1];
#pragma unroll
    for (int c = 0; c <= C; ++c) acc[c] = 0.0f;
    float hw[C];
#pragma unroll
    for (int c = 0; c < C; ++c) hw[c] = head_w[c];
    for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < npix; p += (size_t)gridDim.x * 256) {
        const float s = vis[p];
        const float g = dvis[p] * (s * (1.0f - s));
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float a = act[p * C + c];
            acc[c] += g * a;
            dz[p * C + c] = (a > 0.0f) ? g * hw[c] : 0.0f;
        }
        acc[C] += g;
    }
    // fixed-shape tree reduction per value
    for (int c = 0; c <= C; ++c) {
        red[threadIdx.x] = acc[c];
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * (C + 1) + c] = red[0];
        __syncthreads();
    }
}

__global__ void k_head_reduce(const float* __restrict__ partial, int grid, int n,
                              float* __restrict__ out, int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int b = 0; b < grid; ++b) s += partial[(size_t)b * n + i];
    out[i] = accumulate ? out[i] + s : s;
}

// -------------------------------------------------------------- upsample^T
__device__ __forceinline__ float up_weight(int Y, int m, int hl) {
    const int y0 = (Y - 1) >> 1;
    const float w0 = (Y & 1) ? 0.75f : 0.25f;
    const int a = min(max(y0, 0), hl - 1), b = min(max(y0 + 1, 0), hl - 1);
    return (a == m ? w0 : 0.0f) + (b == m ? 1.0f - w0 : 0.0f);
}

// dz_low[q][c] = (sum over the hi-res pixels whose bilinear taps reach q of
// weight * dup[.][c_off + c]) * (act_low[q][c] > 0).  One thread per low-res
// pixel and 4 channels: 16-byte loads across channels; the at most 4 x 4
// reaching hi-res pixels and their weights are found once per thread.
__global__ void __launch_bounds__(256) k_up_transpose_mask(const float* __restrict__ dup, int ci_total,
                                                           int c_off, const float* __restrict__ act_low,
                                                           int C, int n, int hl, int wl,
                                                           float* __restrict__ dz_low) {
    const int C4 = C >> 2;
    const size_t total = (size_t)n * hl * wl * C4;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int c = (int)(idx % C4) * 4;
    const size_t q = idx / C4;
    const int k = (int)(q % wl);
    const int m = (int)((q / wl) % hl);
    const int f = (int)(q / ((size_t)wl * hl));
    const int H = 2 * hl, W = 2 * wl;
    float wy[4], wx[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int Y = 2 * m - 1 + t, X = 2 * k - 1 + t;
        wy[t] = (Y >= 0 && Y < H) ? up_weight(Y, m, hl) : 0.0f;
        wx[t] = (X >= 0 && X < W) ? up_weight(X, k, wl) : 0.0f;
    }
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int ty = 0; ty < 4; ++ty) {
        if (wy[ty] == 0.0f) continue;
        const int Y = 2 * m - 1 + ty;
#pragma unroll
        for (int tx = 0; tx < 4; ++tx) {
            if (wx[tx] == 0.0f) continue;
            const int X = 2 * k - 1 + tx;
            const float ww = wy[ty] * wx[tx];
            const float4 d = *reinterpret_cast<const float4*>(dup + (((size_t)f * H + Y) * W + X) * ci_total + c_off + c);
            s.x += ww * d.x;
            s.y += ww * d.y;
            s.z += ww * d.z;
            s.w += ww * d.w;
        }
    }
    const float4 av = *reinterpret_cast<const float4*>(act_low + q * C + c);
    float4 o;
    o.x = av.x > 0.0f ? s.x : 0.0f;
    o.y = av.y > 0.0f ? s.y : 0.0f;
    o.z = av.z > 0.0f ? s.z : 0.0f;
    o.w = av.w > 0.0f ? s.w : 0.0f;
    *reinterpret_cast<float4*>(dz_low + q * C + c) = o;
}

// ---------------------------------------------------------------- pool^T
// One channel of the max-pool adjoint: the window's gradient goes to its
// first maximum in (0,0), (0,1), (1,0), (1,1) order; ReLU'(0) = 0.
__device__ __forceinline__ float pool_route(float a0, float a1, float a2, float a3, float me, float d_skip,
                                            float d_pool, int mine) {
    int best = 0;
    float bv = a0;
    if (a1 > bv) { bv = a1; best = 1; }
    if (a2 > bv) { bv = a2; best = 2; }
    if (a3 > bv) { bv = a3; best = 3; }
    if (!(me > 0.0f)) return 0.0f;
    return best == mine ? d_skip + d_pool : d_skip;
}

// dz[p][c] = (dskip[p][c] + routed max-pool gradient) * (act[p][c] > 0).
// One thread per pixel and 4 channels (16-byte accesses).
__global__ void __launch_bounds__(256) k_pool_transpose_mask(const float* __restrict__ dskip, int ci_total,
                                                             const float* __restrict__ dpool,
                                                             const float* __restrict__ act, int C, int n,
                                                             int h, int w, float* __restrict__ dz) {
    const int C4 = C >> 2;
    const size_t total = (size_t)n * h * w * C4;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int c = (int)(idx % C4) * 4;
    const size_t p = idx / C4;
    const int x = (int)(p % w);
    const int y = (int)((p / w) % h);
    const int f = (int)(p / ((size_t)w * h));
    const int y0 = y & ~1, x0 = x & ~1;
    const int mine = ((y - y0) << 1) | (x - x0);
    const float* r0 = act + (((size_t)f * h + y0) * w + x0) * C + c;
    const float* r1 = r0 + (size_t)w * C;
    const float4 w0 = *reinterpret_cast<const float4*>(r0), w1 = *reinterpret_cast<const float4*>(r0 + C);
    const float4 w2 = *reinterpret_cast<const float4*>(r1), w3 = *reinterpret_cast<const float4*>(r1 + C);
    const float4 a = *reinterpret_cast<const float4*>(act + p * C + c);
    const float4 ds = *reinterpret_cast<const float4*>(dskip + p * ci_total + c);
    const float4 dp = *reinterpret_cast<const float4*>(dpool + (((size_t)f * (h >> 1) + (y >> 1)) * (w >> 1) + (x >> 1)) * C + c);
    float4 o;
    o.x = pool_route(w0.x, w1.x, w2.x, w3.x, a.x, ds.x, dp.x, mine);
    o.y = pool_route(w0.y, w1.y, w2.y, w3.y, a.y, ds.y, dp.y, mine);
    o.z = pool_route(w0.z, w1.z, w2.z, w3.z, a.z, ds.z, dp.z, mine);
    o.w = pool_route(w0.w, w1.w, w2.w, w3.w, a.w, ds.w, dp.w, mine);
    *reinterpret_cast<float4*>(dz + p * C + c) = o;
}

// ------------------------------------------------------------------ wgrad
template <int CS, int CU, int CO>
struct WG {
    static constexpr int CSP = round_up(CS, 4);
    static constexpr int CIP = CSP + CU;
    static constexpr int CST = lds_stride<Dt::F32>(CIP);
    static constexpr int NCOL = 9 * CIP;
    static constexpr int NCOLP = round_up(NCOL, 16) + 16;     // + one bias block
    static constexpr int NFCOL = NCOLP / 16;
    static constexpr int NFCO = (CO + 15) / 16;
    static constexpr int COP = NFCO * 16;
    static constexpr int FPW = (NFCOL + 3) / 4;               // column fragments per wave
    static constexpr int PARTIAL = COP * NCOLP;                // floats per block
};

struct WgradArgs {
    const float* in;
    const float* low;
    const float* dz;
    float* partial;
    int n, h, w;
};

template <int CS, int CU, int CO>
__global__ void __launch_bounds__(256) k_wgrad(WgradArgs a) {
    using G = WG<CS, CU, CO>;
    constexpr int TH = kWTH, WP = kTW + 2, NPIX = (TH + 2) * WP, TPX = TH * kTW;
    constexpr int CST = G::CST, FPW = G::FPW, NFCO = G::NFCO;
    __shared__ __attribute__((aligned(16))) float xt[NPIX * CST];
    __shared__ __attribute__((aligned(16))) float dzt[TPX * CO];
    __shared__ __attribute__((aligned(16))) float lowt[LowTile<Dt::F32, CU, TH>::SIZE];

    // the wave index is uniform in the wave: keep it in a scalar register
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;
    // per owned column fragment: LDS offset of this lane's (tap, channel), -1 bias column, -2 padding
    int boff[FPW];
#pragma unroll
    for (int i = 0; i < FPW; ++i) {
        const int fcol = wave * FPW + i;
        const int j = fcol * 16 + col;
        int o = -2;
        if (fcol < G::NFCOL) {
            if (j < G::NCOL) {
                const int tap = j / G::CIP, ci = j - tap * G::CIP;
                const int ky = tap / 3, kx = tap - ky * 3;
                const bool real = ci < CS || ci >= G::CSP;
                o = real ? (ky * WP + kx) * CST + ci : -2;
            } else if (j == G::NCOLP - 16) {
                o = -1;
            }
        }
        boff[i] = o;
    }
    f32x4 acc[NFCO][FPW];
#pragma unroll
    for (int f = 0; f < NFCO; ++f)
#pragma unroll
        for (int i = 0; i < FPW; ++i) acc[f][i] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int tiles_x = (a.w + kTW - 1) / kTW, tiles_y = (a.h + TH - 1) / TH;
    const long long total = (long long)a.n * tiles_x * tiles_y;
    const long long t0 = total * blockIdx.x / gridDim.x, t1 = total * (blockIdx.x + 1) / gridDim.x;
    for (long long t = t0; t < t1; ++t) {
        const int tx = (int)(t % tiles_x);
        const int ty = (int)((t / tiles_x) % tiles_y);
        const int n = (int)(t / ((long long)tiles_x * tiles_y));
        const int x0 = tx * kTW, y0 = ty * TH;
        __syncthreads();
        // pixel-major here (the wgrad walk indexes single channels of a pixel)
        load_halo_tile<Dt::F32, (CS % 4 != 0), CS, CU, CST, DT<Dt::F32>::EPB, TH>(xt, lowt, a.in, a.low, n, a.h,
                                                                                a.w, x0, y0);
        for (int idx = threadIdx.x; idx < TPX * (CO / 4); idx += 256) {
            const int px = idx / (CO / 4), c4 = idx - px * (CO / 4);
            const int y = y0 + px / kTW, x = x0 + (px % kTW);
            f32x4 v = {0.f, 0.f, 0.f, 0.f};
            if (y < a.h && x < a.w)
                v = *reinterpret_cast<const f32x4*>(a.dz + (((size_t)n * a.h + y) * a.w + x) * CO + 4 * c4);
            *reinterpret_cast<f32x4*>(&dzt[px * CO + 4 * c4]) = v;
        }
        __syncthreads();
        for (int s = 0; s < TPX / 4; ++s) {
            const int px = 4 * s + g;
            const int poff = ((px / kTW) * WP + (px % kTW)) * CST;
            float av[NFCO];
#pragma unroll
            for (int f = 0; f < NFCO; ++f) {
                const int co = f * 16 + col;
                av[f] = (co < CO) ? dzt[px * CO + co] : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < FPW; ++i) {
                const int o = boff[i];
                const float bv = o >= 0 ? xt[poff + o] : (o == -1 ? 1.0f : 0.0f);
#pragma unroll
                for (int f = 0; f < NFCO; ++f)
                    acc[f][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[f], bv, acc[f][i], 0, 0, 0);
            }
        }
    }
    float* out = a.partial + (size_t)blockIdx.x * G::PARTIAL;
#pragma unroll
    for (int f = 0; f < NFCO; ++f)
#pragma unroll
        for (int i = 0; i < FPW; ++i) {
            const int fcol = wave * FPW + i;
            if (fcol >= G::NFCOL) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                out[(size_t)(f * 16 + 4 * g + e) * G::NCOLP + fcol * 16 + col] = acc[f][i][e];
        }
}

// Sum the per-block partials in block order into the flat OHWI weights and biases.
__global__ void k_wgrad_reduce(const float* __restrict__ partial, int grid, int partial_floats, int cs,
                               int cu, int co, int csp, int cip, int ncolp, float* __restrict__ dw,
                               float* __restrict__ db, int accumulate) {
    const int ci_tot = cs + cu;
    const int nw = co * 9 * ci_tot;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw + co) return;
    int row, colj;
    if (i < nw) {
        const int ci = i % ci_tot, tap = (i / ci_tot) % 9, o = i / (9 * ci_tot);
        const int lc = ci < cs ? ci : csp + (ci - cs);
        row = o;
        colj = tap * cip + lc;
    } else {
        row = i - nw;
        colj = ncolp - 16;
    }
    float s = 0.0f;
    for (int b = 0; b < grid; ++b) s += partial[(size_t)b * partial_floats + (size_t)row * ncolp + colj];
    float* dst = (i < nw) ? dw + i : db + (i - nw);
    *dst = accumulate ? *dst + s : s;
}

#define NSM_BWD_STAGES(X) \
    X(6, 0, 16)           \
    X(8, 0, 16)           \
    X(16, 0, 32)          \
    X(32, 0, 64)          \
    X(32, 64, 32)         \
    X(16, 32, 16)         \
    X(6, 0, 8)            \
    X(8, 0, 16)           \
    X(8, 16, 8)

inline int div_up(size_t a, int b) { return (int)((a + b - 1) / b); }

}  // namespace

// ------------------------------------------------------------ host entry
bool backward_supported(const ConvStage& st) {
#define NSM_BSUP(CS_, CU_, CO_) \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_) return true;
    NSM_BWD_STAGES(NSM_BSUP)
#undef NSM_BSUP
    return false;
}

int head_grid(size_t npix) { return (int)std::min<size_t>(kHeadGrid, (npix + 255) / 256); }

hipError_t head_backward(int c0, const float* vis, const float* dvis, const float* act,
                         const float* head_w, size_t npix, float* dz, float* partial, hipStream_t s) {
    const int grid = head_grid(npix);
    TraceScope ts("head_bwd", "", s);
    if (c0 == 16)
        k_head_bwd<16><<<grid, 256, 0, s>>>(vis, dvis, act, head_w, npix, dz, partial);
    else if (c0 == 8)
        k_head_bwd<8><<<grid, 256, 0, s>>>(vis, dvis, act, head_w, npix, dz, partial);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t head_reduce(int c0, const float* partial, size_t npix, float* dw, bool accumulate,
                       hipStream_t s) {
    TraceScope ts("head_reduce", "", s);
    k_head_reduce<<<1, 64, 0, s>>>(partial, head_grid(npix), c0 + 1, dw, accumulate ? 1 : 0);
    return hipGetLastError();
}

size_t head_partial_floats(int c0, size_t npix) { return (size_t)head_grid(npix) * (c0 + 1); }

hipError_t up_transpose_mask(int c, int ci_total, int c_off, const float* dup, const float* act_low,
                             int n, int hl, int wl, float* dz_low, hipStream_t s) {
    const size_t total = (size_t)n * hl * wl * (c / 4);
    TraceScope ts("up_transpose_mask", "", s);
    k_up_transpose_mask<<<div_up(total, 256), 256, 0, s>>>(dup, ci_total, c_off, act_low, c, n, hl, wl,
                                                           dz_low);
    return hipGetLastError();
}

hipError_t pool_transpose_mask(int c, int ci_total, const float* dskip, const float* dpool,
                               const float* act, int n, int h, int w, float* dz, hipStream_t s) {
    const size_t total = (size_t)n * h * w * (c / 4);
    TraceScope ts("pool_transpose_mask", "", s);
    k_pool_transpose_mask<<<div_up(total, 256), 256, 0, s>>>(dskip, ci_total, dpool, act, c, n, h, w, dz);
    return hipGetLastError();
}

int wgrad_grid(int n, int h, int w) {
    const long long tiles = (long long)n * ((w + kTW - 1) / kTW) * ((h + kWTH - 1) / kWTH);
    return (int)std::min<long long>(kWgradMaxGrid, tiles);
}

size_t wgrad_partial_floats(const ConvStage& st, int n, int h, int w) {
#define NSM_WPF(CS_, CU_, CO_) \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_) return (size_t)WG<CS_, CU_, CO_>::PARTIAL * wgrad_grid(n, h, w);
    NSM_BWD_STAGES(NSM_WPF)
#undef NSM_WPF
    return 0;
}

hipError_t conv_wgrad(const ConvStage& st, const float* in, const float* low, const float* dz, int n,
                      int h, int w, float* partial, float* dw, float* db, bool accumulate, hipStream_t s) {
    const int grid = wgrad_grid(n, h, w);
    WgradArgs a{in, low, dz, partial, n, h, w};
#define NSM_WCASE(CS_, CU_, CO_)                                                                    \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_) {                                             \
        using G = WG<CS_, CU_, CO_>;                                                                \
        {                                                                                           \
            TraceScope ts("wgrad " #CS_ "+" #CU_ "->" #CO_, "", s);                                 \
            k_wgrad<CS_, CU_, CO_><<<grid, 256, 0, s>>>(a);                                         \
        }                                                                                           \
        const int nout = CO_ * 9 * (CS_ + CU_) + CO_;                                               \
        TraceScope ts2("wgrad_reduce " #CS_ "+" #CU_ "->" #CO_, "", s);                             \
        k_wgrad_reduce<<<div_up(nout, 256), 256, 0, s>>>(partial, grid, G::PARTIAL, CS_, CU_, CO_,  \
                                                         G::CSP, G::CIP, G::NCOLP, dw, db,           \
                                                         accumulate ? 1 : 0);                       \
        return hipGetLastError();                                                                   \
    }
    NSM_BWD_STAGES(NSM_WCASE)
#undef NSM_WCASE
    return hipErrorInvalidValue;
}

// dgrad: a 3x3 conv of dz (st.co channels) producing st.cs + st.cu channels.
size_t dgrad_packed_bytes(const ConvStage& st) {
#define NSM_DPB(CS_, CU_, CO_) \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_) return packed_bytes<Dt::F32, CO_, 0, CS_ + CU_>();
    NSM_BWD_STAGES(NSM_DPB)
#undef NSM_DPB
    return 0;
}

hipError_t pack_dgrad_weights(const ConvStage& st, const float* w_ohwi, void* packed, hipStream_t s) {
#define NSM_DPK(CS_, CU_, CO_)                                                                     \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_) {                                            \
        constexpr size_t nb = packed_bytes<Dt::F32, CO_, 0, CS_ + CU_>();                          \
        constexpr int total = (int)(nb / 16 * 4);                                                  \
        k_pack<Dt::F32, CO_, 0, CS_ + CU_, true><<<(total + 255) / 256, 256, 0, s>>>(w_ohwi, packed); \
        return hipGetLastError();                                                                  \
    }
    NSM_BWD_STAGES(NSM_DPK)
#undef NSM_DPK
    return hipErrorInvalidValue;
}

hipError_t conv_dgrad(const ConvStage& st, const void* wpk, const float* dz, int n, int h, int w,
                      float* dx, hipStream_t s) {
    ConvArgs a{};
    a.in = dz;
    a.wpk = wpk;
    a.out = dx;
    a.n = n;
    a.h = h;
    a.w = w;
#define NSM_DCASE(CS_, CU_, CO_)                                                                   \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_) {                                            \
        dim3 grid((w + kTW - 1) / kTW, (h + 7) / 8, n);                                            \
        TraceScope ts("dgrad " #CO_ "->" #CS_ "+" #CU_, "", s);                                    \
        k_conv3x3<Dt::F32, false, CO_, 0, CS_ + CU_, OutMode::Linear, 8><<<grid, kThreads, 0, s>>>(a); \
        return hipGetLastError();                                                                  \
    }
    NSM_BWD_STAGES(NSM_DCASE)
#undef NSM_DCASE
    return hipErrorInvalidValue;
}

}  // namespace nsm
