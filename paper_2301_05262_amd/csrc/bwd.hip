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
//              sums, which a second kernel adds in a fixed order -- no float
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
// weight * dup[.][c_off + c]) * (act_low[q][c] > 0).  One thread per two
// horizontally adjacent low-res pixels and 4 channels: their 4 x 4 reaching
// windows share two hi-res columns, so the thread loads a 4 x 6 window once
// (16-byte loads across channels) and sums each output over its own 4 x 4
// part in the same order as one pixel alone would.
__global__ void __launch_bounds__(256) k_up_transpose_mask(const float* __restrict__ dup, int ci_total,
                                                           int c_off, const float* __restrict__ act_low,
                                                           int C, int n, int hl, int wl,
                                                           float* __restrict__ dz_low) {
    const int C4 = C >> 2, wp = (wl + 1) >> 1;
    const size_t total = (size_t)n * hl * wp * C4;
    // XCD b % 8 takes a contiguous run of blocks, so that the hi-res rows
    // shared by neighbouring low-res rows meet in one L2
    const size_t idx = (size_t)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int c = (int)(idx % C4) * 4;
    const size_t qp = idx / C4;
    const int kp = (int)(qp % wp);
    const int m = (int)((qp / wp) % hl);
    const int f = (int)(qp / ((size_t)wp * hl));
    const int H = 2 * hl, W = 2 * wl;
    const int k0 = 2 * kp;
    float wy[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int Y = 2 * m - 1 + t;
        wy[t] = (Y >= 0 && Y < H) ? up_weight(Y, m, hl) : 0.0f;
    }
    float wx[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = k0 + u, X = 2 * k - 1 + t;
            wx[u][t] = (k < wl && X >= 0 && X < W) ? up_weight(X, k, wl) : 0.0f;
        }
    float4 s[2] = {make_float4(0.f, 0.f, 0.f, 0.f), make_float4(0.f, 0.f, 0.f, 0.f)};
#pragma unroll
    for (int ty = 0; ty < 4; ++ty) {
        if (wy[ty] == 0.0f) continue;
        const int Y = 2 * m - 1 + ty;
        float4 d[6];
#pragma unroll
        for (int col = 0; col < 6; ++col) {
            const int X = 2 * k0 - 1 + col;
            const bool need = (col < 4 && wx[0][col] != 0.0f) || (col >= 2 && wx[1][col - 2] != 0.0f);
            d[col] = need ? *reinterpret_cast<const float4*>(dup + (((size_t)f * H + Y) * W + X) * ci_total + c_off + c)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int tx = 0; tx < 4; ++tx) {
                if (wx[u][tx] == 0.0f) continue;
                const float ww = wy[ty] * wx[u][tx];
                const float4 v = d[2 * u + tx];
                s[u].x += ww * v.x;
                s[u].y += ww * v.y;
                s[u].z += ww * v.z;
                s[u].w += ww * v.w;
            }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int k = k0 + u;
        if (k >= wl) break;
        const size_t q = ((size_t)f * hl + m) * wl + k;
        const float4 av = *reinterpret_cast<const float4*>(act_low + q * C + c);
        float4 o;
        o.x = av.x > 0.0f ? s[u].x : 0.0f;
        o.y = av.y > 0.0f ? s[u].y : 0.0f;
        o.z = av.z > 0.0f ? s[u].z : 0.0f;
        o.w = av.w > 0.0f ? s[u].w : 0.0f;
        *reinterpret_cast<float4*>(dz_low + q * C + c) = o;
    }
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
// GEMM dW[co][j] = sum_p dz[p][co] X[p][j] over the pixels p, with column
// j = tap * CIP + ci (CIP = channels, the skip part padded to 4) and one more
// column of ones for the bias.  MFMA 16x16x4 f32: A = dz (16 output channels
// x 4 pixels), B = X (4 pixels x 16 columns).  Columns go in groups of 64:
// lane (n, g) of MFMA i of a group covers column 64 grp + 4 n + i, so one
// 16-byte LDS read (channels ci .. ci + 3 of one tap, 16-byte aligned) feeds
// the four MFMAs of the group.  Each wave owns one 16-row output fragment.
// When the groups divide evenly among the WPF waves of a fragment, each wave
// takes every WPF-th group over all pixels; otherwise each wave takes all
// groups over every WPF-th step of 4 pixels, and the waves' sums are added
// in a fixed order at the end.  Either way the waves' MFMA work is balanced
// and every result is reproducible bit for bit.
template <int CS, int CU, int CO>
struct WG {
    static constexpr int CSP = round_up(CS, 4);
    static constexpr int CIP = CSP + CU;
    static constexpr int CST = lds_stride<Dt::F32>(CIP);
    static constexpr int NCOL = 9 * CIP;
    static constexpr int NCOLP = round_up(NCOL + 16, 64);    // bias column at NCOLP - 16
    static constexpr int NG = NCOLP / 64;                     // column groups
    static constexpr int NFCO = (CO + 15) / 16;
    static constexpr int COP = NFCO * 16;
    static constexpr int WPF = 4 / NFCO;                      // waves per output fragment
    static constexpr bool BY_GROUP = NG % WPF == 0;
    static constexpr int PS = BY_GROUP ? 1 : WPF;             // waves splitting the pixel steps
    static constexpr int UPW = BY_GROUP ? NG / WPF : NG;      // groups per wave
    static constexpr int PARTIAL = COP * NCOLP;               // floats per block
    static constexpr int XT = (kWTH + 2) * (kTW + 2) * CST;   // halo tile floats
    static constexpr int AUX = LowTile<Dt::F32, CU, kWTH>::SIZE > kWTH * kTW * CO
                                   ? LowTile<Dt::F32, CU, kWTH>::SIZE : kWTH * kTW * CO;
    static constexpr size_t SMEM = (size_t)(XT + AUX) * 4;
    static_assert(4 % NFCO == 0, "1, 2 or 4 output fragments");
    static_assert(CST % 4 == 0 && CIP % 4 == 0, "16-byte aligned channel runs");
    static_assert((PS - 1) * NFCO * 4 * 64 * 4 <= XT + AUX, "the step-split sums are staged in the tile");
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
    constexpr int TH = kWTH, WP = kTW + 2, TPX = TH * kTW, NSTEP = TPX / 4;
    constexpr int CST = G::CST, UPW = G::UPW, PS = G::PS;
    // the low-res rows are needed only while the tile is built, so the
    // output-gradient tile reuses their space
    __shared__ __attribute__((aligned(16))) float smem[G::XT + G::AUX];
    float* const xt = smem;
    float* const lowt = smem + G::XT;
    float* const dzt = smem + G::XT;

    // the wave index is uniform in the wave: keep it in a scalar register
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int n16 = lane & 15, g = lane >> 4;
    const int f = wave / G::WPF, r = wave - f * G::WPF;
    const int phase = PS > 1 ? r : 0;
    // the wave's groups and, per group, the LDS offset of this lane's run of
    // 4 columns (-1: the run that starts with the bias column, -2: padding)
    int grp[UPW], boff[UPW];
#pragma unroll
    for (int k = 0; k < UPW; ++k) {
        const int gi = G::BY_GROUP ? r + k * G::WPF : k;
        grp[k] = gi;
        const int j = gi * 64 + 4 * n16;
        int o = -2;
        if (j < G::NCOL) {
            const int tap = j / G::CIP, ci = j - tap * G::CIP;
            const int ky = tap / 3, kx = tap - ky * 3;
            o = (ky * WP + kx) * CST + ci;     // padding channels of the tile hold zeros
        } else if (j == G::NCOLP - 16) {
            o = -1;
        }
        boff[k] = o;
    }
    const int co = f * 16 + n16;
    f32x4 acc[UPW][4];
#pragma unroll
    for (int k = 0; k < UPW; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[k][i] = f32x4{0.f, 0.f, 0.f, 0.f};

    auto load_ops = [&](int s, float& av, f32x4 (&bv)[UPW]) {
        const int px = 4 * s + g;
        const int poff = ((px / kTW) * WP + (px % kTW)) * CST;
        av = (co < CO) ? dzt[px * CO + co] : 0.0f;
#pragma unroll
        for (int k = 0; k < UPW; ++k) {
            const int o = boff[k];
            bv[k] = o >= 0 ? *reinterpret_cast<const f32x4*>(&xt[poff + o])
                           : (o == -1 ? f32x4{1.f, 0.f, 0.f, 0.f} : f32x4{0.f, 0.f, 0.f, 0.f});
        }
    };

    const int tiles_x = (a.w + kTW - 1) / kTW, tiles_y = (a.h + TH - 1) / TH;
    const long long total = (long long)a.n * tiles_x * tiles_y;
    const long long t0 = total * blockIdx.x / gridDim.x, t1 = total * (blockIdx.x + 1) / gridDim.x;
    for (long long t = t0; t < t1; ++t) {
        const int tx = (int)(t % tiles_x);
        const int ty = (int)((t / tiles_x) % tiles_y);
        const int n = (int)(t / ((long long)tiles_x * tiles_y));
        const int x0 = tx * kTW, y0 = ty * TH;
        __syncthreads();
        // pixel-major here (the walk reads runs of channels of one pixel)
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
        // the operands of the next step are read while this step's MFMAs run
        float av;
        f32x4 bv[UPW];
        load_ops(phase, av, bv);
        for (int s = phase; s < NSTEP; s += PS) {
            float an = 0.0f;
            f32x4 bn[UPW];
            if (s + PS < NSTEP) load_ops(s + PS, an, bn);
#pragma unroll
            for (int k = 0; k < UPW; ++k) {
                if (!G::BY_GROUP || grp[k] < G::NG) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[k][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[k][i], acc[k][i], 0, 0, 0);
                }
            }
            av = an;
#pragma unroll
            for (int k = 0; k < UPW; ++k) bv[k] = bn[k];
        }
    }
    float* out = a.partial + (size_t)blockIdx.x * G::PARTIAL;
    auto store = [&](int k) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                out[(size_t)(f * 16 + 4 * g + e) * G::NCOLP + grp[k] * 64 + 4 * n16 + i] = acc[k][i][e];
    };
    if constexpr (PS > 1) {
        // group by group: the waves of phase > 0 stage their sums, the phase-0
        // wave of the fragment adds them in phase order and stores
        f32x4* stage = reinterpret_cast<f32x4*>(smem);
#pragma unroll
        for (int k = 0; k < UPW; ++k) {
            __syncthreads();
            if (phase > 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) stage[((f * (PS - 1) + phase - 1) * 4 + i) * 64 + lane] = acc[k][i];
            }
            __syncthreads();
            if (phase == 0) {
                for (int p = 1; p < PS; ++p) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const f32x4 v = stage[((f * (PS - 1) + p - 1) * 4 + i) * 64 + lane];
#pragma unroll
                        for (int e = 0; e < 4; ++e) acc[k][i][e] += v[e];
                    }
                }
                store(k);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < UPW; ++k)
            if (grp[k] < G::NG) store(k);
    }
}

// Sum the per-block partials of one channel range of a stage into the flat
// OHWI weights (channels [c_lo, c_lo + cs + cu) of ci_tot) and, with
// `bias`, the biases.  Column of part channel pc and tap t: t * cip + pc for
// pc < cs, t * cip + csp + (pc - cs) above.  Each block takes 16 outputs x 16
// slices of the blocks' partials; a slice sums its partials in block order
// and the slice sums are added in slice order.
constexpr int kReduceOuts = 16, kReduceSlices = 16;
__global__ void __launch_bounds__(256) k_wgrad_reduce(const float* __restrict__ partial, int grid,
                                                      int partial_floats, int co, int ci_tot, int c_lo, int cs,
                                                      int cu, int csp, int cip, int ncolp, int bias,
                                                      float* __restrict__ dw, float* __restrict__ db,
                                                      int accumulate) {
    __shared__ float part_sum[kReduceSlices][kReduceOuts];
    const int cp = cs + cu;
    const int nw = co * 9 * cp;
    const int nout = nw + (bias ? co : 0);
    const int oi = threadIdx.x % kReduceOuts, slice = threadIdx.x / kReduceOuts;
    const int i = blockIdx.x * kReduceOuts + oi;
    int row = 0, colj = 0;
    if (i < nw) {
        const int pc = i % cp, tap = (i / cp) % 9, o = i / (9 * cp);
        row = o;
        colj = tap * cip + (pc < cs ? pc : csp + (pc - cs));
    } else if (i < nout) {
        row = i - nw;
        colj = ncolp - 16;
    }
    float s = 0.0f;
    if (i < nout) {
        const int b0 = grid * slice / kReduceSlices, b1 = grid * (slice + 1) / kReduceSlices;
        const float* src = partial + (size_t)row * ncolp + colj;
        for (int b = b0; b < b1; ++b) s += src[(size_t)b * partial_floats];
    }
    part_sum[slice][oi] = s;
    __syncthreads();
    if (slice != 0 || i >= nout) return;
    float t = part_sum[0][oi];
#pragma unroll
    for (int k = 1; k < kReduceSlices; ++k) t += part_sum[k][oi];
    float* dst;
    if (i < nw) {
        const int pc = i % cp, tap = (i / cp) % 9, o = i / (9 * cp);
        dst = dw + ((size_t)o * 9 + tap) * ci_tot + c_lo + pc;
    } else {
        dst = db + (i - nw);
    }
    *dst = accumulate ? *dst + t : t;
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
    const size_t total = (size_t)n * hl * ((wl + 1) / 2) * (c / 4);
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

// Blocks of a wgrad GEMM: as many as the device holds at once (up to 4 per
// CU; the small-channel stages are bound by their tile loads and need the
// blocks in flight), never more than there are tiles.  The partial sums, and
// so the bits of the result, depend on this count, which is fixed for a
// given device model.
template <int CS, int CU, int CO>
int wgrad_grid_t(int n, int h, int w) {
    static const int cap = [] {
        int dev = 0, cus = 256, per = 1;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_wgrad<CS, CU, CO>, 256, 0) != hipSuccess || per < 1)
            per = 1;
        return std::min(per, 4) * cus;
    }();
    const long long tiles = (long long)n * ((w + kTW - 1) / kTW) * ((h + kWTH - 1) / kWTH);
    return (int)std::min<long long>(cap, tiles);
}

// A stage whose full tile would hold the LDS to one block per CU runs its
// skip and upsampled channels as two GEMMs over their own (smaller) tiles.
template <int CS, int CU, int CO>
constexpr bool wgrad_split() {
    return CS > 0 && CU > 0 && WG<CS, CU, CO>::SMEM > 80 * 1024;
}

template <int CS, int CU, int CO>
size_t wgrad_partial_floats_t(int n, int h, int w) {
    if constexpr (wgrad_split<CS, CU, CO>())
        return (size_t)WG<CS, 0, CO>::PARTIAL * wgrad_grid_t<CS, 0, CO>(n, h, w) +
               (size_t)WG<0, CU, CO>::PARTIAL * wgrad_grid_t<0, CU, CO>(n, h, w);
    else
        return (size_t)WG<CS, CU, CO>::PARTIAL * wgrad_grid_t<CS, CU, CO>(n, h, w);
}

// One GEMM over channels [c_lo, c_lo + PCS + PCU) of a stage with CI_TOT
// input channels; `bias` adds the bias column's sums.
template <int PCS, int PCU, int CO>
hipError_t wgrad_part(const float* in, const float* low, const float* dz, int n, int h, int w, float* partial,
                      int ci_tot, int c_lo, bool bias, float* dw, float* db, bool accumulate, hipStream_t s,
                      const char* name) {
    using G = WG<PCS, PCU, CO>;
    const int grid = wgrad_grid_t<PCS, PCU, CO>(n, h, w);
    WgradArgs a{in, low, dz, partial, n, h, w};
    {
        TraceScope ts("wgrad ", name, s);
        k_wgrad<PCS, PCU, CO><<<grid, 256, 0, s>>>(a);
    }
    const int nout = CO * 9 * (PCS + PCU) + (bias ? CO : 0);
    TraceScope ts2("wgrad_reduce ", name, s);
    k_wgrad_reduce<<<div_up(nout, kReduceOuts), kReduceOuts * kReduceSlices, 0, s>>>(partial, grid, G::PARTIAL, CO, ci_tot, c_lo, PCS, PCU, G::CSP,
                                                    G::CIP, G::NCOLP, bias ? 1 : 0, dw, db, accumulate ? 1 : 0);
    return hipGetLastError();
}

template <int CS, int CU, int CO>
hipError_t wgrad_stage(const float* in, const float* low, const float* dz, int n, int h, int w, float* partial,
                       float* dw, float* db, bool accumulate, hipStream_t s, const char* name) {
    if constexpr (wgrad_split<CS, CU, CO>()) {
        const size_t skip_floats = (size_t)WG<CS, 0, CO>::PARTIAL * wgrad_grid_t<CS, 0, CO>(n, h, w);
        hipError_t e = wgrad_part<CS, 0, CO>(in, nullptr, dz, n, h, w, partial, CS + CU, 0, true, dw, db,
                                             accumulate, s, name);
        if (e != hipSuccess) return e;
        return wgrad_part<0, CU, CO>(nullptr, low, dz, n, h, w, partial + skip_floats, CS + CU, CS, false, dw, db,
                                     accumulate, s, name);
    } else {
        return wgrad_part<CS, CU, CO>(in, low, dz, n, h, w, partial, CS + CU, 0, true, dw, db, accumulate, s, name);
    }
}

size_t wgrad_partial_floats(const ConvStage& st, int n, int h, int w) {
#define NSM_WPF(CS_, CU_, CO_) \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_) return wgrad_partial_floats_t<CS_, CU_, CO_>(n, h, w);
    NSM_BWD_STAGES(NSM_WPF)
#undef NSM_WPF
    return 0;
}

hipError_t conv_wgrad(const ConvStage& st, const float* in, const float* low, const float* dz, int n,
                      int h, int w, float* partial, float* dw, float* db, bool accumulate, hipStream_t s) {
#define NSM_WCASE(CS_, CU_, CO_)                                                                    \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_)                                               \
        return wgrad_stage<CS_, CU_, CO_>(in, low, dz, n, h, w, partial, dw, db, accumulate, s,     \
                                          #CS_ "+" #CU_ "->" #CO_);
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
