// Fused 3x3 convolution stages of the shadow U-Net as MFMA implicit GEMM.
//
// The network (paper Sec. 4.5) is a U-Net trimmed to one 3x3 convolution per
// level with bilinear upsampling; the paper's measurements (supplemental
// Sec. 3, layer-wise table) show its runtime follows the size of the
// temporary buffers rather than the flop count, so every stage here is one
// kernel that reads its inputs once and writes its outputs once:
//
//   prologue   halo tile (TH+2) x (TW+2) pixels -> LDS, in the storage
//              dtype: zero padding outside the image, float32 features
//              converted on load, and for decoder stages the concat
//              [skip, bilinear-x2(lower level)] formed on the fly;
//   main loop  D[co][px] += W[co][k] * X[k][px] with k = (tap, channel),
//              weights from a pre-packed global layout (one coalesced
//              16-byte load per lane per k-group), im2col operand from LDS
//              (one ds_read_b128 per lane per k-group);
//   epilogue   bias + ReLU, then one of: store; store + 2x2 max-pool; or the
//              1x1 head + sigmoid (visibility in [0, 1]).
//
// MFMA shapes: float32 uses v_mfma_f32_16x16x4_f32 (4 per k-group of 16),
// bf16 / fp16 use v_mfma_f32_16x16x32_{bf16,f16} (1 per k-group of 32); all
// accumulate in float32.  Rows of the MFMA are output channels, columns are
// 16 consecutive pixels of one image row, so each lane ends up holding four
// consecutive channels of one pixel: stores are contiguous NHWC segments.
//
// A "block" is 16 bytes of one pixel's channels (4 floats or 8 halves).  The
// K dimension is the sequence of blocks over (tap, channel block); lane group
// g = lane / 16 of k-group q reads block 4q + g.  Any assignment of k to
// (lane group, element) works as long as weights and pixels agree, and this
// one makes every operand fetch a single 16-byte access.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace nsm {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <Dt D> struct DT;
template <> struct DT<Dt::F32> { using T = float; static constexpr int EPB = 4; };
template <> struct DT<Dt::BF16> { using T = __bf16; static constexpr int EPB = 8; };
template <> struct DT<Dt::F16> { using T = _Float16; static constexpr int EPB = 8; };

constexpr int kThreads = 256;
constexpr int kTW = 32;   // tile width: two 16-pixel MFMA column fragments

__host__ __device__ constexpr int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Channel stride (elements) of one LDS pixel: padded so that the byte
// stride is an odd multiple of 16 (conflict-free 16-byte reads across the
// 16 pixels of a fragment).
template <Dt D>
__host__ __device__ constexpr int lds_stride(int cip) {
    constexpr int sz = sizeof(typename DT<D>::T);
    int units = cip * sz / 16;
    if ((units & 1) == 0) units += 1;
    return units * 16 / sz;
}

template <Dt D, int CS, int CU, int CO>
struct Geo {
    static constexpr int EPB = DT<D>::EPB;
    static constexpr int CSP = round_up(CS, EPB);
    static constexpr int CIP = CSP + CU;
    static constexpr int BPT = CIP / EPB;        // 16-byte blocks per tap
    static constexpr int NB = 9 * BPT;           // blocks along K
    static constexpr int NKG = (NB + 3) / 4;     // k-groups
    static constexpr int NF = (CO + 15) / 16;    // 16-channel output fragments
    static constexpr int CST = lds_stride<D>(CIP);
    static_assert(CU % EPB == 0, "upsampled channels must fill whole blocks");
};

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(__bf16 v) { return (float)v; }
__device__ __forceinline__ float to_f(_Float16 v) { return (float)v; }

template <typename T> __device__ __forceinline__ T from_f(float v);
template <> __device__ __forceinline__ float from_f<float>(float v) { return v; }
template <> __device__ __forceinline__ __bf16 from_f<__bf16>(float v) { return (__bf16)v; }
template <> __device__ __forceinline__ _Float16 from_f<_Float16>(float v) { return (_Float16)v; }

template <Dt D>
__device__ __forceinline__ f32x4 mfma_kgroup(const u32x4& wa, const u32x4& xb, f32x4 acc) {
    if constexpr (D == Dt::F32) {
        const f32x4 a = __builtin_bit_cast(f32x4, wa);
        const f32x4 b = __builtin_bit_cast(f32x4, xb);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], acc, 0, 0, 0);
    } else if constexpr (D == Dt::BF16) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, wa),
                                                      __builtin_bit_cast(bf16x8, xb), acc, 0, 0, 0);
    } else {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, wa),
                                                     __builtin_bit_cast(f16x8, xb), acc, 0, 0, 0);
    }
    return acc;
}

// Pack EPB floats into one 16-byte block of the storage type.
template <Dt D>
__device__ __forceinline__ u32x4 pack_block(const float* v) {
    using T = typename DT<D>::T;
    constexpr int EPB = DT<D>::EPB;
    T t[EPB];
#pragma unroll
    for (int e = 0; e < EPB; ++e) t[e] = from_f<T>(v[e]);
    u32x4 r;
    __builtin_memcpy(&r, t, 16);
    return r;
}

template <Dt D>
__device__ __forceinline__ void unpack_block(const u32x4& r, float* v) {
    using T = typename DT<D>::T;
    constexpr int EPB = DT<D>::EPB;
    T t[EPB];
    __builtin_memcpy(t, &r, 16);
#pragma unroll
    for (int e = 0; e < EPB; ++e) v[e] = to_f(t[e]);
}

template <Dt D, bool IN_F32, int CS, int CU, int CO, OutMode MODE, int TH>
__global__ void __launch_bounds__(kThreads) k_conv3x3(ConvArgs a) {
    using T = typename DT<D>::T;
    using G = Geo<D, CS, CU, CO>;
    constexpr int EPB = G::EPB, CST = G::CST, NKG = G::NKG, NF = G::NF, BPT = G::BPT, NB = G::NB;
    constexpr int HP = TH + 2, WP = kTW + 2, NPIX = HP * WP;
    constexpr int NCH_S = G::CSP / EPB, NCH_U = CU / EPB, NCH = NCH_S + NCH_U;
    constexpr int RPW = TH / 4;                 // rows per wave
    constexpr int MF = RPW * 2;                 // M-fragments per wave
    static_assert(MODE != OutMode::Pool || RPW == 2, "pooling needs row pairs per wave");

    __shared__ __attribute__((aligned(16))) T tile[NPIX * CST];

    const int h = a.h, w = a.w;
    const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * TH, n = blockIdx.z;

    // ---------------- prologue: halo tile to LDS
    for (int idx = threadIdx.x; idx < NPIX * NCH; idx += kThreads) {
        const int pix = idx / NCH, ch = idx - pix * NCH;
        const int ty = pix / WP, tx = pix - ty * WP;
        const int y = y0 + ty - 1, x = x0 + tx - 1;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (y >= 0 && y < h && x >= 0 && x < w) {
            if (ch < NCH_S) {
                const size_t p = ((size_t)n * h + y) * w + x;
                if constexpr (IN_F32) {
                    const float* src = reinterpret_cast<const float*>(a.in) + p * CS;
                    float f[EPB];
#pragma unroll
                    for (int e = 0; e < EPB; ++e) {
                        const int c = ch * EPB + e;
                        f[e] = (c < CS) ? src[c] : 0.0f;
                    }
                    v = pack_block<D>(f);
                } else {
                    v = *reinterpret_cast<const u32x4*>(reinterpret_cast<const T*>(a.in) + p * CS + ch * EPB);
                }
            } else if constexpr (CU > 0) {
                const int hl = h >> 1, wl = w >> 1;
                const int ya = (y - 1) >> 1, xa = (x - 1) >> 1;
                const float wy0 = (y & 1) ? 0.75f : 0.25f, wx0 = (x & 1) ? 0.75f : 0.25f;
                const float wy1 = 1.0f - wy0, wx1 = 1.0f - wx0;
                const int yA = max(ya, 0), yB = min(ya + 1, hl - 1);
                const int xA = max(xa, 0), xB = min(xa + 1, wl - 1);
                const T* low = reinterpret_cast<const T*>(a.low) + (size_t)n * hl * wl * CU + (ch - NCH_S) * EPB;
                float f00[EPB], f01[EPB], f10[EPB], f11[EPB], f[EPB];
                unpack_block<D>(*reinterpret_cast<const u32x4*>(low + ((size_t)yA * wl + xA) * CU), f00);
                unpack_block<D>(*reinterpret_cast<const u32x4*>(low + ((size_t)yA * wl + xB) * CU), f01);
                unpack_block<D>(*reinterpret_cast<const u32x4*>(low + ((size_t)yB * wl + xA) * CU), f10);
                unpack_block<D>(*reinterpret_cast<const u32x4*>(low + ((size_t)yB * wl + xB) * CU), f11);
#pragma unroll
                for (int e = 0; e < EPB; ++e)
                    f[e] = wy0 * (wx0 * f00[e] + wx1 * f01[e]) + wy1 * (wx0 * f10[e] + wx1 * f11[e]);
                v = pack_block<D>(f);
            }
        }
        *reinterpret_cast<u32x4*>(&tile[pix * CST + ch * EPB]) = v;
    }
    __syncthreads();

    // ---------------- main loop
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int px = lane & 15, g = lane >> 4;
    const u32x4* wpk = reinterpret_cast<const u32x4*>(a.wpk);
    f32x4 acc[MF][NF];
#pragma unroll
    for (int m = 0; m < MF; ++m)
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[m][f] = f32x4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int q = 0; q < NKG; ++q) {
        u32x4 wf[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) wf[f] = wpk[(f * NKG + q) * 64 + lane];
        int b = 4 * q + g;
        if (b >= NB) b = NB - 1;               // padding k: weights are zero there
        const int tap = b / BPT, cb = b - tap * BPT;
        const int ky = tap / 3, kx = tap - ky * 3;
        const int base = (ky * WP + kx + px) * CST + cb * EPB;
#pragma unroll
        for (int m = 0; m < MF; ++m) {
            const int r = wave * RPW + (m >> 1), cf = m & 1;
            const u32x4 xb = *reinterpret_cast<const u32x4*>(&tile[base + (r * WP + cf * 16) * CST]);
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[m][f] = mfma_kgroup<D>(wf[f], xb, acc[m][f]);
        }
    }

    // ---------------- epilogue
    float bias[NF][4];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = f * 16 + 4 * g + e;
            bias[f][e] = (co < CO) ? a.bias[co] : 0.0f;
        }
#pragma unroll
    for (int m = 0; m < MF; ++m)
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[m][f][e] = fmaxf(acc[m][f][e] + bias[f][e], 0.0f);

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
#pragma unroll
        for (int m = 0; m < MF; ++m) {
            const int y = y0 + wave * RPW + (m >> 1), x = x0 + (m & 1) * 16 + px;
            const bool ok = y < h && x < w;
            const size_t p = ((size_t)n * h + y) * w + x;
            float s = 0.0f;
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int e = 0; e < 4; ++e) s += hw[f][e] * acc[m][f][e];
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            if (ok && g == 0) {
                const float logit = s + hb;
                a.vis[p] = 1.0f / (1.0f + __expf(-logit));
                if (a.logits) a.logits[p] = logit;
            }
            if (ok && a.act_out) {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const int co = f * 16 + 4 * g;
                    if (co < CO) *reinterpret_cast<f32x4*>(a.act_out + p * CO + co) = acc[m][f];
                }
            }
        }
    } else {
        T* out = reinterpret_cast<T*>(a.out);
#pragma unroll
        for (int m = 0; m < MF; ++m) {
            const int y = y0 + wave * RPW + (m >> 1), x = x0 + (m & 1) * 16 + px;
            if (y < h && x < w) {
                const size_t p = ((size_t)n * h + y) * w + x;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const int co = f * 16 + 4 * g;
                    if (co < CO) {
                        T t4[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) t4[e] = from_f<T>(acc[m][f][e]);
                        if constexpr (sizeof(T) == 4) {
                            f32x4 v;
                            __builtin_memcpy(&v, t4, 16);
                            *reinterpret_cast<f32x4*>(out + p * CO + co) = v;
                        } else {
                            uint2 v;
                            __builtin_memcpy(&v, t4, 8);
                            *reinterpret_cast<uint2*>(out + p * CO + co) = v;
                        }
                    }
                }
            }
        }
        if constexpr (MODE == OutMode::Pool) {
            T* pooled = reinterpret_cast<T*>(a.pooled);
            const int hp = h >> 1, wp = w >> 1;
#pragma unroll
            for (int cf = 0; cf < 2; ++cf) {
                const int yp = (y0 >> 1) + wave, xp = ((x0 + cf * 16 + px) >> 1);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    float mx[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float v = fmaxf(acc[cf][f][e], acc[2 + cf][f][e]);
                        mx[e] = fmaxf(v, __shfl_xor(v, 1));
                    }
                    const int co = f * 16 + 4 * g;
                    if ((px & 1) == 0 && yp < hp && xp < wp && co < CO) {
                        const size_t p = ((size_t)n * hp + yp) * wp + xp;
                        T t4[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) t4[e] = from_f<T>(mx[e]);
                        if constexpr (sizeof(T) == 4) {
                            f32x4 v;
                            __builtin_memcpy(&v, t4, 16);
                            *reinterpret_cast<f32x4*>(pooled + p * CO + co) = v;
                        } else {
                            uint2 v;
                            __builtin_memcpy(&v, t4, 8);
                            *reinterpret_cast<uint2*>(pooled + p * CO + co) = v;
                        }
                    }
                }
            }
        }
    }
}

// Weight repack: OHWI float32 [CO][3][3][CS+CU] -> [NF][NKG][64 lanes][EPB] storage type.
template <Dt D, int CS, int CU, int CO>
__global__ void k_pack(const float* __restrict__ w, void* __restrict__ out) {
    using T = typename DT<D>::T;
    using G = Geo<D, CS, CU, CO>;
    constexpr int EPB = G::EPB;
    constexpr int total = G::NF * G::NKG * 64 * EPB;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int e = idx % EPB;
    const int lane = (idx / EPB) % 64;
    const int q = (idx / (EPB * 64)) % G::NKG;
    const int f = idx / (EPB * 64 * G::NKG);
    const int co = f * 16 + (lane & 15);
    const int b = 4 * q + (lane >> 4);
    float v = 0.0f;
    if (b < G::NB && co < CO) {
        const int tap = b / G::BPT, cb = b % G::BPT;
        const int c = cb * EPB + e;
        int ci = -1;
        if (c < G::CSP) ci = (c < CS) ? c : -1;
        else ci = CS + (c - G::CSP);
        if (ci >= 0) v = w[((size_t)co * 9 + tap) * (CS + CU) + ci];
    }
    reinterpret_cast<T*>(out)[idx] = from_f<T>(v);
}

template <Dt D, int CS, int CU, int CO>
constexpr size_t packed_bytes() {
    using G = Geo<D, CS, CU, CO>;
    return (size_t)G::NF * G::NKG * 64 * 16;
}

// ---------------------------------------------------------------- dispatch
// Supported stages: (cs, cu, co, mode, float32 input, tile rows) per dtype.
#define NSM_STAGES(X)                           \
    X(6, 0, 16, Pool, true, 8)                  \
    X(8, 0, 16, Pool, true, 8)                  \
    X(16, 0, 32, Pool, false, 8)                \
    X(32, 0, 64, Store, false, 8)               \
    X(32, 64, 32, Store, false, 4)              \
    X(16, 32, 16, Head, false, 8)               \
    X(6, 0, 8, Pool, true, 8)                   \
    X(8, 0, 16, Store, false, 8)                \
    X(8, 16, 8, Head, false, 8)

template <Dt D> constexpr const char* dt_suffix() {
    return D == Dt::F32 ? " f32" : (D == Dt::BF16 ? " bf16" : " f16");
}

template <Dt D>
hipError_t launch(const ConvStage& st, OutMode mode, const ConvArgs& a, hipStream_t s, bool* found) {
#define NSM_CASE(CS_, CU_, CO_, MODE_, F32_, TH_)                                              \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_ && mode == OutMode::MODE_ &&             \
        a.in_f32 == F32_) {                                                                    \
        *found = true;                                                                         \
        dim3 grid((a.w + kTW - 1) / kTW, (a.h + TH_ - 1) / TH_, a.n);                          \
        TraceScope ts("conv3x3 " #CS_ "+" #CU_ "->" #CO_ " " #MODE_, dt_suffix<D>(), s);      \
        k_conv3x3<D, F32_, CS_, CU_, CO_, OutMode::MODE_, TH_><<<grid, kThreads, 0, s>>>(a);   \
        return hipGetLastError();                                                              \
    }
    NSM_STAGES(NSM_CASE)
#undef NSM_CASE
    *found = false;
    return hipErrorInvalidValue;
}

template <Dt D>
bool pack_dispatch(const ConvStage& st, const float* w, void* out, hipStream_t s, size_t* bytes) {
#define NSM_PCASE(CS_, CU_, CO_, MODE_, F32_, TH_)                                             \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_) {                                        \
        constexpr size_t nb = packed_bytes<D, CS_, CU_, CO_>();                                \
        if (bytes) *bytes = nb;                                                                \
        if (out) {                                                                             \
            constexpr int total = (int)(nb / 16 * DT<D>::EPB);                                 \
            k_pack<D, CS_, CU_, CO_><<<(total + 255) / 256, 256, 0, s>>>(w, out);              \
        }                                                                                      \
        return true;                                                                           \
    }
    NSM_STAGES(NSM_PCASE)
#undef NSM_PCASE
    return false;
}

}  // namespace

bool conv_supported(const ConvStage& st, Dt dt, OutMode mode, bool in_f32) {
#define NSM_SCASE(CS_, CU_, CO_, MODE_, F32_, TH_)                                             \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_ && mode == OutMode::MODE_ && in_f32 == F32_) \
        return true;
    NSM_STAGES(NSM_SCASE)
#undef NSM_SCASE
    (void)dt;
    return false;
}

size_t packed_weight_bytes(const ConvStage& st, Dt dt) {
    size_t b = 0;
    bool ok = false;
    switch (dt) {
        case Dt::F32: ok = pack_dispatch<Dt::F32>(st, nullptr, nullptr, nullptr, &b); break;
        case Dt::BF16: ok = pack_dispatch<Dt::BF16>(st, nullptr, nullptr, nullptr, &b); break;
        case Dt::F16: ok = pack_dispatch<Dt::F16>(st, nullptr, nullptr, nullptr, &b); break;
    }
    return ok ? b : 0;
}

hipError_t pack_weights(const ConvStage& st, Dt dt, const float* w_ohwi, void* packed, hipStream_t s) {
    bool ok = false;
    switch (dt) {
        case Dt::F32: ok = pack_dispatch<Dt::F32>(st, w_ohwi, packed, s, nullptr); break;
        case Dt::BF16: ok = pack_dispatch<Dt::BF16>(st, w_ohwi, packed, s, nullptr); break;
        case Dt::F16: ok = pack_dispatch<Dt::F16>(st, w_ohwi, packed, s, nullptr); break;
    }
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t conv_forward(const ConvStage& st, Dt dt, OutMode mode, const ConvArgs& a, hipStream_t s) {
    bool found = false;
    hipError_t e = hipErrorInvalidValue;
    switch (dt) {
        case Dt::F32: e = launch<Dt::F32>(st, mode, a, s, &found); break;
        case Dt::BF16: e = launch<Dt::BF16>(st, mode, a, s, &found); break;
        case Dt::F16: e = launch<Dt::F16>(st, mode, a, s, &found); break;
    }
    return found ? e : hipErrorInvalidValue;
}

}  // namespace nsm
