// Fused 3x3 convolution stages of the shadow U-Net as MFMA implicit GEMM.
//
// The network (paper Sec. 3.5) is a U-Net trimmed to one 3x3 convolution per
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
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace nsm {
namespace ck {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <Dt D> struct DT;
template <> struct DT<Dt::F32> { using T = float; static constexpr int EPB = 4; };
template <> struct DT<Dt::BF16> { using T = __bf16; static constexpr int EPB = 8; };
template <> struct DT<Dt::F16> { using T = _Float16; static constexpr int EPB = 8; };
// 8-bit temporary storage: bfloat16 in LDS and in the MFMAs, FP8 E4M3 in
// global memory (ST below).
template <> struct DT<Dt::F8> { using T = __bf16; static constexpr int EPB = 8; };

// One FP8 E4M3 (OCP: bias 7, 3 mantissa bits, max 448, no infinities) value.
struct e4m3 {
    unsigned char bits;
};
// FP8 compute form: E4M3 in LDS and in the MFMAs, a block holds 16 values.
template <> struct DT<Dt::F8M> { using T = e4m3; static constexpr int EPB = 16; };

// Storage type of activations in global memory: the compute type, except
// for the 8-bit storage form.
template <Dt D> struct ST { using S = typename DT<D>::T; };
template <> struct ST<Dt::F8> { using S = e4m3; };
template <> struct ST<Dt::F8M> { using S = e4m3; };

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

// LDS tiles of the conv kernels are block-major: one plane per 16-byte
// channel block, pixel-consecutive inside the plane, planes a multiple of
// 256 bytes (16 pixels) apart.  In the main loops the four 16-lane groups of
// a wave read different blocks (or taps) of the same 16 pixels; measured on
// gfx950, ds_read_b128 is conflict-free when the groups' planes are 256-byte
// aligned apart, while a pixel-major layout (blocks of a pixel 16 bytes
// apart) costs a second pass on every read.
template <Dt D>
__host__ __device__ constexpr int plane_stride(int npix) {
    return (npix + 15) / 16 * 16 * DT<D>::EPB;
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
__device__ __forceinline__ float to_f(e4m3 v) { return __builtin_amdgcn_cvt_f32_fp8((int)v.bits, 0); }

template <typename T> __device__ __forceinline__ T from_f(float v);
template <> __device__ __forceinline__ float from_f<float>(float v) { return v; }
template <> __device__ __forceinline__ __bf16 from_f<__bf16>(float v) { return (__bf16)v; }
template <> __device__ __forceinline__ _Float16 from_f<_Float16>(float v) { return (_Float16)v; }

// float -> E4M3: saturate to +-448, then the hardware conversion (round to
// nearest, ties to even).
template <> __device__ __forceinline__ e4m3 from_f<e4m3>(float v) {
    const float c = __builtin_amdgcn_fmed3f(v, 448.0f, -448.0f);
    return e4m3{(unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(c, c, 0, false) & 0xFF)};
}

// Four floats -> four E4M3 bytes (v[0] in the lowest byte).
__device__ __forceinline__ unsigned int pack4_e4m3(const float* v) {
    float c[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) c[e] = __builtin_amdgcn_fmed3f(v[e], 448.0f, -448.0f);
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], w, true);
    return (unsigned int)w;
}

// Eight E4M3 bytes -> eight bfloat16 (exact: every E4M3 value is a bfloat16).
__device__ __forceinline__ u32x4 widen8_e4m3(unsigned int lo, unsigned int hi) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 a = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(lo, 1.0f, false);
    const bf16x2 b = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(lo, 1.0f, true);
    const bf16x2 c = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(hi, 1.0f, false);
    const bf16x2 d = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(hi, 1.0f, true);
    return u32x4{__builtin_bit_cast(unsigned int, a), __builtin_bit_cast(unsigned int, b),
                 __builtin_bit_cast(unsigned int, c), __builtin_bit_cast(unsigned int, d)};
}

template <Dt D>
__device__ __forceinline__ f32x4 mfma_kgroup(const u32x4& wa, const u32x4& xb, f32x4 acc) {
    if constexpr (D == Dt::F32) {
        const f32x4 a = __builtin_bit_cast(f32x4, wa);
        const f32x4 b = __builtin_bit_cast(f32x4, xb);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b[3], acc, 0, 0, 0);
    } else if constexpr (D == Dt::BF16 || D == Dt::F8) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, wa),
                                                      __builtin_bit_cast(bf16x8, xb), acc, 0, 0, 0);
    } else if constexpr (D == Dt::F8M) {
        // a block of 16 E4M3 values feeds two K = 32 FP8 MFMAs: bytes 0-7 of
        // every lane group, then bytes 8-15 (weights and pixels split alike)
        const long a0 = (long)(((unsigned long)wa[1] << 32) | wa[0]), a1 = (long)(((unsigned long)wa[3] << 32) | wa[2]);
        const long b0 = (long)(((unsigned long)xb[1] << 32) | xb[0]), b1 = (long)(((unsigned long)xb[3] << 32) | xb[2]);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, acc, 0, 0, 0);
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
    if constexpr (D == Dt::F8M)
        return u32x4{pack4_e4m3(v), pack4_e4m3(v + 4), pack4_e4m3(v + 8), pack4_e4m3(v + 12)};
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

// Raw buffer access: a resource over [base, base + 2 GiB) in scalar registers
// and a byte offset split into a per-lane part and a scalar part, so a load
// or store whose scalar part is a compile-time constant costs no vector ALU
// for its address.  Reads past the range return zero.
constexpr int kBufWord3 = 0x00020000;   // raw 32-bit data format
// v summed over the wave's four 16-lane rows: every lane gets
// (v_r0 + v_r1) + (v_r2 + v_r3) of its position within the row (the same
// values as v + xor-16 shuffle, then + xor-32 shuffle, by commutativity),
// from two VALU row swaps instead of two LDS permutes.
__device__ __forceinline__ float sum_rows4(float v) {
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    const float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(s), __float_as_uint(s), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, kBufWord3);
}
__device__ __forceinline__ u32x4 buf_load16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
}

// One block of EPB activations at byte offset voff of a storage-type tensor,
// as EPB compute-type values (16 bytes): a 16-byte load, or for the 8-bit
// storage form an 8-byte load widened to bfloat16.
template <Dt D>
__device__ __forceinline__ u32x4 load_blk(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    if constexpr (D == Dt::F8) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 q = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        return widen8_e4m3(q[0], q[1]);
    } else {
        return buf_load16(r, voff, soff);
    }
}
// Bytes of one block in global memory.
template <Dt D> constexpr int blk_bytes() { return DT<D>::EPB * (int)sizeof(typename ST<D>::S); }

// Four consecutive channels (converted to T) as one 8- or 16-byte buffer store.
template <typename T>
__device__ __forceinline__ void buf_store4(__amdgpu_buffer_rsrc_t r, int voff, int soff, const f32x4& v) {
    T t4[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) t4[e] = from_f<T>(v[e]);
    if constexpr (sizeof(T) == 4) {
        u32x4 q;
        __builtin_memcpy(&q, t4, 16);
        __builtin_amdgcn_raw_buffer_store_b128(q, r, voff, soff, 0);
    } else if constexpr (sizeof(T) == 1) {
        const float f4[4] = {v[0], v[1], v[2], v[3]};
        __builtin_amdgcn_raw_buffer_store_b32(pack4_e4m3(f4), r, voff, soff, 0);
    } else {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        u32x2 q;
        __builtin_memcpy(&q, t4, 8);
        __builtin_amdgcn_raw_buffer_store_b64(q, r, voff, soff, 0);
    }
}

// Sigmoid with the hardware reciprocal (within 1 ulp of 1 / (1 + e^-x)).
__device__ __forceinline__ float sigmoid_fast(float x) {
    return __builtin_amdgcn_rcpf(1.0f + __expf(-x));
}

// Global -> LDS copy of N1 + N2 16-byte items by the whole block: every load
// of a thread is issued before its first LDS store, so the tile costs about
// one memory latency instead of one per item.  src(idx) returns the item,
// dst(idx, v) stores it.
template <int N1, int N2, class S1, class D1, class S2, class D2>
__device__ __forceinline__ void copy_batched(S1 src1, D1 dst1, S2 src2, D2 dst2) {
    constexpr int P1 = (N1 + kThreads - 1) / kThreads, P2 = (N2 + kThreads - 1) / kThreads;
    u32x4 v1[P1 > 0 ? P1 : 1], v2[P2 > 0 ? P2 : 1];
#pragma unroll
    for (int k = 0; k < P1; ++k) {
        const int idx = threadIdx.x + k * kThreads;
        if (idx < N1) v1[k] = src1(idx);
    }
#pragma unroll
    for (int k = 0; k < P2; ++k) {
        const int idx = threadIdx.x + k * kThreads;
        if (idx < N2) v2[k] = src2(idx);
    }
#pragma unroll
    for (int k = 0; k < P1; ++k) {
        const int idx = threadIdx.x + k * kThreads;
        if (idx < N1) dst1(idx, v1[k]);
    }
#pragma unroll
    for (int k = 0; k < P2; ++k) {
        const int idx = threadIdx.x + k * kThreads;
        if (idx < N2) dst2(idx, v2[k]);
    }
}

// Row-structured variant for tiles whose rows are contiguous runs of K
// 16-byte chunks in global memory: thread t copies chunk t % K of rows
// t / K, t / K + R, ... (R = 256 / K rows per pass), so the only per-item
// index arithmetic is one division at the start and the per-pass offsets are
// uniform.  ld(r, k) loads chunk k of row r, st(r, k, v) stores it; both
// tiles' loads are all issued before the first store.
// Rows longer than the block are split into NS equal pieces (virtual rows).
template <int ROWS1, int K1, int ROWS2, int K2, class L1, class S1, class L2, class S2>
__device__ __forceinline__ void copy_rows2(L1 ld1, S1 st1, L2 ld2, S2 st2, int tid);

__host__ __device__ constexpr int row_pieces(int k) {
    int ns = (k + kThreads - 1) / kThreads;
    while (k % ns != 0) ++ns;
    return ns;
}

template <int K>
struct RowSplit {
    static constexpr int NS = row_pieces(K);      // fewest equal pieces of at most kThreads chunks
    static constexpr int KP = K / NS;
};

template <int ROWS1, int K1, int ROWS2, int K2, class L1, class S1, class L2, class S2>
__device__ __forceinline__ void copy_rows2_split(L1 ld1, S1 st1, L2 ld2, S2 st2, int tid) {
    using A = RowSplit<K1>;
    using B = RowSplit<K2>;
    auto l1 = [&](int vr, int k) { return ld1(vr / A::NS, (vr % A::NS) * A::KP + k); };
    auto s1 = [&](int vr, int k, const u32x4& v) { st1(vr / A::NS, (vr % A::NS) * A::KP + k, v); };
    auto l2 = [&](int vr, int k) { return ld2(vr / B::NS, (vr % B::NS) * B::KP + k); };
    auto s2 = [&](int vr, int k, const u32x4& v) { st2(vr / B::NS, (vr % B::NS) * B::KP + k, v); };
    copy_rows2<ROWS1 * A::NS, A::KP, ROWS2 * B::NS, B::KP>(l1, s1, l2, s2, tid);
}

template <int ROWS1, int K1, int ROWS2, int K2, class L1, class S1, class L2, class S2>
__device__ __forceinline__ void copy_rows2(L1 ld1, S1 st1, L2 ld2, S2 st2, int tid) {
    if constexpr (K1 > kThreads || K2 > kThreads) {
        copy_rows2_split<ROWS1, K1, ROWS2, K2>(ld1, st1, ld2, st2, tid);
        return;
    } else {
    constexpr int R1 = kThreads / K1, R2 = kThreads / K2;
    constexpr int P1 = (ROWS1 + R1 - 1) / R1, P2 = (ROWS2 + R2 - 1) / R2;
    const int k1 = tid % K1, r1 = tid / K1;
    const int k2 = tid % K2, r2 = tid / K2;
    // loads are unconditional (rows clamped into the tile) so that no value
    // has to be merged across branches; only the stores are predicated
    u32x4 v1[P1], v2[P2];
#pragma unroll
    for (int p = 0; p < P1; ++p) v1[p] = ld1(min(r1 + p * R1, ROWS1 - 1), k1);
#pragma unroll
    for (int p = 0; p < P2; ++p) v2[p] = ld2(min(r2 + p * R2, ROWS2 - 1), k2);
#pragma unroll
    for (int p = 0; p < P1; ++p)
        if (r1 < R1 && r1 + p * R1 < ROWS1) st1(r1 + p * R1, k1, v1[p]);
#pragma unroll
    for (int p = 0; p < P2; ++p)
        if (r2 < R2 && r2 + p * R2 < ROWS2) st2(r2 + p * R2, k2, v2[p]);
    }
}

// One tile only; loads and stores go in batches of at most MAXP passes (the
// staging registers a batch needs).
template <int ROWS, int K, int MAXP = 64, class L, class S>
__device__ __forceinline__ void copy_rows1(L ld, S st, int tid) {
    if constexpr (K > kThreads) {
        using A = RowSplit<K>;
        auto l = [&](int vr, int k) { return ld(vr / A::NS, (vr % A::NS) * A::KP + k); };
        auto s = [&](int vr, int k, const u32x4& v) { st(vr / A::NS, (vr % A::NS) * A::KP + k, v); };
        copy_rows1<ROWS * A::NS, A::KP, MAXP>(l, s, tid);
    } else {
        constexpr int R = kThreads / K, P = (ROWS + R - 1) / R;
        constexpr int PB = P < MAXP ? P : MAXP;
        const int k = tid % K, r0 = tid / K;
#pragma unroll
        for (int p0 = 0; p0 < P; p0 += PB) {
            u32x4 v[PB];
#pragma unroll
            for (int p = 0; p < PB; ++p) v[p] = ld(min(r0 + (p0 + p) * R, ROWS - 1), k);
#pragma unroll
            for (int p = 0; p < PB; ++p)
                if (p0 + p < P && r0 < R && r0 + (p0 + p) * R < ROWS) st(r0 + (p0 + p) * R, k, v[p]);
        }
    }
}

// Low-res source tile of the upsampled channels: rows/cols y0/2-1 .. y0/2+TH/2
// (x likewise), each clamped to the low-res image, LCST elements per pixel.
template <Dt D, int CU, int TH>
struct LowTile {
    static constexpr int LH = TH / 2 + 2, LW = kTW / 2 + 2;
    static constexpr int LCST = CU > 0 ? lds_stride<D>(CU) : 1;
    static constexpr int SIZE = CU > 0 ? LH * LW * LCST : 1;
};

// Halo tile (TH+2) x (kTW+2) pixels of the stage input -> LDS, in the
// compute dtype, block b of pixel p at element p * PXS + b * BKS (block-major
// planes: PXS = EPB, BKS = plane stride): channels [0, CS) from `in` ([n][h][w][CS],
// float32 when IN_F32, zero-padded up to a whole block), channels
// [CSP, CSP+CU) from the bilinear x2 upsampling of `low` ([n][h/2][w/2][CU]):
// (an `in` in the stage dtype holds CSP channels per pixel, those past CS
// zero: a first stage reading features already in the storage type)
// source row s = (y + 0.5)/2 - 0.5, taps floor(s) (weight 0.25 for even y,
// 0.75 for odd y) and floor(s) + 1, both clamped to the low-res image; the
// same along x.  Pixels outside the image are zero (the conv's padding).
// The low-res source rows are first staged in `lowt` (each read once from
// global memory), then every upsampled value is formed from LDS.  Ends with
// a barrier: the tile is ready when it returns.
// With SUM the upsampled channels are added to channels [0, CU) of `in`
// (CU == CS) instead of being appended: the skip merge by algebraic sum.
// With S2D, `in` is the float32 full-resolution input [n][2h][2w][CS/4] read
// through space-to-depth: channel (2 dy + dx) CS/4 + c of pixel (y, x) is
// channel c of input pixel (2y + dy, 2x + dx), so every block of channels is
// one contiguous run of an input row.
template <Dt D, bool IN_F32, int CS, int CU, int PXS, int BKS, int TH, bool SUM = false, bool S2D = false>
__device__ __forceinline__ void load_halo_tile(typename DT<D>::T* tile, typename DT<D>::T* lowt,
                                               const void* in, const void* low, int n, int h, int w,
                                               int x0, int y0) {
    using T = typename DT<D>::T;
    using LT = LowTile<D, CU, TH>;
    constexpr int EPB = DT<D>::EPB;
    constexpr int CSP = round_up(CS, EPB);
    static_assert(!SUM || CS == CU, "a sum skip needs equal channel counts");
    static_assert(!S2D || (IN_F32 && CS == 16), "space-to-depth reads 4-channel float32 input");
    constexpr int WP = kTW + 2, NPIX = (TH + 2) * WP;
    constexpr int NCH_S = CSP / EPB, NCH_U = CU / EPB;
    // phase 1: same-resolution channels, and the low-res source rows.
    // Buffer offsets are relative to each tile's first (halo) pixel, taken
    // at clamped coordinates; pixels outside the image then read as zero.
    using S = typename ST<D>::S;
    constexpr int SB = (int)sizeof(S);                              // bytes per stored element
    constexpr int SZ_IN = IN_F32 ? 4 : SB;
    constexpr int CST = IN_F32 ? CS : CSP;                          // stored channels per pixel
    constexpr int SPX = S2D ? 2 * (CS / 4) * 4 : CST * SZ_IN;         // bytes per pixel step
    const int srow = S2D ? 2 * (2 * w) * (CS / 4) * 4 : w * CST * SZ_IN;  // bytes per row step
    const char* sbase = reinterpret_cast<const char*>(in) + ((long long)n * h + y0 - 1) * srow +
                        (long long)(x0 - 1) * SPX;
    const __amdgpu_buffer_rsrc_t sr = buf_rsrc(sbase);
    auto skip_ld = [&](int r, int k) -> u32x4 {
        const int ch = k / WP, c = k - ch * WP;       // block-major: see the copy note below
        const int y = y0 + r - 1, x = x0 + c - 1;
        const bool ok = y >= 0 && y < h && x >= 0 && x < w;
        const int yr = min(max(y, 0), h - 1) - (y0 - 1), xr = min(max(x, 0), w - 1) - (x0 - 1);
        const int voff = yr * srow + xr * SPX;
        u32x4 v;
        if constexpr (S2D) {
            // channels [ch EPB, ch EPB + EPB): input row 2y + (ch EPB) / 8, floats
            // (ch EPB) % 8 .. of the two pixels 2x, 2x + 1
            const int off = voff + ((ch * EPB) >> 3) * (srow >> 1) + ((ch * EPB) & 7) * 4;
            float f[EPB];
#pragma unroll
            for (int q = 0; q < EPB / 4; ++q) {
                // copied as bytes: a bit_cast of a vector element here read element 0
                // for every e
                const u32x4 u = buf_load16(sr, off + 16 * q, 0);
                __builtin_memcpy(&f[4 * q], &u, 16);
            }
            v = pack_block<D>(f);
        } else if constexpr (IN_F32) {
            // float32 features: EPB channels of block ch, zero past CS
            float f[EPB];
#pragma unroll
            for (int e = 0; e < EPB; e += 2) {
                const int c0 = ch * EPB + e;
                if (c0 + 1 < CS) {
                    typedef float f32x2 __attribute__((ext_vector_type(2)));
                    const f32x2 q = __builtin_bit_cast(
                        f32x2, __builtin_amdgcn_raw_buffer_load_b64(sr, voff + c0 * 4, 0, 0));
                    f[e] = q[0];
                    f[e + 1] = q[1];
                } else {
                    f[e] = (c0 < CS) ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(sr, voff + c0 * 4, 0, 0))
                                     : 0.0f;
                    f[e + 1] = 0.0f;
                }
            }
            v = pack_block<D>(f);
        } else {
            v = load_blk<D>(sr, voff + ch * blk_bytes<D>(), 0);
        }
        return ok ? v : u32x4{0u, 0u, 0u, 0u};
    };
    auto skip_st = [&](int r, int k, const u32x4& v) {
        const int ch = k / WP, c = k - ch * WP;       // block-major: see the copy note below
        *reinterpret_cast<u32x4*>(&tile[(r * WP + c) * PXS + ch * BKS]) = v;
    };
    const int hl = h >> 1, wl = w >> 1;
    const int ly0 = (y0 >> 1) - 1, lx0 = (x0 >> 1) - 1;
    const char* lbase = reinterpret_cast<const char*>(low) +
                        ((((long long)n * hl + ly0) * wl + lx0) * CU) * (long long)SB;
    const __amdgpu_buffer_rsrc_t lr = buf_rsrc(lbase);
    const int lrow = wl * CU * SB;
    auto low_ld = [&](int r, int k) -> u32x4 {
        const int ch = k / LT::LW, c = k - ch * LT::LW;
        const int gy = min(max(ly0 + r, 0), hl - 1) - ly0, gx = min(max(lx0 + c, 0), wl - 1) - lx0;
        return load_blk<D>(lr, gy * lrow + gx * (CU * SB) + ch * blk_bytes<D>(), 0);
    };
    auto low_st = [&](int r, int k, const u32x4& v) {
        const int ch = k / LT::LW, c = k - ch * LT::LW;
        *reinterpret_cast<u32x4*>(&lowt[(r * LT::LW + c) * LT::LCST + ch * EPB]) = v;
    };
    // Copy note: chunk k of a tile row is block ch = k / (pixels per row) of
    // pixel c = k % (pixels per row), so that consecutive lanes store the same
    // block of consecutive pixels: LDS addresses an odd number of 16-byte
    // units apart, which never share a bank group (pixel-major chunks put the
    // blocks of neighbouring pixels on the same banks).  The wave's loads
    // still cover whole runs of pixels in global memory.
    if constexpr (NCH_S > 0 && CU > 0)
        copy_rows2<TH + 2, WP * NCH_S, LT::LH, LT::LW * NCH_U>(skip_ld, skip_st, low_ld, low_st, threadIdx.x);
    else if constexpr (NCH_S > 0)
        copy_rows1<TH + 2, WP * NCH_S>(skip_ld, skip_st, threadIdx.x);
    else if constexpr (CU > 0)
        copy_rows1<LT::LH, LT::LW * NCH_U>(low_ld, low_st, threadIdx.x);
    if constexpr (CU > 0) {
        __syncthreads();
        // phase 2: upsampled channels from the staged rows, pixel-fastest so
        // that a wave writes consecutive pixels of one block
        for (int idx = threadIdx.x; idx < NPIX * NCH_U; idx += kThreads) {
            const int ch = idx / NPIX, pix = idx - ch * NPIX;
            const int ty = pix / WP, tx = pix - ty * WP;
            const int y = y0 + ty - 1, x = x0 + tx - 1;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (y >= 0 && y < h && x >= 0 && x < w) {
                const int ra = ((y - 1) >> 1) - ly0, ca = ((x - 1) >> 1) - lx0;
                const float wy0 = (y & 1) ? 0.75f : 0.25f, wx0 = (x & 1) ? 0.75f : 0.25f;
                const float wy1 = 1.0f - wy0, wx1 = 1.0f - wx0;
                const T* l00 = &lowt[(ra * LT::LW + ca) * LT::LCST + ch * EPB];
                float f00[EPB], f01[EPB], f10[EPB], f11[EPB], f[EPB];
                unpack_block<D>(*reinterpret_cast<const u32x4*>(l00), f00);
                unpack_block<D>(*reinterpret_cast<const u32x4*>(l00 + LT::LCST), f01);
                unpack_block<D>(*reinterpret_cast<const u32x4*>(l00 + LT::LW * LT::LCST), f10);
                unpack_block<D>(*reinterpret_cast<const u32x4*>(l00 + (LT::LW + 1) * LT::LCST), f11);
#pragma unroll
                for (int e = 0; e < EPB; ++e)
                    f[e] = wy0 * (wx0 * f00[e] + wx1 * f01[e]) + wy1 * (wx0 * f10[e] + wx1 * f11[e]);
                if constexpr (SUM) {
                    float sk[EPB];
                    unpack_block<D>(*reinterpret_cast<const u32x4*>(&tile[pix * PXS + ch * BKS]), sk);
#pragma unroll
                    for (int e = 0; e < EPB; ++e) f[e] = sk[e] + f[e];
                }
                v = pack_block<D>(f);
            }
            *reinterpret_cast<u32x4*>(&tile[pix * PXS + ((SUM ? 0 : NCH_S) + ch) * BKS]) = v;
        }
    }
    __syncthreads();
}

// Hardware dispatches consecutive workgroups round-robin over the 8 XCDs;
// give each XCD a contiguous run of logical tiles so that neighbouring
// tiles (which share halo rows and low-res rows) meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int total) {
    const int xcd = b & 7, k = b >> 3;
    const int q = total >> 3, r = total & 7;
    return xcd * q + min(xcd, r) + k;
}

// Border tiles of a phase-form decoder launch (conv_up.h): the phase kernel
// covers the tiles of a band x 32 tiling that are at least one tile away from
// every edge; this maps a linear index over the rest, in tiles of TH x 32
// (band is a multiple of TH), to (x0, y0, n): the top band, the bottom band,
// then the first and last tile columns in between.
__host__ __device__ __forceinline__ int border_tiles_per_image(int band, int th, int h, int w) {
    const int gx = (w + kTW - 1) / kTW, gyb = (h + band - 1) / band, ylast = (gyb - 1) * band;
    return (band / th) * gx + ((h - ylast + th - 1) / th) * gx + ((ylast - band) / th) * 2;
}

__device__ __forceinline__ void border_tile(int lt, int band, int th, int h, int w, int* x0, int* y0, int* n) {
    const int gx = (w + kTW - 1) / kTW, gyb = (h + band - 1) / band, ylast = (gyb - 1) * band;
    const int top = (band / th) * gx, bot = ((h - ylast + th - 1) / th) * gx;
    const int per = border_tiles_per_image(band, th, h, w);
    *n = lt / per;
    int r = lt - *n * per;
    if (r < top) {
        *y0 = (r / gx) * th;
        *x0 = (r % gx) * kTW;
    } else if (r - top < bot) {
        r -= top;
        *y0 = ylast + (r / gx) * th;
        *x0 = (r % gx) * kTW;
    } else {
        r -= top + bot;
        *y0 = band + (r >> 1) * th;
        *x0 = (r & 1) ? (gx - 1) * kTW : 0;
    }
}

// Store four consecutive channels co..co+3 (fewer at the end of an odd-sized
// channel vector) of one pixel.
template <typename T, int CO>
__device__ __forceinline__ void store4(T* dst, int co, const float* v) {
    T t4[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) t4[e] = from_f<T>(v[e]);
    if constexpr (CO % 4 != 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (co + e < CO) dst[e] = t4[e];
    } else if constexpr (sizeof(T) == 4) {
        f32x4 q;
        __builtin_memcpy(&q, t4, 16);
        *reinterpret_cast<f32x4*>(dst) = q;
    } else if constexpr (sizeof(T) == 1) {
        *reinterpret_cast<unsigned int*>(dst) = pack4_e4m3(v);
    } else {
        uint2 q;
        __builtin_memcpy(&q, t4, 8);
        *reinterpret_cast<uint2*>(dst) = q;
    }
}

// LDS elements of one tile of the general kernel (halo tile, then low rows).
template <Dt D, int CS, int CU, int CO, int TH>
struct GenTile {
    static constexpr int PS = plane_stride<D>((TH + 2) * (kTW + 2));
    static constexpr int TILE = Geo<D, CS, CU, CO>::BPT * PS;
    static constexpr int LOW = LowTile<D, CU, TH>::SIZE;
    static constexpr int LOW_OFF = (TILE + 7) / 8 * 8;   // 16-byte aligned for every storage type
    static constexpr int ELEMS = LOW_OFF + LOW;
};

// One TH x 32 output tile at (x0, y0) of image n: the whole stage for it.
template <Dt D, bool IN_F32, int CS, int CU, int CO, OutMode MODE, int TH>
__device__ __forceinline__ void conv_tile(const ConvArgs& a, int x0, int y0, int n,
                                          typename DT<D>::T* tile, typename DT<D>::T* lowt) {
    using T = typename DT<D>::T;
    using G = Geo<D, CS, CU, CO>;
    constexpr int EPB = G::EPB, NKG = G::NKG, NF = G::NF, BPT = G::BPT, NB = G::NB;
    constexpr int PS = GenTile<D, CS, CU, CO, TH>::PS;
    constexpr int WP = kTW + 2;
    constexpr int RPW = TH / 4;                 // rows per wave
    constexpr int MF = RPW * 2;                 // M-fragments per wave
    static_assert(MODE != OutMode::Pool || RPW % 2 == 0, "pooling needs whole row pairs per wave");
    const int h = a.h, w = a.w;

    // ---------------- prologue: halo tile to LDS
    load_halo_tile<D, IN_F32, CS, CU, EPB, PS, TH>(tile, lowt, a.in, a.low, n, h, w, x0, y0);

    // ---------------- main loop
    // the wave index is uniform in the wave: keep it in a scalar register
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int px = lane & 15, g = lane >> 4;
    const __amdgpu_buffer_rsrc_t wr = buf_rsrc(a.wpk);
    const int wl16 = lane * 16;
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
        for (int f = 0; f < NF; ++f) dst[f] = buf_load16(wr, wl16, (f * NKG + q) * 1024);
    };
#pragma unroll
    for (int q = 0; q < PD && q < NKG; ++q) wload(q, wbuf[q]);
#pragma unroll
    for (int q = 0; q < NKG; ++q) {
        if (q + PD < NKG) wload(q + PD, wbuf[(q + PD) % (PD + 1)]);
        const u32x4 (&wf)[NF] = wbuf[q % (PD + 1)];
        int b = 4 * q + g;
        if (b >= NB) b = NB - 1;               // padding k: weights are zero there
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

    // ---------------- epilogue
    if constexpr (MODE != OutMode::Linear) {
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
    }

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
            s = sum_rows4(s);
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
        using S = typename ST<D>::S;
        S* out = reinterpret_cast<S*>(a.out);
#pragma unroll
        for (int m = 0; m < MF; ++m) {
            const int y = y0 + wave * RPW + (m >> 1), x = x0 + (m & 1) * 16 + px;
            if (y < h && x < w) {
                const size_t p = ((size_t)n * h + y) * w + x;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const int co = f * 16 + 4 * g;
                    if (co < CO) {
                        float v4[4] = {acc[m][f][0], acc[m][f][1], acc[m][f][2], acc[m][f][3]};
                        store4<S, CO>(out + p * CO + co, co, v4);
                    }
                }
            }
        }
        if constexpr (MODE == OutMode::Pool) {
            S* pooled = reinterpret_cast<S*>(a.pooled);
            const int hp = h >> 1, wp = w >> 1;
            // row pair pr of this wave = fragments 4 pr + cf (upper row) and 4 pr + 2 + cf
#pragma unroll
            for (int pr = 0; pr < RPW / 2; ++pr)
#pragma unroll
            for (int cf = 0; cf < 2; ++cf) {
                const int yp = (y0 >> 1) + wave * (RPW / 2) + pr, xp = ((x0 + cf * 16 + px) >> 1);
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    // 2x2 max of ReLU outputs: non-negative and never NaN, so
                    // their float order is the order of their bit patterns as
                    // signed integers (a -0 sorts below +0 and pools to the
                    // same value); integer max needs no NaN canonicalisation,
                    // and the neighbouring column is lane ^ 1 (a DPP quad
                    // permute instead of an LDS shuffle)
                    float mx[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int v = max(__float_as_int(acc[4 * pr + cf][f][e]),
                                          __float_as_int(acc[4 * pr + 2 + cf][f][e]));
                        const int o = __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
                        mx[e] = __int_as_float(max(v, o));
                    }
                    const int co = f * 16 + 4 * g;
                    if ((px & 1) == 0 && yp < hp && xp < wp && co < CO) {
                        const size_t p = ((size_t)n * hp + yp) * wp + xp;
                        store4<S, CO>(pooled + p * CO + co, co, mx);
                    }
                }
            }
        }
    }
}

template <Dt D, bool IN_F32, int CS, int CU, int CO, OutMode MODE, int TH>
__global__ void __launch_bounds__(kThreads) k_conv3x3(ConvArgs a) {
    using T = typename DT<D>::T;
    using GT = GenTile<D, CS, CU, CO, TH>;
    __shared__ __attribute__((aligned(16))) T smem[GT::ELEMS];
    const int gx = gridDim.x, gy = gridDim.y;
    const int lt = xcd_remap(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    conv_tile<D, IN_F32, CS, CU, CO, MODE, TH>(a, (lt % gx) * kTW, ((lt / gx) % gy) * TH, lt / (gx * gy), smem,
                                               smem + GT::LOW_OFF);
}

// Persistent form of k_conv3x3: a grid sized to the resident capacity of the
// device (a multiple of 8, so that block b stays on XCD b % 8) walks the
// gx x gy x n tiles with a stride of the grid; the per-tile work and its
// arithmetic are those of k_conv3x3, so both give the same bits.
template <Dt D, bool IN_F32, int CS, int CU, int CO, OutMode MODE, int TH>
__global__ void __launch_bounds__(kThreads) k_conv3x3_persist(ConvArgs a, int gx, int gy) {
    using T = typename DT<D>::T;
    using GT = GenTile<D, CS, CU, CO, TH>;
    __shared__ __attribute__((aligned(16))) T smem[GT::ELEMS];
    const int total = gx * gy * a.n;
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        if (b != (int)blockIdx.x) __syncthreads();     // the previous tile's LDS reads are done
        const int lt = xcd_remap(b, total);
        conv_tile<D, IN_F32, CS, CU, CO, MODE, TH>(a, (lt % gx) * kTW, ((lt / gx) % gy) * TH, lt / (gx * gy), smem,
                                                   smem + GT::LOW_OFF);
    }
}

// Weight repack: OHWI float32 [CO][3][3][CS+CU] -> [NF][NKG][64 lanes][EPB]
// storage type.  With FLIP the source is the forward weight W[CI'][3][3][CO']
// of a stage whose input gradient this conv computes: the packed kernel is
// W'[co][ky][kx][ci] = W[ci][2-ky][2-kx][co] (CS = CO', CO = CI', CU = 0).
template <Dt D, int CS, int CU, int CO, bool FLIP = false>
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
        if (ci >= 0) {
            if constexpr (FLIP)
                v = w[((size_t)ci * 9 + (8 - tap)) * CO + co];
            else
                v = w[((size_t)co * 9 + tap) * (CS + CU) + ci];
        }
    }
    reinterpret_cast<T*>(out)[idx] = from_f<T>(v);
}

template <Dt D, int CS, int CU, int CO>
constexpr size_t packed_bytes() {
    using G = Geo<D, CS, CU, CO>;
    return (size_t)G::NF * G::NKG * 64 * 16;
}

}  // namespace ck
}  // namespace nsm
