// Forward dispatch of the fused conv stages (kernels in conv_kernels.h and,
// for decoder stages, the phase form of conv_up.h plus the general kernel on
// the border bands).
#include <hip/hip_runtime.h>

#include "conv_kernels.h"
#include "conv_up.h"

namespace nsm {
namespace {
using namespace ck;
// ---------------------------------------------------------------- dispatch
// Supported stages: (cs, cu, co, mode, float32 input, tile rows, alternative
// tile rows, features stored in the stage dtype) per dtype.  For decoder stages the tile rows
// are those of the general kernel's border tiles (the phase-form interior
// keeps its own);
// 4 rows keep the 16+32 stage's border tile below its phase tile in LDS, so
// that four blocks fit per CU (the 32+64 stage has no taller border tile:
// at 8 rows its float32 tile exceeds the LDS).  A launch variant (0..3) picks, bit 0, the
// persistent grid and, bit 1, the alternative tile rows; every variant
// computes each output pixel with the same arithmetic in the same order, so
// all give the same bits (the phase-form interior is the same in all).
// The first stages also read features already stored in the stage dtype
// (stored: whole 16-byte blocks per pixel, the channels past the stage's
// inputs zero), which gives the same bits as the float32 input rounded to
// that dtype when the tile is staged; their trace names end in "stored".
#define NSM_STAGES(X)                           \
    X(6, 0, 16, Pool, true, 8, 16, false)       \
    X(8, 0, 16, Pool, true, 8, 16, false)       \
    X(6, 0, 16, Pool, false, 8, 16, true)       \
    X(8, 0, 16, Pool, false, 8, 16, true)       \
    X(16, 0, 32, Pool, false, 8, 16, false)     \
    X(32, 0, 64, Store, false, 8, 4, false)     \
    X(32, 64, 32, Store, false, 4, 4, false)    \
    X(16, 32, 16, Head, false, 4, 8, false)     \
    X(6, 0, 8, Pool, true, 8, 16, false)        \
    X(6, 0, 8, Pool, false, 8, 16, true)        \
    X(8, 0, 16, Store, false, 8, 4, false)      \
    X(8, 16, 8, Head, false, 8, 4, false)

template <Dt D> constexpr const char* dt_suffix() {
    return D == Dt::F32 ? " f32"
         : (D == Dt::BF16 ? " bf16" : (D == Dt::F16 ? " f16" : (D == Dt::F8 ? " f8" : " f8mfma")));
}
template <Dt D> constexpr const char* phase_suffix() {
    return D == Dt::F32 ? " phase f32"
         : (D == Dt::BF16 ? " phase bf16"
                          : (D == Dt::F16 ? " phase f16" : (D == Dt::F8 ? " phase f8" : " phase f8mfma")));
}

// The FP8 compute form packs 16 channels per block: a stage whose stored
// inputs are not whole blocks of 16 channels has no kernel in it (the
// float32 network input is padded on load, stored features by the gather).
template <Dt D, bool F32, int CS, int CU, bool STORED = false>
constexpr bool stage_fits() {
    return D != Dt::F8M || ((F32 || STORED || CS % 16 == 0) && CU % 16 == 0);
}

// Tile rows of the phase-form kernel: 16, or 8 for wide stages (96 input
// channels), whose 16-row tiles hold 75 KB of LDS and 200+ registers per
// lane in bfloat16 (two blocks per CU) and do not fit twice in float32.
template <Dt D, int CS, int CU>
constexpr int up_tile_rows() { return CS + CU >= 96 ? 8 : 16; }

constexpr size_t align256c(size_t x) { return (x + 255) & ~(size_t)255; }

template <Dt D, int CS, int CU, int CO>
constexpr size_t stage_packed_bytes() {
    size_t b = align256c(packed_bytes<D, CS, CU, CO>());
    if constexpr (CU > 0 && (D != Dt::F8M || (CS % 16 == 0 && CU % 16 == 0)))
        b += align256c(UpGeo<D, CS, CU, CO>::BYTES);
    return b;
}

// Blocks of one kernel that fit on the device at once (a multiple of 8: the
// XCD of block b is b % 8), looked up once per kernel.
template <typename K>
int resident_blocks(K kernel) {
    static const int cap = [&]() {
        int dev = 0, cus = 256, per = 1;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kThreads, 0) != hipSuccess || per < 1) per = 1;
        return ((per * cus + 7) / 8) * 8;
    }();
    return cap;
}

template <Dt D, bool F32, int CS, int CU, int CO, OutMode MODE, int TH, bool STORED = false>
hipError_t launch_stage(const ConvArgs& a, hipStream_t s, const char* name, bool persist) {
    if constexpr (!stage_fits<D, F32, CS, CU, STORED>()) {
        return hipErrorInvalidValue;
    } else {
    if constexpr (CU > 0 && !F32 && (MODE == OutMode::Store || MODE == OutMode::Head)) {
        constexpr int THU = up_tile_rows<D, CS, CU>();
        const int gxt = (a.w + kTW - 1) / kTW, gyt = (a.h + THU - 1) / THU;
        if (gxt >= 3 && gyt >= 3) {
            TraceScope ts(name, phase_suffix<D>(), s);
            const void* wup = reinterpret_cast<const char*>(a.wpk) + align256c(packed_bytes<D, CS, CU, CO>());
            const int blocks = border_tiles_per_image(THU, TH, a.h, a.w) * a.n + (gxt - 2) * (gyt - 2) * a.n;
            if (persist) {
                auto* k = k_conv3x3_up_persist<D, CS, CU, CO, MODE, THU, TH>;
                k<<<min(blocks, resident_blocks(k)), kThreads, 0, s>>>(a, wup, blocks);
            } else {
                k_conv3x3_up<D, CS, CU, CO, MODE, THU, TH><<<blocks, kThreads, 0, s>>>(a, wup);
            }
            return hipGetLastError();
        }
    }
    const int gx = (a.w + kTW - 1) / kTW, gy = (a.h + TH - 1) / TH;
    TraceScope ts(name, dt_suffix<D>(), s);
    if (persist) {
        auto* k = k_conv3x3_persist<D, F32, CS, CU, CO, MODE, TH>;
        k<<<min(gx * gy * a.n, resident_blocks(k)), kThreads, 0, s>>>(a, gx, gy);
    } else {
        k_conv3x3<D, F32, CS, CU, CO, MODE, TH><<<dim3(gx, gy, a.n), kThreads, 0, s>>>(a);
    }
    return hipGetLastError();
    }
}

template <Dt D>
hipError_t launch(const ConvStage& st, OutMode mode, const ConvArgs& a, hipStream_t s, int variant, bool* found) {
    const bool persist = (variant & 1) != 0, alt = (variant & 2) != 0;
#define NSM_CASE(CS_, CU_, CO_, MODE_, F32_, TH_, THA_, STORED_)                               \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_ && mode == OutMode::MODE_ &&             \
        a.in_f32 == F32_) {                                                                    \
        *found = true;                                                                         \
        const char* nm = STORED_ ? "conv3x3 " #CS_ "+" #CU_ "->" #CO_ " " #MODE_ " stored"     \
                                 : "conv3x3 " #CS_ "+" #CU_ "->" #CO_ " " #MODE_;              \
        if (alt)                                                                               \
            return launch_stage<D, F32_, CS_, CU_, CO_, OutMode::MODE_, THA_, STORED_>(a, s, nm, persist); \
        return launch_stage<D, F32_, CS_, CU_, CO_, OutMode::MODE_, TH_, STORED_>(a, s, nm, persist);      \
    }
    NSM_STAGES(NSM_CASE)
#undef NSM_CASE
    *found = false;
    return hipErrorInvalidValue;
}

template <Dt D, int CS, int CU, int CO>
void pack_stage(const float* w, void* out, hipStream_t s) {
    constexpr size_t nb = packed_bytes<D, CS, CU, CO>();
    constexpr int total = (int)(nb / 16 * DT<D>::EPB);
    k_pack<D, CS, CU, CO><<<(total + 255) / 256, 256, 0, s>>>(w, out);
    if constexpr (CU > 0 && (D != Dt::F8M || (CS % 16 == 0 && CU % 16 == 0))) {
        using G = UpGeo<D, CS, CU, CO>;
        constexpr int tu = (int)(G::SKIP_ELEMS + 4 * G::PHASE_ELEMS);
        k_pack_up<D, CS, CU, CO><<<(tu + 255) / 256, 256, 0, s>>>(w, reinterpret_cast<char*>(out) + align256c(nb));
    }
}

template <Dt D>
bool pack_dispatch(const ConvStage& st, const float* w, void* out, hipStream_t s, size_t* bytes) {
#define NSM_PCASE(CS_, CU_, CO_, MODE_, F32_, TH_, THA_, STORED_)                                       \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_) {                                        \
        if constexpr (!stage_fits<D, F32_, CS_, CU_>()) return false;                          \
        if (bytes) *bytes = stage_packed_bytes<D, CS_, CU_, CO_>();                            \
        if (out) pack_stage<D, CS_, CU_, CO_>(w, out, s);                                      \
        return true;                                                                           \
    }
    NSM_STAGES(NSM_PCASE)
#undef NSM_PCASE
    return false;
}

}  // namespace

bool conv_supported(const ConvStage& st, Dt dt, OutMode mode, bool in_f32) {
#define NSM_SCASE(CS_, CU_, CO_, MODE_, F32_, TH_, THA_, STORED_)                                       \
    if (st.cs == CS_ && st.cu == CU_ && st.co == CO_ && mode == OutMode::MODE_ && in_f32 == F32_) \
        return dt != Dt::F8M || stage_fits<Dt::F8M, F32_, CS_, CU_, STORED_>();
    NSM_STAGES(NSM_SCASE)
#undef NSM_SCASE
    return false;
}

size_t packed_weight_bytes(const ConvStage& st, Dt dt) {
    size_t b = 0;
    bool ok = false;
    switch (dt) {
        case Dt::F32: ok = pack_dispatch<Dt::F32>(st, nullptr, nullptr, nullptr, &b); break;
        case Dt::BF16: ok = pack_dispatch<Dt::BF16>(st, nullptr, nullptr, nullptr, &b); break;
        case Dt::F16: ok = pack_dispatch<Dt::F16>(st, nullptr, nullptr, nullptr, &b); break;
        // the 8-bit storage form keeps bfloat16 weights: the same pack
        case Dt::F8: ok = pack_dispatch<Dt::BF16>(st, nullptr, nullptr, nullptr, &b); break;
        case Dt::F8M: ok = pack_dispatch<Dt::F8M>(st, nullptr, nullptr, nullptr, &b); break;
    }
    return ok ? b : 0;
}

hipError_t pack_weights(const ConvStage& st, Dt dt, const float* w_ohwi, void* packed, hipStream_t s) {
    bool ok = false;
    switch (dt) {
        case Dt::F32: ok = pack_dispatch<Dt::F32>(st, w_ohwi, packed, s, nullptr); break;
        case Dt::BF16: ok = pack_dispatch<Dt::BF16>(st, w_ohwi, packed, s, nullptr); break;
        case Dt::F16: ok = pack_dispatch<Dt::F16>(st, w_ohwi, packed, s, nullptr); break;
        case Dt::F8: ok = pack_dispatch<Dt::BF16>(st, w_ohwi, packed, s, nullptr); break;
        case Dt::F8M: ok = pack_dispatch<Dt::F8M>(st, w_ohwi, packed, s, nullptr); break;
    }
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t conv_forward(const ConvStage& st, Dt dt, OutMode mode, const ConvArgs& a, hipStream_t s, int variant) {
    bool found = false;
    hipError_t e = hipErrorInvalidValue;
    switch (dt) {
        case Dt::F32: e = launch<Dt::F32>(st, mode, a, s, variant, &found); break;
        case Dt::BF16: e = launch<Dt::BF16>(st, mode, a, s, variant, &found); break;
        case Dt::F16: e = launch<Dt::F16>(st, mode, a, s, variant, &found); break;
        case Dt::F8: e = launch<Dt::F8>(st, mode, a, s, variant, &found); break;
        case Dt::F8M: e = launch<Dt::F8M>(st, mode, a, s, variant, &found); break;
    }
    return found ? e : hipErrorInvalidValue;
}

}  // namespace nsm
