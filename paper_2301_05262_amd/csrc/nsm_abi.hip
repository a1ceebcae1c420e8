// C-ABI entry points: argument validation, context and workspace planning,
// and the order of kernel launches for each call.  All validation happens
// before the first HIP call so that a non-OK status never leaves work on the
// stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using namespace nsm;

namespace {

constexpr int kMaxImage = 16384;
constexpr int kMaxFrames = 4096;
// Triangle counts are carried in 32-bit ints (two passes of virtual
// triangles, per-triangle offsets); 2^28 keeps every such index in range.
constexpr int kMaxTris = 1 << 28;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct StagePlan {
    const char* name;
    ConvStage st;
    OutMode mode;
    bool in_f32;
    int level;          // resolution level the stage runs at
    size_t w_off;       // offset (floats) of the OHWI weights in the flat vector
    size_t b_off;       // offset (floats) of the biases
    size_t pk_off;      // byte offset of packed weights in the device buffer
    size_t pk_bwd_off;  // byte offset of the input-gradient (flipped) pack, FP32 only
    // paper-network stages: the fused 1x1 that follows the 3x3
    PStage ps;
    size_t w2_off, b2_off;
};

bool device_ok() {
    int dev = -1;
    return hipGetDevice(&dev) == hipSuccess && dev >= 0;
}

}  // namespace

struct nsm_ctx {
    nsm_net_desc desc;
    Dt dt;
    std::vector<StagePlan> stages;   // 3x3 stages in execution order
    size_t head_w_off;               // flat offset of the head weights ([w0] then bias)
    size_t n_params;
    // device buffer: [packed stages][flat float32 copy]
    void* dbuf = nullptr;
    size_t dbuf_bytes = 0;
    size_t flat_off = 0;             // byte offset of the float32 flat copy
    bool has_weights = false;
    bool trainable = false;          // FP32 context with backward kernels for every stage
    int variant[16] = {};            // launch variant per stage (NSM_ARCH_UNET): see conv_forward
    unsigned weights_gen = 0;        // bumped by every nsm_set_weights
    // the forward whose activations a training workspace holds (nsm_forward_train
    // or nsm_backward); any other call that may write a workspace clears it
    struct {
        const void* ws = nullptr;
        const float* feat = nullptr;
        int n = 0, h = 0, w = 0;
        unsigned gen = 0;
        bool valid = false;
    } saved;
};

extern "C" {

int nsm_abi_version(void) { return NSM_ABI_VERSION; }

const char* nsm_status_str(int s) {
    switch (s) {
        case NSM_OK: return "ok";
        case NSM_E_INVALID_ARG: return "invalid argument";
        case NSM_E_SHAPE: return "unsupported shape";
        case NSM_E_UNSUPPORTED: return "unsupported network or dtype";
        case NSM_E_WORKSPACE: return "workspace missing or too small";
        case NSM_E_NO_WEIGHTS: return "weights not set";
        case NSM_E_DEVICE: return "no HIP device or HIP runtime error";
        case NSM_E_LAUNCH: return "kernel launch failed";
        default: return "unknown status";
    }
}

// ----------------------------------------------------------------- features
nsm_status nsm_features_workspace_bytes(int n_tris, int h, int w, int sm_size, size_t* bytes) {
    if (!bytes || n_tris < 0) return NSM_E_INVALID_ARG;
    if (n_tris > kMaxTris) return NSM_E_SHAPE;
    if (h < 1 || w < 1 || h > kMaxImage || w > kMaxImage || sm_size < 1 || sm_size > kMaxImage)
        return NSM_E_SHAPE;
    *bytes = align256(raster_workspace_bytes(n_tris)) + align256((size_t)h * (size_t)w * 8) +
             linear_map_bytes(sm_size);
    return NSM_OK;
}

// od: 0 float32 features, 1 bfloat16, 2 float16, 3 FP8 E4M3 (gather()).
static nsm_status build_features(const float* tris, const float* tri_normals, int n_tris,
                                 const nsm_frame_params* fp, int h, int w, nsm_feature_set fs,
                                 const uint64_t* gbuf_in, uint64_t* gbuf_out, uint32_t* sm_out, int od,
                                 void* feat_out, uint8_t* mask_out, void* workspace, size_t ws_bytes,
                                 void* stream) {
    if (!fp || !sm_out || !feat_out || n_tris < 0) return NSM_E_INVALID_ARG;
    if (n_tris > 0 && (!tris || !tri_normals)) return NSM_E_INVALID_ARG;
    if (fs != NSM_FEAT_HARD6 && fs != NSM_FEAT_SOFT8 && fs != NSM_FEAT_PAPER4) return NSM_E_INVALID_ARG;
    size_t need = 0;
    nsm_status st = nsm_features_workspace_bytes(n_tris, h, w, fp->sm_size, &need);
    if (st != NSM_OK) return st;
    if (!workspace || ws_bytes < need) return NSM_E_WORKSPACE;
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    debug_sync_begin();
    char* ws = reinterpret_cast<char*>(workspace);
    uint64_t* gbuf_ws = reinterpret_cast<uint64_t*>(ws + align256(raster_workspace_bytes(n_tris)));
    float* lsm_ws = reinterpret_cast<float*>(ws + align256(raster_workspace_bytes(n_tris)) +
                                             align256((size_t)h * (size_t)w * 8));

    Mat4 ml, mc;
    std::memcpy(ml.m, fp->m_light, sizeof(ml.m));
    std::memcpy(mc.m, fp->m_cam, sizeof(mc.m));
    const int S = fp->sm_size;
    // light-view map and (unless the caller provides it) the camera G-buffer
    // in one setup / scan / raster sequence
    RasterPasses P{};
    P.p[0] = RasterPass{ml, S, S, 0, sm_out};
    P.npass = 1;
    const uint64_t* gb = gbuf_in;
    if (!gb) {
        uint64_t* target = gbuf_out ? gbuf_out : gbuf_ws;
        P.p[1] = RasterPass{mc, w, h, 1, target};
        P.npass = 2;
        gb = target;
    }
    if (raster(tris, n_tris, P, ws, s) != hipSuccess) return NSM_E_LAUNCH;
    GatherParams gp;
    gp.ml = ml;
    for (int k = 0; k < 3; ++k) {
        gp.L[k] = fp->light_pos[k];
        gp.E[k] = fp->cam_pos[k];
        gp.fwd[k] = fp->cam_fwd[k];
        gp.right[k] = fp->cam_right[k];
        gp.up[k] = fp->cam_up[k];
    }
    gp.r_e = fp->light_radius;
    gp.nl = fp->light_near;
    gp.fl = fp->light_far;
    gp.tanl = fp->light_tan_half_fov;
    gp.S = S;
    gp.tanx = fp->cam_tan_half_x;
    gp.tany = fp->cam_tan_half_y;
    gp.fc = fp->cam_far;
    if (gather(tris, tri_normals, n_tris, gp, gb, sm_out, lsm_ws, w, h, (int)fs, od, feat_out,
               mask_out, s) != hipSuccess)
        return NSM_E_LAUNCH;
    if (debug_sync_end(s) != hipSuccess) return NSM_E_LAUNCH;
    return NSM_OK;
}

nsm_status nsm_build_features(const float* tris, const float* tri_normals, int n_tris,
                              const nsm_frame_params* fp, int h, int w, nsm_feature_set fs,
                              const uint64_t* gbuf_in, uint64_t* gbuf_out, uint32_t* sm_out,
                              float* feat_out, uint8_t* mask_out, void* workspace, size_t ws_bytes,
                              void* stream) {
    return build_features(tris, tri_normals, n_tris, fp, h, w, fs, gbuf_in, gbuf_out, sm_out, 0, feat_out,
                          mask_out, workspace, ws_bytes, stream);
}

nsm_status nsm_build_features_stored(const float* tris, const float* tri_normals, int n_tris,
                                     const nsm_frame_params* fp, int h, int w, nsm_feature_set fs,
                                     const uint64_t* gbuf_in, uint64_t* gbuf_out, uint32_t* sm_out,
                                     nsm_dtype feat_dtype, void* feat_out, uint8_t* mask_out,
                                     void* workspace, size_t ws_bytes, void* stream) {
    if (feat_dtype != NSM_BF16 && feat_dtype != NSM_F16 && feat_dtype != NSM_F8_MFMA) return NSM_E_INVALID_ARG;
    if (fs == NSM_FEAT_PAPER4) return NSM_E_UNSUPPORTED;
    const int od = feat_dtype == NSM_BF16 ? 1 : (feat_dtype == NSM_F16 ? 2 : 3);
    return build_features(tris, tri_normals, n_tris, fp, h, w, fs, gbuf_in, gbuf_out, sm_out, od, feat_out,
                          mask_out, workspace, ws_bytes, stream);
}

// ------------------------------------------------------------------ network
nsm_status nsm_create(const nsm_net_desc* desc, nsm_dtype dtype, nsm_ctx** out) {
    if (!desc || !out) return NSM_E_INVALID_ARG;
    *out = nullptr;
    if (dtype != NSM_F32 && dtype != NSM_BF16 && dtype != NSM_F16 && dtype != NSM_F8 && dtype != NSM_F8_MFMA)
        return NSM_E_INVALID_ARG;
    const int L = desc->levels;
    if (L < 2 || L > 5 || desc->c_in < 1) return NSM_E_UNSUPPORTED;
    if (desc->arch == NSM_ARCH_UNET && L > 4) return NSM_E_UNSUPPORTED;
    if (desc->arch != NSM_ARCH_UNET && (dtype == NSM_F8 || dtype == NSM_F8_MFMA))
        return NSM_E_UNSUPPORTED;   // 8-bit forms: U-Net only
    for (int l = 0; l < L; ++l)
        if (desc->widths[l] < 1) return NSM_E_UNSUPPORTED;
    if (desc->arch != NSM_ARCH_UNET && desc->arch != NSM_ARCH_PAPER && desc->arch != NSM_ARCH_PAPER_S2D)
        return NSM_E_INVALID_ARG;
    nsm_ctx* c = new (std::nothrow) nsm_ctx();
    if (!c) return NSM_E_DEVICE;
    c->desc = *desc;
    c->dt = static_cast<Dt>(dtype);
    const int* wd = desc->widths;
    size_t off = 0;
    if (desc->arch == NSM_ARCH_PAPER || desc->arch == NSM_ARCH_PAPER_S2D) {
        // the space-to-depth form has no level-0 convolutions: its first encoder
        // stage reads the input rearranged to 2x2 blocks at level 1, and its
        // last decoder stage ends in the four-channel output conv
        const bool s2d = desc->arch == NSM_ARCH_PAPER_S2D;
        if (L != 3 && L != 5) {
            delete c;
            return NSM_E_UNSUPPORTED;
        }
        auto addp = [&](const char* name, PStage ps, int level) {
            StagePlan p{};
            p.name = name;
            p.ps = ps;
            p.level = level;
            p.w_off = off;
            off += (size_t)ps.c1 * 9 * (ps.cs + (ps.sum ? 0 : ps.cu));
            p.b_off = off;
            off += ps.c1;
            p.w2_off = off;
            off += (size_t)ps.c2 * ps.c1;
            p.b2_off = off;
            off += ps.c2;
            c->stages.push_back(p);
        };
        static const char* pe[] = {"E0", "E1", "E2", "E3"};
        static const char* pd[] = {"D0", "D1", "D2", "D3"};
        for (int l = s2d ? 1 : 0; l < L - 1; ++l) {
            const bool s2d_in = s2d && l == 1;
            addp(pe[l], PStage{l == 0 ? desc->c_in : (s2d_in ? 4 * desc->c_in : wd[l - 1]), 0, false, wd[l],
                               wd[l], l == 0 ? PMode::PoolOnly : PMode::PoolSkip, l == 0 || s2d_in, s2d_in},
                 l);
        }
        addp("B", PStage{wd[L - 2], 0, false, wd[L - 1], wd[L - 2], PMode::Store, false}, L - 1);
        for (int l = L - 2; l >= 1; --l)
            addp(pd[l], PStage{wd[l], wd[l], true, wd[l], wd[l - 1],
                               (s2d && l == 1) ? PMode::D2S : PMode::Store, false}, l);
        if (!s2d) addp("D0", PStage{0, wd[0], false, wd[0], wd[0], PMode::Head, false}, 0);
        c->head_w_off = off;
        off += s2d ? 4 * wd[0] + 4 : wd[0] + 1;
        c->n_params = off;
        size_t pk = 0;
        for (auto& p : c->stages) {
            if (!pconv_supported(p.ps)) {
                delete c;
                return NSM_E_UNSUPPORTED;
            }
            p.pk_off = pk;
            pk += align256(pconv_packed_bytes(p.ps, c->dt));
        }
        c->trainable = false;
        c->flat_off = pk;
        c->dbuf_bytes = pk + align256(c->n_params * 4);
        *out = c;
        return NSM_OK;
    }
    auto add = [&](const char* name, ConvStage st, OutMode mode, bool f32, int level) {
        StagePlan p;
        p.name = name;
        p.st = st;
        p.mode = mode;
        p.in_f32 = f32;
        p.level = level;
        p.w_off = off;
        off += (size_t)st.co * 9 * (st.cs + st.cu);
        p.b_off = off;
        off += st.co;
        p.pk_off = 0;
        c->stages.push_back(p);
    };
    static const char* enames[] = {"E0", "E1", "E2"};
    static const char* dnames[] = {"D0", "D1", "D2"};
    for (int l = 0; l < L - 1; ++l)
        add(enames[l], ConvStage{l == 0 ? desc->c_in : wd[l - 1], 0, wd[l]}, OutMode::Pool, l == 0, l);
    add("B", ConvStage{wd[L - 2], 0, wd[L - 1]}, OutMode::Store, false, L - 1);
    for (int l = L - 2; l >= 0; --l)
        add(dnames[l], ConvStage{wd[l], wd[l + 1], wd[l]}, l == 0 ? OutMode::Head : OutMode::Store,
            false, l);
    c->head_w_off = off;
    off += wd[0] + 1;
    c->n_params = off;
    size_t pk = 0;
    for (auto& p : c->stages) {
        if (!conv_supported(p.st, c->dt, p.mode, p.in_f32)) {
            delete c;
            return NSM_E_UNSUPPORTED;
        }
        p.pk_off = pk;
        pk += align256(packed_weight_bytes(p.st, c->dt));
    }
    // the FP32 context also keeps the flipped/transposed packs its input-gradient convs use
    c->trainable = c->dt == Dt::F32;
    for (auto& p : c->stages) c->trainable = c->trainable && backward_supported(p.st);
    if (c->trainable) {
        for (auto& p : c->stages) {
            p.pk_bwd_off = pk;
            pk += align256(dgrad_packed_bytes(p.st));
        }
    }
    c->flat_off = pk;
    c->dbuf_bytes = pk + align256(c->n_params * 4);
    *out = c;
    return NSM_OK;
}

nsm_status nsm_destroy(nsm_ctx* ctx) {
    if (!ctx) return NSM_E_INVALID_ARG;
    if (ctx->dbuf) (void)hipFree(ctx->dbuf);
    delete ctx;
    return NSM_OK;
}

nsm_status nsm_param_count(const nsm_ctx* ctx, size_t* n) {
    if (!ctx || !n) return NSM_E_INVALID_ARG;
    *n = ctx->n_params;
    return NSM_OK;
}

nsm_status nsm_set_weights(nsm_ctx* ctx, const float* w, size_t n, void* stream) {
    if (!ctx || !w) return NSM_E_INVALID_ARG;
    if (n != ctx->n_params) return NSM_E_INVALID_ARG;
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    debug_sync_begin();
    if (!ctx->dbuf) {
        if (hipMalloc(&ctx->dbuf, ctx->dbuf_bytes) != hipSuccess) {
            ctx->dbuf = nullptr;
            return NSM_E_DEVICE;
        }
    }
    ctx->weights_gen++;
    ctx->saved.valid = false;
    char* base = reinterpret_cast<char*>(ctx->dbuf);
    float* flat = reinterpret_cast<float*>(base + ctx->flat_off);
    if (hipMemcpyAsync(flat, w, n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return NSM_E_DEVICE;
    for (const auto& p : ctx->stages) {
        if (ctx->desc.arch != NSM_ARCH_UNET) {
            if (pconv_pack(p.ps, ctx->dt, flat + p.w_off, flat + p.w2_off, base + p.pk_off, s) != hipSuccess)
                return NSM_E_LAUNCH;
            continue;
        }
        if (pack_weights(p.st, ctx->dt, flat + p.w_off, base + p.pk_off, s) != hipSuccess)
            return NSM_E_LAUNCH;
        if (ctx->trainable &&
            pack_dgrad_weights(p.st, flat + p.w_off, base + p.pk_bwd_off, s) != hipSuccess)
            return NSM_E_LAUNCH;
    }
    if (debug_sync_end(s) != hipSuccess) return NSM_E_LAUNCH;
    ctx->has_weights = true;
    return NSM_OK;
}

}  // extern "C"

namespace {

// Activation buffers of one forward pass (n frames), in the stage dtype.
struct FwdLayout {
    size_t skip[4], pool[4], bott, dec[4], d0act, head4, total;
};

// bytes of one stored activation
size_t elem_size(Dt dt) { return dt == Dt::F32 ? 4 : ((dt == Dt::F8 || dt == Dt::F8M) ? 1 : 2); }

FwdLayout plan_forward(const nsm_ctx* c, int n, int h, int w, bool training) {
    FwdLayout L{};
    const int lv = c->desc.levels;
    const int* wd = c->desc.widths;
    const size_t es = elem_size(c->dt);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    for (int l = 0; l < lv - 1; ++l) {
        size_t hw = (size_t)(h >> l) * (w >> l);
        L.skip[l] = take((size_t)n * hw * wd[l] * es);
        L.pool[l] = take((size_t)n * (hw / 4) * wd[l] * es);
    }
    L.bott = take((size_t)n * (size_t)(h >> (lv - 1)) * (w >> (lv - 1)) * wd[lv - 1] * es);
    for (int l = 1; l <= lv - 2; ++l) L.dec[l] = take((size_t)n * (size_t)(h >> l) * (w >> l) * wd[l] * es);
    L.d0act = training ? take((size_t)n * (size_t)h * w * wd[0] * 4) : 0;
    L.total = off;
    return L;
}

// Paper network: skip[l] = x_l (l >= 1), pool[l] = avgpool(x_l), dec[l] = y_l
// (decoder output at level l >= 1, w_{l-1} channels; dec[L-1] is the bottleneck).
// Space-to-depth form: no level-0 buffers and no dec[1]; head4 holds the
// level-1 four-channel output (float32).
FwdLayout plan_forward_paper(const nsm_ctx* c, int n, int h, int w) {
    FwdLayout L{};
    const int lv = c->desc.levels;
    const int* wd = c->desc.widths;
    const size_t es = elem_size(c->dt);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    auto px = [&](int l) { return (size_t)n * (size_t)(h >> l) * (size_t)(w >> l); };
    const bool s2d = c->desc.arch == NSM_ARCH_PAPER_S2D;
    for (int l = s2d ? 1 : 0; l < lv - 1; ++l) {
        if (l >= 1) L.skip[l] = take(px(l) * wd[l] * es);
        L.pool[l] = take(px(l + 1) * wd[l] * es);
    }
    for (int l = s2d ? 2 : 1; l <= lv - 1; ++l) L.dec[l] = take(px(l) * wd[l - 1] * es);
    if (s2d) L.head4 = take(px(1) * 4 * sizeof(float));
    L.total = off;
    return L;
}

hipError_t run_forward_paper(const nsm_ctx* c, const float* feat, int n, int h, int w, float* vis,
                             float* logits, char* ws, const FwdLayout& L, hipStream_t s) {
    const char* base = reinterpret_cast<const char*>(c->dbuf);
    const float* flat = reinterpret_cast<const float*>(base + c->flat_off);
    const int lv = c->desc.levels;
    const void* prev = feat;
    for (size_t i = 0; i < c->stages.size(); ++i) {
        const StagePlan& p = c->stages[i];
        const int l = p.level;
        PConvArgs a{};
        a.wpk = base + p.pk_off;
        a.b1 = flat + p.b_off;
        a.w1pk = base + p.pk_off + pconv_w1_offset(p.ps, c->dt);
        a.b2 = flat + p.b2_off;
        a.n = n;
        a.h = h >> l;
        a.w = w >> l;
        if (p.ps.mode == PMode::PoolOnly || p.ps.mode == PMode::PoolSkip) {     // encoder
            a.in = prev;
            if (p.ps.mode == PMode::PoolSkip) a.out = ws + L.skip[l];
            a.pooled = ws + L.pool[l];
            prev = a.pooled;
        } else if (l == lv - 1) {                                              // bottleneck
            a.in = prev;
            a.out = ws + L.dec[l];
        } else if (p.ps.mode == PMode::Store) {                                // decoder, sum skip
            a.in = ws + L.skip[l];
            a.low = ws + L.dec[l + 1];
            a.out = ws + L.dec[l];
        } else if (p.ps.mode == PMode::D2S) {                                  // level 1 + output conv
            a.in = ws + L.skip[l];
            a.low = ws + L.dec[l + 1];
            a.out = ws + L.head4;
            a.head_w = flat + c->head_w_off;
            hipError_t e = pconv_forward(p.ps, c->dt, a, s);
            if (e != hipSuccess) return e;
            e = d2s_forward(reinterpret_cast<const float*>(ws + L.head4), n, h >> 1, w >> 1, vis, logits, s);
            if (e != hipSuccess) return e;
            continue;
        } else {                                                               // level 0 + output
            a.low = ws + L.dec[1];
            a.head_w = flat + c->head_w_off;
            a.vis = vis;
            a.logits = logits;
        }
        hipError_t e = pconv_forward(p.ps, c->dt, a, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

nsm_status check_net_shape(const nsm_ctx* c, int n, int h, int w) {
    if (n < 1 || n > kMaxFrames || h < 1 || w < 1 || h > kMaxImage || w > kMaxImage) return NSM_E_SHAPE;
    const int m = 1 << (c->desc.levels - 1);
    if (h % m || w % m) return NSM_E_SHAPE;
    return NSM_OK;
}

// The arguments of every stage of the forward pass; `act_out` (float32
// [n][h][w][w0]) receives the last decoder activation when non-null
// (training).
std::vector<ConvArgs> forward_args(const nsm_ctx* c, const void* feat, int n, int h, int w, float* vis,
                                   float* logits, char* ws, const FwdLayout& L, float* act_out,
                                   bool feat_stored = false) {
    const char* base = reinterpret_cast<const char*>(c->dbuf);
    const float* flat = reinterpret_cast<const float*>(base + c->flat_off);
    const int lv = c->desc.levels;
    const void* prev = feat;          // input of the next encoder stage
    std::vector<ConvArgs> out;
    for (const auto& p : c->stages) {
        ConvArgs a{};
        a.wpk = base + p.pk_off;
        a.bias = flat + p.b_off;
        a.n = n;
        a.h = h >> p.level;
        a.w = w >> p.level;
        a.in_f32 = p.in_f32 && !(feat_stored && out.empty());
        const int l = p.level;
        if (p.mode == OutMode::Pool) {
            a.in = prev;
            a.out = ws + L.skip[l];
            a.pooled = ws + L.pool[l];
            prev = a.pooled;
        } else if (p.st.cu == 0) {    // bottleneck
            a.in = prev;
            a.out = ws + L.bott;
        } else {                      // decoder: skip + upsampled lower level
            a.in = ws + L.skip[l];
            a.low = (l == lv - 2) ? (const void*)(ws + L.bott) : (const void*)(ws + L.dec[l + 1]);
            if (p.mode == OutMode::Head) {
                a.head_w = flat + c->head_w_off;
                a.vis = vis;
                a.logits = logits;
                a.act_out = act_out;
            } else {
                a.out = ws + L.dec[l];
            }
        }
        out.push_back(a);
    }
    return out;
}

// Enqueue the forward pass with the context's launch variants.
hipError_t run_forward(const nsm_ctx* c, const void* feat, int n, int h, int w, float* vis,
                       float* logits, char* ws, const FwdLayout& L, float* act_out, hipStream_t s,
                       bool feat_stored = false) {
    const std::vector<ConvArgs> args = forward_args(c, feat, n, h, w, vis, logits, ws, L, act_out, feat_stored);
    for (size_t i = 0; i < c->stages.size(); ++i) {
        const StagePlan& p = c->stages[i];
        hipError_t e = conv_forward(p.st, c->dt, p.mode, args[i], s, c->variant[i]);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// A context whose first stage can read features stored in its own dtype.
bool stored_input_ok(const nsm_ctx* c) {
    if (c->desc.arch != NSM_ARCH_UNET || (c->dt != Dt::BF16 && c->dt != Dt::F16 && c->dt != Dt::F8M) ||
        c->stages.empty())
        return false;
    const StagePlan& p = c->stages[0];
    return p.in_f32 && (p.st.cs == 6 || p.st.cs == 8) && conv_supported(p.st, c->dt, p.mode, false);
}

// Training workspace: the float32 forward activations (including the last
// decoder activation and the visibility) plus every gradient buffer.
struct TrainLayout {
    FwdLayout f;
    size_t vis, dzD[4], dxD[4], dzB, dp[4], head_part, wg_part, total;
};

TrainLayout plan_training(const nsm_ctx* c, int n, int h, int w) {
    TrainLayout T{};
    T.f = plan_forward(c, n, h, w, true);
    const int lv = c->desc.levels;
    const int* wd = c->desc.widths;
    size_t off = T.f.total;
    auto take = [&](size_t floats) {
        size_t o = off;
        off += align256(floats * 4);
        return o;
    };
    auto px = [&](int l) { return (size_t)n * (size_t)(h >> l) * (size_t)(w >> l); };
    T.vis = take(px(0));
    for (int l = 0; l < lv - 1; ++l) {
        T.dzD[l] = take(px(l) * wd[l]);
        T.dxD[l] = take(px(l) * (wd[l] + wd[l + 1]));
        T.dp[l] = take(px(l + 1) * wd[l]);
    }
    T.dzB = take(px(lv - 1) * wd[lv - 1]);
    T.head_part = take(head_partial_floats(wd[0], px(0)));
    size_t wg = 0;
    for (const auto& p : c->stages)
        wg = std::max(wg, wgrad_partial_floats(p.st, n, h >> p.level, w >> p.level));
    T.wg_part = take(wg);
    T.total = off;
    return T;
}

hipError_t run_backward(const nsm_ctx* c, const float* feat, const float* dvis, int n, int h, int w,
                        float* dw, bool acc, float* dfeat, char* ws, const TrainLayout& T, bool recompute,
                        hipStream_t s) {
    const char* base = reinterpret_cast<const char*>(c->dbuf);
    const float* flat = reinterpret_cast<const float*>(base + c->flat_off);
    const int lv = c->desc.levels;
    const int* wd = c->desc.widths;
    const FwdLayout& L = T.f;
    auto F = [&](size_t off) { return reinterpret_cast<float*>(ws + off); };
    const auto& st = c->stages;
    auto enc = [&](int l) -> const StagePlan& { return st[l]; };
    const StagePlan& bott = st[lv - 1];
    auto dec = [&](int l) -> const StagePlan& { return st[2 * lv - 2 - l]; };
    float* part = F(T.wg_part);
    hipError_t e;
#define NSM_TRY(x) \
    if ((e = (x)) != hipSuccess) return e
    // recompute the forward, keeping every activation (float32), unless the
    // workspace already holds them
    if (recompute) NSM_TRY(run_forward(c, feat, n, h, w, F(T.vis), nullptr, ws, L, F(L.d0act), s));
    // sigmoid + 1x1 head
    const size_t npix = (size_t)n * h * w;
    NSM_TRY(head_backward(wd[0], F(T.vis), dvis, F(L.d0act), flat + c->head_w_off, npix, F(T.dzD[0]),
                          F(T.head_part), s));
    NSM_TRY(head_reduce(wd[0], F(T.head_part), npix, dw + c->head_w_off, acc, s));
    // decoder stages, top level first
    for (int l = 0; l < lv - 1; ++l) {
        const StagePlan& p = dec(l);
        const int hl = h >> l, wl = w >> l;
        const float* lower = (l == lv - 2) ? F(L.bott) : F(L.dec[l + 1]);
        NSM_TRY(conv_dgrad(p.st, base + p.pk_bwd_off, F(T.dzD[l]), n, hl, wl, F(T.dxD[l]), s));
        NSM_TRY(conv_wgrad(p.st, F(L.skip[l]), lower, F(T.dzD[l]), n, hl, wl, part, dw + p.w_off,
                           dw + p.b_off, acc, s));
        float* target = (l == lv - 2) ? F(T.dzB) : F(T.dzD[l + 1]);
        NSM_TRY(up_transpose_mask(wd[l + 1], wd[l] + wd[l + 1], wd[l], F(T.dxD[l]), lower, n, hl >> 1,
                                  wl >> 1, target, s));
    }
    // bottleneck
    {
        const int hb = h >> (lv - 1), wb = w >> (lv - 1);
        NSM_TRY(conv_dgrad(bott.st, base + bott.pk_bwd_off, F(T.dzB), n, hb, wb, F(T.dp[lv - 2]), s));
        NSM_TRY(conv_wgrad(bott.st, F(L.pool[lv - 2]), nullptr, F(T.dzB), n, hb, wb, part,
                           dw + bott.w_off, dw + bott.b_off, acc, s));
    }
    // encoder stages, bottom level first
    for (int l = lv - 2; l >= 0; --l) {
        const StagePlan& p = enc(l);
        const int hl = h >> l, wl = w >> l;
        float* dz = F(T.dzD[l]);     // the decoder gradient at this level is no longer needed
        NSM_TRY(pool_transpose_mask(wd[l], wd[l] + wd[l + 1], F(T.dxD[l]), F(T.dp[l]), F(L.skip[l]), n,
                                    hl, wl, dz, s));
        const float* in = (l == 0) ? feat : F(L.pool[l - 1]);
        NSM_TRY(conv_wgrad(p.st, in, nullptr, dz, n, hl, wl, part, dw + p.w_off, dw + p.b_off, acc, s));
        if (l > 0) {
            NSM_TRY(conv_dgrad(p.st, base + p.pk_bwd_off, dz, n, hl, wl, F(T.dp[l - 1]), s));
        } else if (dfeat) {
            NSM_TRY(conv_dgrad(p.st, base + p.pk_bwd_off, dz, n, hl, wl, dfeat, s));
        }
    }
#undef NSM_TRY
    return hipSuccess;
}

}  // namespace

extern "C" {

nsm_status nsm_workspace_bytes(const nsm_ctx* ctx, int n, int h, int w, int training, size_t* bytes) {
    if (!ctx || !bytes) return NSM_E_INVALID_ARG;
    nsm_status st = check_net_shape(ctx, n, h, w);
    if (st != NSM_OK) return st;
    if (training) {
        if (!ctx->trainable) return NSM_E_UNSUPPORTED;
        *bytes = plan_training(ctx, n, h, w).total;
        return NSM_OK;
    }
    *bytes = ctx->desc.arch != NSM_ARCH_UNET ? plan_forward_paper(ctx, n, h, w).total
                                             : plan_forward(ctx, n, h, w, false).total;
    return NSM_OK;
}

nsm_status nsm_forward(nsm_ctx* ctx, const float* feat, int n, int h, int w, float* vis_out,
                       float* logits_out, void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx || !feat || !vis_out) return NSM_E_INVALID_ARG;
    nsm_status st = check_net_shape(ctx, n, h, w);
    if (st != NSM_OK) return st;
    if (!ctx->has_weights) return NSM_E_NO_WEIGHTS;
    const bool paper = ctx->desc.arch != NSM_ARCH_UNET;
    FwdLayout L = paper ? plan_forward_paper(ctx, n, h, w) : plan_forward(ctx, n, h, w, false);
    if (!workspace || ws_bytes < L.total) return NSM_E_WORKSPACE;
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ctx->saved.valid = false;
    debug_sync_begin();
    char* ws = reinterpret_cast<char*>(workspace);
    const hipError_t e = paper ? run_forward_paper(ctx, feat, n, h, w, vis_out, logits_out, ws, L, s)
                               : run_forward(ctx, feat, n, h, w, vis_out, logits_out, ws, L, nullptr, s);
    if (e != hipSuccess) return NSM_E_LAUNCH;
    if (debug_sync_end(s) != hipSuccess) return NSM_E_LAUNCH;
    return NSM_OK;
}

nsm_status nsm_forward_stored(nsm_ctx* ctx, const void* feat, int n, int h, int w, float* vis_out,
                              float* logits_out, void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx || !feat || !vis_out) return NSM_E_INVALID_ARG;
    if (!stored_input_ok(ctx)) return NSM_E_UNSUPPORTED;
    nsm_status st = check_net_shape(ctx, n, h, w);
    if (st != NSM_OK) return st;
    if (!ctx->has_weights) return NSM_E_NO_WEIGHTS;
    const FwdLayout L = plan_forward(ctx, n, h, w, false);
    if (!workspace || ws_bytes < L.total) return NSM_E_WORKSPACE;
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ctx->saved.valid = false;
    debug_sync_begin();
    if (run_forward(ctx, feat, n, h, w, vis_out, logits_out, reinterpret_cast<char*>(workspace), L, nullptr, s,
                    true) != hipSuccess)
        return NSM_E_LAUNCH;
    if (debug_sync_end(s) != hipSuccess) return NSM_E_LAUNCH;
    return NSM_OK;
}

static nsm_status autotune(nsm_ctx* ctx, const void* feat, bool feat_stored, int n, int h, int w, float* vis_out,
                           void* workspace, size_t ws_bytes, int reps, int* variants_out, void* stream) {
    if (!ctx || !feat || !vis_out || reps < 1 || reps > 1000) return NSM_E_INVALID_ARG;
    if (ctx->desc.arch != NSM_ARCH_UNET) return NSM_E_UNSUPPORTED;
    if (feat_stored && !stored_input_ok(ctx)) return NSM_E_UNSUPPORTED;
    nsm_status st = check_net_shape(ctx, n, h, w);
    if (st != NSM_OK) return st;
    if (!ctx->has_weights) return NSM_E_NO_WEIGHTS;
    const FwdLayout L = plan_forward(ctx, n, h, w, false);
    if (!workspace || ws_bytes < L.total) return NSM_E_WORKSPACE;
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ctx->saved.valid = false;
    char* ws = reinterpret_cast<char*>(workspace);
    // one forward with the current variants leaves every stage's input in the workspace
    if (run_forward(ctx, feat, n, h, w, vis_out, nullptr, ws, L, nullptr, s, feat_stored) != hipSuccess)
        return NSM_E_LAUNCH;
    const std::vector<ConvArgs> args = forward_args(ctx, feat, n, h, w, vis_out, nullptr, ws, L, nullptr, feat_stored);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return NSM_E_DEVICE;
    }
    nsm_status res = NSM_OK;
    for (size_t i = 0; i < ctx->stages.size() && res == NSM_OK; ++i) {
        const StagePlan& p = ctx->stages[i];
        float best = 0.0f;
        int pick = ctx->variant[i];
        for (int v = 0; v < kConvVariants && res == NSM_OK; ++v) {
            // one untimed launch (first-use set-up of the variant), then `reps` timed ones
            if (conv_forward(p.st, ctx->dt, p.mode, args[i], s, v) != hipSuccess ||
                hipEventRecord(e0, s) != hipSuccess) {
                res = NSM_E_LAUNCH;
                break;
            }
            for (int r = 0; r < reps; ++r)
                if (conv_forward(p.st, ctx->dt, p.mode, args[i], s, v) != hipSuccess) res = NSM_E_LAUNCH;
            float ms = 0.0f;
            if (res != NSM_OK || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                res = res == NSM_OK ? NSM_E_DEVICE : res;
                break;
            }
            if (v == 0 || ms < best) {
                best = ms;
                pick = v;
            }
        }
        ctx->variant[i] = pick;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (res != NSM_OK) return res;
    if (variants_out)
        for (size_t i = 0; i < ctx->stages.size(); ++i) variants_out[i] = ctx->variant[i];
    return NSM_OK;
}

nsm_status nsm_autotune(nsm_ctx* ctx, const float* feat, int n, int h, int w, float* vis_out, void* workspace,
                        size_t ws_bytes, int reps, int* variants_out, void* stream) {
    return autotune(ctx, feat, false, n, h, w, vis_out, workspace, ws_bytes, reps, variants_out, stream);
}

nsm_status nsm_autotune_stored(nsm_ctx* ctx, const void* feat, int n, int h, int w, float* vis_out,
                               void* workspace, size_t ws_bytes, int reps, int* variants_out, void* stream) {
    return autotune(ctx, feat, true, n, h, w, vis_out, workspace, ws_bytes, reps, variants_out, stream);
}

nsm_status nsm_set_stage_variant(nsm_ctx* ctx, int stage, int variant) {
    if (!ctx || variant < 0 || variant >= kConvVariants) return NSM_E_INVALID_ARG;
    if (ctx->desc.arch != NSM_ARCH_UNET) return NSM_E_UNSUPPORTED;
    if (stage < 0 || stage >= (int)ctx->stages.size()) return NSM_E_INVALID_ARG;
    ctx->variant[stage] = variant;
    return NSM_OK;
}

nsm_status nsm_get_stage_variants(const nsm_ctx* ctx, int* variants, int max, int* n_stages) {
    if (!ctx || !n_stages || max < 0 || (max > 0 && !variants)) return NSM_E_INVALID_ARG;
    const int ns = (int)ctx->stages.size();
    *n_stages = ns;
    for (int i = 0; i < ns && i < max; ++i) variants[i] = ctx->variant[i];
    return NSM_OK;
}

static nsm_status backward_common(nsm_ctx* ctx, const float* feat, const float* dvis, int n, int h, int w,
                                  float* dw_out, int accumulate, float* dfeat_out, void* workspace, size_t ws_bytes,
                                  void* stream, bool saved) {
    if (!ctx || !feat || !dvis || !dw_out) return NSM_E_INVALID_ARG;
    nsm_status st = check_net_shape(ctx, n, h, w);
    if (st != NSM_OK) return st;
    if (!ctx->trainable) return NSM_E_UNSUPPORTED;
    if (!ctx->has_weights) return NSM_E_NO_WEIGHTS;
    TrainLayout T = plan_training(ctx, n, h, w);
    if (!workspace || ws_bytes < T.total) return NSM_E_WORKSPACE;
    if (saved) {
        const auto& sv = ctx->saved;
        if (!sv.valid || sv.ws != workspace || sv.feat != feat || sv.n != n || sv.h != h || sv.w != w ||
            sv.gen != ctx->weights_gen)
            return NSM_E_INVALID_ARG;
    }
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ctx->saved.valid = false;
    debug_sync_begin();
    if (run_backward(ctx, feat, dvis, n, h, w, dw_out, accumulate != 0, dfeat_out,
                     reinterpret_cast<char*>(workspace), T, !saved, s) != hipSuccess)
        return NSM_E_LAUNCH;
    if (debug_sync_end(s) != hipSuccess) return NSM_E_LAUNCH;
    // the workspace holds this forward's activations (the adjoint only reads them)
    ctx->saved = {workspace, feat, n, h, w, ctx->weights_gen, true};
    return NSM_OK;
}

nsm_status nsm_backward(nsm_ctx* ctx, const float* feat, const float* dvis, int n, int h, int w,
                        float* dw_out, int accumulate, float* dfeat_out, void* workspace,
                        size_t ws_bytes, void* stream) {
    return backward_common(ctx, feat, dvis, n, h, w, dw_out, accumulate, dfeat_out, workspace, ws_bytes, stream,
                           false);
}

nsm_status nsm_backward_saved(nsm_ctx* ctx, const float* feat, const float* dvis, int n, int h, int w,
                              float* dw_out, int accumulate, float* dfeat_out, void* workspace,
                              size_t ws_bytes, void* stream) {
    return backward_common(ctx, feat, dvis, n, h, w, dw_out, accumulate, dfeat_out, workspace, ws_bytes, stream,
                           true);
}

nsm_status nsm_forward_train(nsm_ctx* ctx, const float* feat, int n, int h, int w, float* vis_out,
                             void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx || !feat) return NSM_E_INVALID_ARG;
    nsm_status st = check_net_shape(ctx, n, h, w);
    if (st != NSM_OK) return st;
    if (!ctx->trainable) return NSM_E_UNSUPPORTED;
    if (!ctx->has_weights) return NSM_E_NO_WEIGHTS;
    TrainLayout T = plan_training(ctx, n, h, w);
    if (!workspace || ws_bytes < T.total) return NSM_E_WORKSPACE;
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    ctx->saved.valid = false;
    debug_sync_begin();
    char* ws = reinterpret_cast<char*>(workspace);
    float* vis = reinterpret_cast<float*>(ws + T.vis);
    if (run_forward(ctx, feat, n, h, w, vis, nullptr, ws, T.f, reinterpret_cast<float*>(ws + T.f.d0act), s) !=
        hipSuccess)
        return NSM_E_LAUNCH;
    if (vis_out && hipMemcpyAsync(vis_out, vis, (size_t)n * h * w * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return NSM_E_LAUNCH;
    if (debug_sync_end(s) != hipSuccess) return NSM_E_LAUNCH;
    ctx->saved = {workspace, feat, n, h, w, ctx->weights_gen, true};
    return NSM_OK;
}


// ------------------------------------------------------ temporal stability
constexpr int kMaxPerturb = 16;

nsm_status nsm_perturbation_loss_workspace_bytes(int n, int p, int h, int w, size_t* bytes) {
    if (!bytes) return NSM_E_INVALID_ARG;
    if (n < 1 || n > kMaxFrames || p < 0 || p > kMaxPerturb || h < 1 || w < 1 || h > kMaxImage ||
        w > kMaxImage)
        return NSM_E_SHAPE;
    *bytes = perturb_loss_workspace_bytes((long long)n * h * w);
    return NSM_OK;
}

nsm_status nsm_perturbation_loss(const float* vis, const float* target, int n, int p, int h, int w,
                                 float alpha, double* loss_out, float* dvis0_out, void* workspace,
                                 size_t ws_bytes, void* stream) {
    if (!vis || !target || !loss_out || !dvis0_out) return NSM_E_INVALID_ARG;
    if (n < 1 || n > kMaxFrames || p < 0 || p > kMaxPerturb || h < 1 || w < 1 || h > kMaxImage ||
        w > kMaxImage)
        return NSM_E_SHAPE;
    if (!workspace || ws_bytes < perturb_loss_workspace_bytes((long long)n * h * w)) return NSM_E_WORKSPACE;
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    debug_sync_begin();
    if (perturb_loss(vis, target, n, p, h, w, alpha, loss_out, dvis0_out, workspace, s) != hipSuccess)
        return NSM_E_LAUNCH;
    if (debug_sync_end(s) != hipSuccess) return NSM_E_LAUNCH;
    return NSM_OK;
}

nsm_status nsm_perturbation_loss_noalloc(const float* vis, const float* target, int n, int p, int h, int w,
                                         float alpha, double* loss_out, float* dvis0_out, void* stream) {
    if (!vis || !target || !loss_out || !dvis0_out) return NSM_E_INVALID_ARG;
    if (n < 1 || n > kMaxFrames || p < 0 || p > kMaxPerturb || h < 1 || w < 1 || h > kMaxImage ||
        w > kMaxImage)
        return NSM_E_SHAPE;
    if ((long long)n * h * w > kStaticLossMaxPixels) return NSM_E_SHAPE;
    if (!device_ok()) return NSM_E_DEVICE;
    double* partials = nullptr;
    if (static_loss_partials(&partials) != hipSuccess) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    debug_sync_begin();
    if (perturb_loss(vis, target, n, p, h, w, alpha, loss_out, dvis0_out, partials, s) != hipSuccess)
        return NSM_E_LAUNCH;
    if (debug_sync_end(s) != hipSuccess) return NSM_E_LAUNCH;
    return NSM_OK;
}

nsm_status nsm_temporal_workspace_bytes(int h, int w, size_t* bytes) {
    if (!bytes) return NSM_E_INVALID_ARG;
    if (h < 1 || w < 1 || h > kMaxImage || w > kMaxImage) return NSM_E_SHAPE;
    *bytes = temporal_workspace_bytes(h, w);
    return NSM_OK;
}

static CamParams cam_params(const nsm_frame_params* fp) {
    CamParams c;
    for (int k = 0; k < 16; ++k) c.m[k] = fp->m_cam[k];
    for (int k = 0; k < 3; ++k) {
        c.E[k] = fp->cam_pos[k];
        c.fwd[k] = fp->cam_fwd[k];
        c.right[k] = fp->cam_right[k];
        c.up[k] = fp->cam_up[k];
    }
    c.tanx = fp->cam_tan_half_x;
    c.tany = fp->cam_tan_half_y;
    return c;
}

nsm_status nsm_temporal_instability(const float* tris, const float* tri_normals, int n_tris,
                                    const nsm_frame_params* prev, const nsm_frame_params* cur,
                                    const uint64_t* gbuf_prev, const uint64_t* gbuf_cur,
                                    const float* vis_prev, const float* vis_cur, int h, int w, float alpha,
                                    float depth_tol, float cos_tol, int accumulate, double* acc_out,
                                    float* d_out, void* workspace, size_t ws_bytes, void* stream) {
    if (!prev || !cur || !gbuf_prev || !gbuf_cur || !vis_prev || !vis_cur || !acc_out || n_tris < 0)
        return NSM_E_INVALID_ARG;
    if (n_tris > 0 && (!tris || !tri_normals)) return NSM_E_INVALID_ARG;
    if (n_tris > kMaxTris) return NSM_E_SHAPE;
    if (h < 1 || w < 1 || h > kMaxImage || w > kMaxImage) return NSM_E_SHAPE;
    if (!workspace || ws_bytes < temporal_workspace_bytes(h, w)) return NSM_E_WORKSPACE;
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    debug_sync_begin();
    if (temporal_pair(tris, tri_normals, n_tris, cam_params(prev), cam_params(cur), gbuf_prev, gbuf_cur,
                      vis_prev, vis_cur, h, w, alpha, depth_tol, cos_tol, accumulate, acc_out, d_out,
                      workspace, s) != hipSuccess)
        return NSM_E_LAUNCH;
    if (debug_sync_end(s) != hipSuccess) return NSM_E_LAUNCH;
    return NSM_OK;
}

}  // extern "C"
