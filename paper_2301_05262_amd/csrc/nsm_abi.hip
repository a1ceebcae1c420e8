// C-ABI entry points: argument validation, context and workspace planning,
// and the order of kernel launches for each call.  All validation happens
// before the first HIP call so that a non-OK status never leaves work on the
// stream.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using namespace nsm;

namespace {

constexpr int kMaxImage = 16384;
constexpr int kMaxFrames = 4096;

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
    if (h < 1 || w < 1 || h > kMaxImage || w > kMaxImage || sm_size < 1 || sm_size > kMaxImage)
        return NSM_E_SHAPE;
    *bytes = align256(raster_workspace_bytes(n_tris)) + align256((size_t)h * (size_t)w * 8);
    return NSM_OK;
}

nsm_status nsm_build_features(const float* tris, const float* tri_normals, int n_tris,
                              const nsm_frame_params* fp, int h, int w, nsm_feature_set fs,
                              const uint64_t* gbuf_in, uint64_t* gbuf_out, uint32_t* sm_out,
                              float* feat_out, uint8_t* mask_out, void* workspace, size_t ws_bytes,
                              void* stream) {
    if (!fp || !sm_out || !feat_out || n_tris < 0) return NSM_E_INVALID_ARG;
    if (n_tris > 0 && (!tris || !tri_normals)) return NSM_E_INVALID_ARG;
    if (fs != NSM_FEAT_HARD6 && fs != NSM_FEAT_SOFT8) return NSM_E_INVALID_ARG;
    size_t need = 0;
    nsm_status st = nsm_features_workspace_bytes(n_tris, h, w, fp->sm_size, &need);
    if (st != NSM_OK) return st;
    if (!workspace || ws_bytes < need) return NSM_E_WORKSPACE;
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* ws = reinterpret_cast<char*>(workspace);
    uint64_t* gbuf_ws = reinterpret_cast<uint64_t*>(ws + align256(raster_workspace_bytes(n_tris)));

    Mat4 ml, mc;
    std::memcpy(ml.m, fp->m_light, sizeof(ml.m));
    std::memcpy(mc.m, fp->m_cam, sizeof(mc.m));
    const int S = fp->sm_size;
    if (raster(tris, n_tris, ml, S, S, false, sm_out, ws, s) != hipSuccess) return NSM_E_LAUNCH;
    const uint64_t* gb = gbuf_in;
    if (!gb) {
        uint64_t* target = gbuf_out ? gbuf_out : gbuf_ws;
        if (raster(tris, n_tris, mc, w, h, true, target, ws, s) != hipSuccess) return NSM_E_LAUNCH;
        gb = target;
    }
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
    if (gather(tris, tri_normals, n_tris, gp, gb, sm_out, w, h, fs == NSM_FEAT_SOFT8, feat_out,
               mask_out, s) != hipSuccess)
        return NSM_E_LAUNCH;
    return NSM_OK;
}

// ------------------------------------------------------------------ network
nsm_status nsm_create(const nsm_net_desc* desc, nsm_dtype dtype, nsm_ctx** out) {
    if (!desc || !out) return NSM_E_INVALID_ARG;
    *out = nullptr;
    if (dtype != NSM_F32 && dtype != NSM_BF16 && dtype != NSM_F16) return NSM_E_INVALID_ARG;
    const int L = desc->levels;
    if (L < 2 || L > 4 || desc->c_in < 1) return NSM_E_UNSUPPORTED;
    for (int l = 0; l < L; ++l)
        if (desc->widths[l] < 1) return NSM_E_UNSUPPORTED;
    nsm_ctx* c = new (std::nothrow) nsm_ctx();
    if (!c) return NSM_E_DEVICE;
    c->desc = *desc;
    c->dt = static_cast<Dt>(dtype);
    const int* wd = desc->widths;
    size_t off = 0;
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
    if (!ctx->dbuf) {
        if (hipMalloc(&ctx->dbuf, ctx->dbuf_bytes) != hipSuccess) {
            ctx->dbuf = nullptr;
            return NSM_E_DEVICE;
        }
    }
    char* base = reinterpret_cast<char*>(ctx->dbuf);
    float* flat = reinterpret_cast<float*>(base + ctx->flat_off);
    if (hipMemcpyAsync(flat, w, n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return NSM_E_DEVICE;
    for (const auto& p : ctx->stages)
        if (pack_weights(p.st, ctx->dt, flat + p.w_off, base + p.pk_off, s) != hipSuccess)
            return NSM_E_LAUNCH;
    ctx->has_weights = true;
    return NSM_OK;
}

}  // extern "C"

namespace {

// Activation buffers of one forward pass (n frames), in the stage dtype.
struct FwdLayout {
    size_t skip[4], pool[4], bott, dec[4], d0act, total;
};

size_t elem_size(Dt dt) { return dt == Dt::F32 ? 4 : 2; }

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

nsm_status check_net_shape(const nsm_ctx* c, int n, int h, int w) {
    if (n < 1 || n > kMaxFrames || h < 1 || w < 1 || h > kMaxImage || w > kMaxImage) return NSM_E_SHAPE;
    const int m = 1 << (c->desc.levels - 1);
    if (h % m || w % m) return NSM_E_SHAPE;
    return NSM_OK;
}

// Enqueue the forward pass; `act_out` (float32 [n][h][w][w0]) receives the
// last decoder activation when non-null (training).
hipError_t run_forward(const nsm_ctx* c, const float* feat, int n, int h, int w, float* vis,
                       float* logits, char* ws, const FwdLayout& L, float* act_out, hipStream_t s) {
    const char* base = reinterpret_cast<const char*>(c->dbuf);
    const float* flat = reinterpret_cast<const float*>(base + c->flat_off);
    const int lv = c->desc.levels;
    const void* prev = feat;          // input of the next encoder stage
    for (const auto& p : c->stages) {
        ConvArgs a{};
        a.wpk = base + p.pk_off;
        a.bias = flat + p.b_off;
        a.n = n;
        a.h = h >> p.level;
        a.w = w >> p.level;
        a.in_f32 = p.in_f32;
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
        hipError_t e = conv_forward(p.st, c->dt, p.mode, a, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

nsm_status nsm_workspace_bytes(const nsm_ctx* ctx, int n, int h, int w, int training, size_t* bytes) {
    if (!ctx || !bytes) return NSM_E_INVALID_ARG;
    nsm_status st = check_net_shape(ctx, n, h, w);
    if (st != NSM_OK) return st;
    if (training) return NSM_E_UNSUPPORTED;
    *bytes = plan_forward(ctx, n, h, w, false).total;
    return NSM_OK;
}

nsm_status nsm_forward(nsm_ctx* ctx, const float* feat, int n, int h, int w, float* vis_out,
                       float* logits_out, void* workspace, size_t ws_bytes, void* stream) {
    if (!ctx || !feat || !vis_out) return NSM_E_INVALID_ARG;
    nsm_status st = check_net_shape(ctx, n, h, w);
    if (st != NSM_OK) return st;
    if (!ctx->has_weights) return NSM_E_NO_WEIGHTS;
    FwdLayout L = plan_forward(ctx, n, h, w, false);
    if (!workspace || ws_bytes < L.total) return NSM_E_WORKSPACE;
    if (!device_ok()) return NSM_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (run_forward(ctx, feat, n, h, w, vis_out, logits_out, reinterpret_cast<char*>(workspace), L,
                    nullptr, s) != hipSuccess)
        return NSM_E_LAUNCH;
    return NSM_OK;
}

nsm_status nsm_backward(nsm_ctx* ctx, const float* feat, const float* dvis, int n, int h, int w,
                        float* dw_out, int accumulate, float* dfeat_out, void* workspace,
                        size_t ws_bytes, void* stream) {
    (void)feat; (void)dvis; (void)n; (void)h; (void)w; (void)dw_out; (void)accumulate;
    (void)dfeat_out; (void)workspace; (void)ws_bytes; (void)stream;
    if (!ctx) return NSM_E_INVALID_ARG;
    return NSM_E_UNSUPPORTED;
}

}  // extern "C"
