// Internal launch interface between the C-ABI layer and the kernel files.
// Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/nsm.h"

namespace nsm {

// ------------------------------------------------------------- tracing
// Per-kernel timing hooks (no-ops unless nsm_trace_enable(1) was called).
bool trace_on();
void trace_begin(const char* name, const char* suffix, hipStream_t s);
void trace_end(hipStream_t s);

// Debug mode (environment NSM_DEBUG_SYNC=1, read at every entry point):
// debug_sync_begin() arms it for the calling thread's current entry point;
// debug_check(s) then synchronises `s` after each launch and keeps the first
// runtime error; debug_sync_end(s) synchronises once more and returns that
// error (hipSuccess when the mode is off).
bool debug_sync_begin();
void debug_check(hipStream_t s);
hipError_t debug_sync_end(hipStream_t s);

// Every kernel launch of the library sits inside one of these scopes: it
// brackets the launch with trace events when tracing is on and, in debug
// mode, synchronises after it.
struct TraceScope {
    hipStream_t s;
    bool on;
    TraceScope(const char* name, const char* suffix, hipStream_t st) : s(st), on(trace_on()) {
        if (on) trace_begin(name, suffix, s);
    }
    ~TraceScope() {
        if (on) trace_end(s);
        debug_check(s);
    }
};

// ------------------------------------------------------------ rasteriser
// 64-byte per-triangle record written by the setup kernel.
struct alignas(16) TriSetup {
    int32_t x[3], y[3];   // 24.8 fixed-point screen coordinates, CCW order
    float z[3];           // ndc depth per vertex
    int32_t tx0, ty0;     // first raster tile of the texel bounding box
    int32_t ntx;          // tiles per bounding-box row (count = ntx * nty)
    int64_t area;         // doubled signed area (> 0 after reordering)
    int32_t pad;
};
static_assert(sizeof(TriSetup) == 64, "TriSetup must stay 64 bytes");

struct Mat4 { float m[16]; };

// One rasterisation target: clear `out` (w*h texels of 4 or 8 bytes) and
// keep the nearest fragment; key64 selects the camera key
// (depth bits << 32 | id) instead of plain depth bits.
struct RasterPass {
    Mat4 m;
    int w, h;
    int key64;
    void* out;
};
struct RasterPasses {
    RasterPass p[2];
    int npass;          // 1 or 2; both passes share one setup / scan / raster launch
};
// Workspace for up to two passes over n_tris triangles.
size_t raster_workspace_bytes(int n_tris);
hipError_t raster(const float* tris, int n_tris, const RasterPasses& P, void* ws, hipStream_t s);

struct GatherParams {
    Mat4 ml;
    float L[3], r_e, nl, fl, tanl;
    int S;
    float E[3], fwd[3], right[3], up[3];
    float tanx, tany, fc;
    // filled by gather(): per-launch constants of the per-pixel arithmetic
    float tau;                // (2 tanl) / S, float32
    double rw, rh;            // 1 / w and 1 / h, float64, rounded to nearest
    // the camera's float32 values widened to float64 (exact), once per launch
    double E_d[3], fwd_d[3], right_d[3], up_d[3], tanx_d, tany_d;
};
// Bytes of the linear-depth copy of an S x S shadow map (SOFT8's blocker search).
size_t linear_map_bytes(int sm_size);
// `lsm` (linear_map_bytes) receives the linear-depth copy of the map first
// when fs is SOFT8; unused otherwise.  od: 0 writes float32 [h][w][C]; 1
// (bfloat16) and 2 (float16) write [h][w][8] in that type, each channel
// rounded to nearest even, channels past C zero; 3 writes FP8 E4M3 bytes
// [h][w][16] (saturated to +-448, nearest even), bytes past C zero.  od > 0
// takes HARD6 or SOFT8.
hipError_t gather(const float* tris, const float* normals, int n_tris, const GatherParams& p,
                  const uint64_t* gbuf, const uint32_t* sm, float* lsm, int w, int h, int fs, int od, void* feat,
                  uint8_t* mask, hipStream_t s);

// ------------------------------------------------------ temporal stability
// One camera as the receiver reconstruction and the reprojection see it.
struct CamParams {
    float m[16];                 // world -> clip, row-major
    float E[3], fwd[3], right[3], up[3];
    float tanx, tany;
};
size_t perturb_loss_workspace_bytes(long long npx);
// Partials of the allocation-free entry point: one float64 per 256 pixels,
// so at most kStaticLossPartials * 256 pixels per call (2 MiB of scratch).
constexpr long long kStaticLossPartials = 1 << 18;
constexpr long long kStaticLossMaxPixels = kStaticLossPartials * 256;
// This device's address of the library-held partials array (looked up once
// per device, with that device current).
hipError_t static_loss_partials(double** out);
hipError_t perturb_loss(const float* vis, const float* target, int n, int p, int h, int w, float alpha,
                        double* loss, float* dvis0, void* ws, hipStream_t s);
size_t temporal_workspace_bytes(int h, int w);
hipError_t temporal_pair(const float* tris, const float* normals, int n_tris, const CamParams& prev,
                         const CamParams& cur, const uint64_t* gprev, const uint64_t* gcur, const float* vprev,
                         const float* vcur, int h, int w, float alpha, float depth_tol, float cos_tol,
                         int accumulate, double* acc_out, float* d_out, void* ws, hipStream_t s);

// --------------------------------------------------------------- network
// F8: 8-bit temporary storage -- activations stored in global memory as FP8
// E4M3 (OCP), weights and compute in bfloat16.  F8M: FP8 E4M3 throughout --
// stored activations, LDS tiles and weights -- on the FP8 MFMA.
enum class Dt { F32 = 0, BF16 = 1, F16 = 2, F8 = 3, F8M = 4 };

// One 3x3 conv stage as the kernels see it.
struct ConvStage {
    int cs;      // channels read from the same-resolution input (skip / plain input)
    int cu;      // channels produced by bilinear x2 upsampling of the lower level (0 if none)
    int co;      // output channels
};

// Packed-weight bytes of one stage for a dtype (layout private to conv.hip).
size_t packed_weight_bytes(const ConvStage& st, Dt dt);
// Repack OHWI float32 weights of one stage into the kernel layout.
hipError_t pack_weights(const ConvStage& st, Dt dt, const float* w_ohwi, void* packed,
                        hipStream_t s);

enum class OutMode { Store = 0, Pool = 1, Head = 2, Linear = 3 };  // Linear: no bias, no ReLU

struct ConvArgs {
    const void* in;      // plain input [n][h][w][cs] (float32 when in_f32, else the stage dtype)
    const void* low;     // lower level [n][h/2][w/2][cu] for upsampling (stage dtype)
    const void* wpk;     // packed weights
    const float* bias;   // [co]
    void* out;           // [n][h][w][co] stage dtype (Store/Pool), or NULL for Head
    void* pooled;        // [n][h/2][w/2][co] (Pool)
    const float* head_w; // [co] + bias at head_w[co] (Head)
    float* vis;          // [n][h][w] (Head)
    float* logits;       // [n][h][w] or NULL (Head)
    float* act_out;      // [n][h][w][co] float32 post-ReLU copy or NULL (Head, training)
    int n, h, w;
    bool in_f32;
};
// variant 0..3: bit 0 the persistent grid, bit 1 the stage's alternative tile
// rows; all variants give the same bits.
constexpr int kConvVariants = 4;
hipError_t conv_forward(const ConvStage& st, Dt dt, OutMode mode, const ConvArgs& a, hipStream_t s,
                        int variant = 0);
bool conv_supported(const ConvStage& st, Dt dt, OutMode mode, bool in_f32);

// ---------------------------------------------- the paper's network (P-net)
// D2S: the stage ends in the output 1x1 conv to four channels, stored as
// float32 [n][h][w][4] for the depth-to-space head (d2s_forward).
enum class PMode { Store = 0, PoolOnly = 1, PoolSkip = 2, Head = 3, D2S = 4 };

// One P-net stage: 3x3 conv (cs [+ cu] -> c1) + ReLU, 1x1 (c1 -> c2) + ReLU.
// Input: `in` ([.., cs]) and/or up(low) ([.., cu] at half resolution), summed
// when `sum` (cs == cu), concatenated otherwise (cs = 0: upsampled input only).
// s2d: `in` is the float32 full-resolution input read through space-to-depth.
struct PStage {
    int cs, cu;
    bool sum;
    int c1, c2;
    PMode mode;
    bool in_f32;
    bool s2d = false;
};

struct PConvArgs {
    const void* in;
    const void* low;
    const void* wpk;      // packed 3x3 weights
    const float* b1;      // [c1]
    const void* w1pk;     // packed 1x1 weights
    const float* b2;      // [c2]
    void* out;            // [n][h][w][c2] (Store, PoolSkip)
    void* pooled;         // [n][h/2][w/2][c2] average-pooled (PoolOnly, PoolSkip)
    const float* head_w;  // [c2] + bias (Head); [4][c2] + 4 biases (D2S)
    float* vis;
    float* logits;
    int n, h, w;
};

bool pconv_supported(const PStage& st);
size_t pconv_packed_bytes(const PStage& st, Dt dt);
size_t pconv_w1_offset(const PStage& st, Dt dt);
hipError_t pconv_pack(const PStage& st, Dt dt, const float* w3, const float* w1, void* packed,
                      hipStream_t s);
hipError_t pconv_forward(const PStage& st, Dt dt, const PConvArgs& a, hipStream_t s);
// Depth-to-space head: y4 float32 [n][h][w][4] -> vis (and logits when non-null)
// float32 [n][2h][2w].
hipError_t d2s_forward(const float* y4, int n, int h, int w, float* vis, float* logits, hipStream_t s);

// ------------------------------------------------------ backward (float32)
bool backward_supported(const ConvStage& st);
size_t head_partial_floats(int c0, size_t npix);
hipError_t head_backward(int c0, const float* vis, const float* dvis, const float* act,
                         const float* head_w, size_t npix, float* dz, float* partial, hipStream_t s);
hipError_t head_reduce(int c0, const float* partial, size_t npix, float* dw, bool accumulate,
                       hipStream_t s);
// dz_low = upsample^T(dup[..., c_off : c_off + c]) * (act_low > 0)
hipError_t up_transpose_mask(int c, int ci_total, int c_off, const float* dup, const float* act_low,
                             int n, int hl, int wl, float* dz_low, hipStream_t s);
// dz = (dskip[..., :c] + maxpool^T(dpool)) * (act > 0)
hipError_t pool_transpose_mask(int c, int ci_total, const float* dskip, const float* dpool,
                               const float* act, int n, int h, int w, float* dz, hipStream_t s);
size_t wgrad_partial_floats(const ConvStage& st, int n, int h, int w);
hipError_t conv_wgrad(const ConvStage& st, const float* in, const float* low, const float* dz, int n,
                      int h, int w, float* partial, float* dw, float* db, bool accumulate, hipStream_t s);
size_t dgrad_packed_bytes(const ConvStage& st);
hipError_t pack_dgrad_weights(const ConvStage& st, const float* w_ohwi, void* packed, hipStream_t s);
hipError_t conv_dgrad(const ConvStage& st, const void* wpk, const float* dz, int n, int h, int w,
                      float* dx, hipStream_t s);

}  // namespace nsm
