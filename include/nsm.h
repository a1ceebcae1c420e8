/*
 * nsm.h -- C ABI of the neural shadow-mapping hot path on MI355X (gfx950).
 *
 * The method (Datta et al., "Neural Shadow Mapping", SIGGRAPH 2022) takes the
 * buffers of a vanilla rasterised shadow-mapping pipeline -- a G-buffer with
 * view depth and normals, a single light-view depth map, the receiver's
 * depth towards the emitter and the emitter size -- composes a few
 * screen-space feature channels from them (Sec. 3.1, 3.2) and runs a compact
 * U-Net (Sec. 3.5) that outputs per-pixel shadow visibility in [0, 1].
 *
 * Three calls make up the path:
 *   nsm_build_features  light-view z-buffer, camera G-buffer, feature gather
 *   nsm_forward         U-Net inference (FP32, or BF16/FP16 on MFMA)
 *   nsm_backward        gradient of the visibility w.r.t. the weights and
 *                       the features (the differentiation form; FP32;
 *                       nsm_forward_train + nsm_backward_saved split it
 *                       around the loss without recomputing the forward)
 * and two around it for temporal stability:
 *   nsm_perturbation_loss     Eq. 2's loss and its gradient through x_0
 *   nsm_temporal_instability  Eq. 3's metric over a pair of frames
 *
 * Conventions shared by every call:
 *   - Every tensor argument is a device pointer owned by the caller unless
 *     marked "host".  The library never allocates or frees inside these
 *     calls; scratch memory is the caller's `workspace`, sized by the
 *     matching *_workspace_bytes query.  The one allocation the library
 *     makes is the context's packed weight copy, in nsm_set_weights.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is
 *     the null stream).  Inputs must stay valid until the stream has run.
 *   - All arguments are validated before anything is launched; a non-OK
 *     status means nothing was enqueued.  Faults inside kernels surface at
 *     the caller's next synchronisation.  No C++ exception crosses the ABI.
 *   - Debug mode: with the environment variable NSM_DEBUG_SYNC=1 (read at
 *     every call), each call synchronises its stream after every kernel it
 *     launches and returns NSM_E_LAUNCH if the launch or the kernel failed,
 *     so a fault is reported by the call that caused it.  Results are the
 *     same bits as without it; only the calls become blocking.
 *   - Images are row-major with row 0 at the bottom (ndc y = -1) and the
 *     column index growing with ndc x; tensors are NHWC.
 *   - A context is not internally synchronised: use one per stream.  Its
 *     packed weights are read by every nsm_forward / nsm_backward, so a
 *     nsm_set_weights on one stream must be ordered (events) against calls
 *     on other streams that use the same context; likewise a workspace
 *     must not be shared by calls that may run concurrently.
 *   - Triangle counts are at most 2^28 (NSM_E_SHAPE above).
 */
#ifndef NSM_H
#define NSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NSM_ABI_VERSION 3

typedef enum {
    NSM_OK = 0,
    NSM_E_INVALID_ARG = 1,  /* null pointer, negative size, bad enum value      */
    NSM_E_SHAPE = 2,        /* H or W not divisible by 2^(levels-1), size limits */
    NSM_E_UNSUPPORTED = 3,  /* network or dtype the library has no kernels for   */
    NSM_E_WORKSPACE = 4,    /* workspace missing or smaller than required        */
    NSM_E_NO_WEIGHTS = 5,   /* nsm_set_weights has not been called               */
    NSM_E_DEVICE = 6,       /* no HIP device, or a HIP runtime call failed       */
    NSM_E_LAUNCH = 7        /* a kernel launch was rejected                      */
} nsm_status;

typedef enum { NSM_F32 = 0, NSM_BF16 = 1, NSM_F16 = 2, NSM_F8 = 3, NSM_F8_MFMA = 4 } nsm_dtype;

/* Feature sets (channel order, NHWC, float32):
 *   HARD6:  [d/f_C, n.x, n.y, n.z, (z - z_f)/f_L, z/f_L]
 *   SOFT8:  HARD6 + [r_e/0.2, z_blk/f_L]
 *   PAPER4: [c_e + r_e/0.0625, z/z_f, (z - z_f)/f_L, c_c/d], the set the paper
 *           selects (Sec. 3.2); c_e = n.l and c_c = n.v are the cosines with
 *           the emitter and view directions, and the emitter size enters as a
 *           DC offset on c_e on the paper's 0..4 scale (Sec. 3.1.1; 4 = radius
 *           0.25 scene units, i.e. a 50 cm diameter with metres as units).
 * d: view depth along the camera axis; n: face normal turned towards the
 * camera; z: light-view linear depth stored in the shadow map at the
 * receiver's texel; z_f: the receiver's own light-view linear depth; r_e:
 * emitter radius; z_blk: mean linear depth of the 7x7 map texels in front
 * of the receiver (z_f when there are none).  Background pixels are 0. */
typedef enum { NSM_FEAT_HARD6 = 0, NSM_FEAT_SOFT8 = 1, NSM_FEAT_PAPER4 = 2 } nsm_feature_set;

typedef struct nsm_ctx nsm_ctx;

/* Network architectures.
 * NSM_ARCH_UNET: `levels` resolution levels with channel widths
 *   widths[0..levels-1].  Stages, in execution order: encoder 3x3 conv +
 *   ReLU + 2x2 max-pool for levels 0..L-2, bottleneck 3x3 conv + ReLU at
 *   level L-1, decoder bilinear x2 upsample, concat [skip, up], 3x3 conv +
 *   ReLU for levels L-2..0, then a 1x1 head to one channel and a sigmoid
 *   (one 3x3 conv per level and bilinear upsampling follow Sec. 3.5).
 *   Supported: c_in in {6, 8}; widths {8, 16} or {16, 32, 64}.
 * NSM_ARCH_PAPER: the paper's trimmed network (Sec. 3.5): per level a 3x3
 *   and a 1x1 conv (each + ReLU); 2x2 average pooling; decoder input
 *   up(y_{l+1}) + x_l (sum skip) for l >= 1 and up(y_1) alone at level 0;
 *   encoder level l: 3x3 C_{l-1} -> w_l, 1x1 w_l -> w_l; bottleneck: 3x3
 *   w_{L-2} -> w_{L-1}, 1x1 w_{L-1} -> w_{L-2}; decoder level l >= 1:
 *   3x3 w_l -> w_l, 1x1 w_l -> w_{l-1}; level 0: 3x3 and 1x1 w_0 -> w_0,
 *   then a 1x1 output conv to one channel and a sigmoid.  Flat parameters
 *   list the convs in that order (each OHWI weights then biases).
 *   Supported: c_in = 4; widths {16, 32, 64} or {16, 32, 64, 128, 256}.
 * NSM_ARCH_PAPER_S2D: the paper's network after its first-level optimisation
 *   (Sec. 3.5): the level-0 convolutions are removed.  The input is read as
 *   2x2 blocks, (h, w, c_in) -> (h/2, w/2, 4 c_in), channel (2 dy + dx) c_in
 *   + c of block (i, j) being channel c of pixel (2i + dy, 2j + dx), and
 *   feeds the level-1 encoder (3x3 4 c_in -> w_1).  Levels 1..L-1 are those
 *   of NSM_ARCH_PAPER; the level-1 decoder's 1x1 (w_1 -> w_0) is followed by
 *   a 1x1 output conv w_0 -> 4.  Full-resolution logit at (2i + dy, 2j + dx):
 *   the bilinear x2 upsampling of output channel 0, plus output channel
 *   2 dy + dx unless dy = dx = 0; then the sigmoid.  Flat parameters: the
 *   convs of NSM_ARCH_PAPER without E0 and D0, the output conv last
 *   ([4][w_0] then 4 biases).  h and w must be even (and multiples of
 *   2^(L-1) as for every network).  Supported: c_in = 4; widths {16, 32, 64}
 *   or {16, 32, 64, 128, 256}. */
typedef enum { NSM_ARCH_UNET = 0, NSM_ARCH_PAPER = 1, NSM_ARCH_PAPER_S2D = 2 } nsm_arch;

typedef struct nsm_net_desc {
    int32_t arch;       /* nsm_arch */
    int32_t c_in;
    int32_t levels;
    int32_t widths[8];
} nsm_net_desc;

/* Per-frame light and camera (host struct, float32).  Matrices are
 * row-major world -> clip with depth range [0, 1]; w_clip is the depth along
 * the view axis.  The camera basis and tangents define the pixel-centre
 * rays used to place each receiver on its triangle's plane. */
typedef struct nsm_frame_params {
    float m_light[16];
    float light_pos[3];
    float light_radius;         /* r_e; 0 for a point light               */
    float light_near;
    float light_far;            /* f_L                                    */
    float light_tan_half_fov;   /* square light frustum                   */
    int32_t sm_size;            /* S: the shadow map is S x S             */
    float m_cam[16];
    float cam_pos[3];
    float cam_fwd[3];
    float cam_right[3];
    float cam_up[3];
    float cam_tan_half_x;
    float cam_tan_half_y;
    float cam_near;
    float cam_far;              /* f_C                                    */
} nsm_frame_params;

/* Library metadata. */
int nsm_abi_version(void);
const char *nsm_status_str(int status);

/* ------------------------------------------------------------ features
 * nsm_build_features -- one frame's network input from raw geometry
 * (paper Sec. 3.1: "a G-buffer pass followed by a shadow mapping pass").
 *
 *   tris        [n_tris][3][3] float32, world-space vertices.
 *   tri_normals [n_tris][3] float32 unit face normals.
 *   fp          host; light and camera for this frame.
 *   h, w        screen size (1..16384 each); sm_size likewise.
 *   fs          feature set (HARD6, SOFT8 or PAPER4).
 *   gbuf_in     [h][w] uint64 camera key buffer to use as the G-buffer, or
 *               NULL to rasterise it from `tris` with fp->m_cam.
 *   gbuf_out    [h][w] uint64; where the camera raster writes when gbuf_in
 *               is NULL (NULL = keep it in the workspace).  Key =
 *               depth_bits << 32 | triangle id, all ones where empty.
 *   sm_out      [S][S] uint32 light-view depth bits (float32 ndc depth in
 *               [0, 1], +inf bits where empty).
 *   feat_out    [h][w][C] float32, C = 6 (HARD6), 8 (SOFT8) or 4 (PAPER4).
 *   mask_out    [h][w] uint8 hard depth-test result (1 = shadowed), or NULL.
 * The rasteriser and the gather are deterministic: repeated calls give
 * identical bits.  With SOFT8 the workspace also holds the linear-depth copy
 * of the light-view map that the z_blk search reads.  Triangles with a vertex at w_clip <= 1e-6 or beyond the
 * guard band [-8, 9] x the target size are skipped. */
nsm_status nsm_features_workspace_bytes(int n_tris, int h, int w, int sm_size, size_t *bytes);
nsm_status nsm_build_features(const float *tris, const float *tri_normals, int n_tris,
                              const nsm_frame_params *fp, int h, int w, nsm_feature_set fs,
                              const uint64_t *gbuf_in, uint64_t *gbuf_out, uint32_t *sm_out,
                              float *feat_out, uint8_t *mask_out, void *workspace,
                              size_t ws_bytes, void *stream);

/* nsm_build_features_stored -- the same features written in a network
 * context's storage type, the input nsm_forward_stored reads (the paper's
 * network runs in half precision, Sec. 3.5, so its input can be handed over
 * at half the bytes; a first stage given float32 features rounds them to the
 * storage type anyway).
 *   feat_dtype  NSM_BF16, NSM_F16 or NSM_F8_MFMA (NSM_E_INVALID_ARG
 *               otherwise).
 *   feat_out    NSM_BF16 / NSM_F16: [h][w][8] of that type, channel c < C
 *               the float32 feature of nsm_build_features rounded to
 *               nearest even, channels C..7 zero.  NSM_F8_MFMA: [h][w][16]
 *               E4M3 bytes, channel c < C the feature saturated to +-448
 *               and rounded to nearest even, bytes C..15 zero.  HARD6 and
 *               SOFT8 only (NSM_E_UNSUPPORTED for PAPER4).
 * Every other argument, the workspace and the error behaviour are those of
 * nsm_build_features. */
nsm_status nsm_build_features_stored(const float *tris, const float *tri_normals, int n_tris,
                                     const nsm_frame_params *fp, int h, int w, nsm_feature_set fs,
                                     const uint64_t *gbuf_in, uint64_t *gbuf_out, uint32_t *sm_out,
                                     nsm_dtype feat_dtype, void *feat_out, uint8_t *mask_out,
                                     void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------- network
 * nsm_create -- a context for one network descriptor and compute dtype.
 * Host only (no device call).  NSM_F32 runs the FP32 network; NSM_BF16 and
 * NSM_F16 run the precision form (activations and 3x3 weights stored in
 * that type, MFMA products accumulated in float32; the paper quantises its
 * network to half precision, Sec. 3.5).  Inputs and outputs of every call
 * stay float32, except the features nsm_forward_stored takes in the storage
 * type.  Decoder stages fold the bilinear x2 upsampling into their
 * weights away from the image border (four phase kernels per stage, formed
 * in float64 and rounded once to the storage type), so the upsampled tensor
 * is never rounded to the storage type there.
 * NSM_F8 is 8-bit temporary storage (suggested as future work in the
 * paper's supplemental Sec. 3 and Sec. 8): activations between stages are
 * stored as FP8 E4M3 (OCP: bias 7, 3 mantissa bits, saturated to +-448,
 * rounded to nearest even), widened to bfloat16 when staged, and computed
 * with bfloat16 weights on bfloat16 MFMA; it halves the activation bytes of
 * NSM_BF16 at E4M3's precision (relative step 1/8).  NSM_ARCH_UNET only
 * (NSM_E_UNSUPPORTED otherwise).
 * NSM_F8_MFMA is the same 8-bit storage with FP8 arithmetic: features are
 * rounded to E4M3 on load, the 3x3 weights (and the decoders' phase kernels)
 * to E4M3, the LDS tiles hold E4M3 and the products run on the FP8 MFMA
 * (v_mfma_f32_16x16x32_fp8_fp8), accumulating in float32; biases, the head
 * and the sigmoid stay float32.  Its kernels take 16 channels per 16-byte
 * block, so every stored tensor must have a multiple of 16 channels: the
 * U-Nets with widths {16, 32, 64} (NSM_E_UNSUPPORTED for {8, 16}). */
nsm_status nsm_create(const nsm_net_desc *desc, nsm_dtype dtype, nsm_ctx **out);
nsm_status nsm_destroy(nsm_ctx *ctx);

/* Number of float32 entries in the flat parameter vector: stages in
 * execution order E0..E(L-2), B, D(L-2)..D0, H; each stage's weights in
 * OHWI order [C_out][k][k][C_in] followed by its biases [C_out]. */
nsm_status nsm_param_count(const nsm_ctx *ctx, size_t *n);

/* Copies (and converts / repacks) the flat float32 parameter vector `w`
 * (device pointer, n entries) into the context.  Allocates the context's
 * device copy on first use.  The caller may free `w` once the stream has
 * run this call. */
nsm_status nsm_set_weights(nsm_ctx *ctx, const float *w, size_t n, void *stream);

/* Workspace bytes for nsm_forward (training = 0) or nsm_backward
 * (training = 1) on n frames of h x w. */
nsm_status nsm_workspace_bytes(const nsm_ctx *ctx, int n, int h, int w, int training,
                               size_t *bytes);

/* nsm_forward -- visibility for n frames.
 *   feat       [n][h][w][c_in] float32.
 *   vis_out    [n][h][w] float32 in (0, 1).
 *   logits_out [n][h][w] float32 pre-sigmoid values, or NULL.
 * h and w must be divisible by 2^(levels-1).
 * On return (once the stream has run) the workspace holds the stored
 * activations of NSM_ARCH_UNET, in the context's storage type (float32,
 * bfloat16, float16, or E4M3 bytes for NSM_F8), NHWC over the n frames, each
 * tensor starting at a multiple of 256 bytes right after the previous one:
 * for l = 0 .. L-2 the encoder output e_l (h_l x w_l x widths[l], post-ReLU)
 * then its 2x2 max-pool p_l; the bottleneck output b; the decoder outputs
 * d_l for l = 1 .. L-2 (h_l = h >> l).  The level-0 decoder output feeds the
 * head in float32 registers and is not stored.  This layout lets a caller
 * inspect intermediate tensors; it is fixed for a given ABI version. */
nsm_status nsm_forward(nsm_ctx *ctx, const float *feat, int n, int h, int w, float *vis_out,
                       float *logits_out, void *workspace, size_t ws_bytes, void *stream);

/* nsm_forward_stored -- nsm_forward on features already in the context's
 * storage type (NSM_BF16, NSM_F16 and NSM_F8_MFMA contexts of
 * NSM_ARCH_UNET with c_in 6 or 8; NSM_E_UNSUPPORTED otherwise).
 *   feat  the layout of nsm_build_features_stored for the context's dtype:
 *         [n][h][w][8] bfloat16 / float16, or [n][h][w][16] E4M3 bytes;
 *         channels past c_in zero.
 * Gives the same bits as nsm_forward on the float32 features that round to
 * `feat`: the float32 path rounds each feature the same way when it stages
 * the first tile.  Workspace, outputs and errors as nsm_forward. */
nsm_status nsm_forward_stored(nsm_ctx *ctx, const void *feat, int n, int h, int w, float *vis_out,
                              float *logits_out, void *workspace, size_t ws_bytes, void *stream);

/* Launch variants of the NSM_ARCH_UNET forward stages (the batched
 * multi-frame pipeline's tuning knob).  Each stage can run as one workgroup
 * per output tile (variant bit 0 clear) or as a persistent grid sized to the
 * device's resident capacity that strides over the tiles (bit 0 set), with
 * its default or its alternative tile height (bit 1).  Every variant
 * computes each output with the same arithmetic in the same order, so all
 * give the same bits; only the speed differs.
 *
 * nsm_autotune times every variant of every stage on the caller's input
 * (one forward first, so that each stage reads real data; then per stage
 * and variant one untimed and `reps` timed launches between hipEvents on
 * `stream`) and keeps the fastest in the context.  It synchronises the
 * stream, so call it before capturing a graph, never inside one.
 *   feat      [n][h][w][c_in] float32; vis_out [n][h][w] float32 (scratch
 *             output of the timed launches); workspace as for nsm_forward.
 *   reps      1..1000.
 *   variants_out  host int[number of stages] or NULL: the chosen variants,
 *             stages in execution order.
 * nsm_set_stage_variant sets one stage's variant (0..3) by hand;
 * nsm_get_stage_variants copies up to `max` of them and the stage count.
 * NSM_E_UNSUPPORTED for the paper's architectures. */
nsm_status nsm_autotune(nsm_ctx *ctx, const float *feat, int n, int h, int w, float *vis_out,
                        void *workspace, size_t ws_bytes, int reps, int *variants_out, void *stream);
/* nsm_autotune_stored -- nsm_autotune timing the stages as nsm_forward_stored
 * runs them (feat as for nsm_forward_stored; NSM_E_UNSUPPORTED where that
 * call is).  The chosen variants serve both forward calls. */
nsm_status nsm_autotune_stored(nsm_ctx *ctx, const void *feat, int n, int h, int w, float *vis_out,
                               void *workspace, size_t ws_bytes, int reps, int *variants_out,
                               void *stream);
nsm_status nsm_set_stage_variant(nsm_ctx *ctx, int stage, int variant);
nsm_status nsm_get_stage_variants(const nsm_ctx *ctx, int *variants, int max, int *n_stages);

/* nsm_backward -- gradient of sum(dvis * vis) (FP32 NSM_ARCH_UNET contexts):
 * the network's training pass (paper Sec. 3.3 trains the network on
 * per-pixel losses against ray-traced targets; supplemental Sec. 5 on the
 * temporal windows), so dvis is the loss gradient with respect to the
 * visibility (e.g. 2 (vis - target) / (n h w) for the mean squared error).
 * Recomputes the forward activations into the workspace, then applies the
 * adjoint of every stage: the sigmoid and 1x1 head, each 3x3 convolution
 * (input gradient by the flipped kernel, weight gradient as a sum over
 * pixels), ReLU (gradient where the pre-activation is > 0), the concat
 * split, the bilinear upsampling's transpose and the max-pool routing to
 * the first maximum of each window in (0,0), (0,1), (1,0), (1,1) order.
 *   dvis       [n][h][w] float32 upstream gradient.
 *   dw_out     [n_params] float32 in the flat parameter order; overwritten,
 *              or added to when accumulate != 0.
 *   dfeat_out  [n][h][w][c_in] float32 gradient w.r.t. the features, or NULL.
 * The weight gradients are reduced in a fixed order (no float atomics), so
 * results are bitwise reproducible. */
nsm_status nsm_backward(nsm_ctx *ctx, const float *feat, const float *dvis, int n, int h, int w,
                        float *dw_out, int accumulate, float *dfeat_out, void *workspace,
                        size_t ws_bytes, void *stream);

/* nsm_forward_train / nsm_backward_saved -- the same training pass without
 * the recomputed forward: backpropagation reuses the forward's activations
 * (paper Sec. 3.3 trains by gradient descent; this pair only moves where the
 * activations come from).  nsm_forward_train runs the FP32 forward with the
 * training workspace (nsm_workspace_bytes with training = 1), keeps every
 * activation there and copies the visibility to vis_out ([n][h][w] float32,
 * or NULL); its visibility is the same bits as nsm_forward's.
 * nsm_backward_saved then computes what nsm_backward computes, the same bits,
 * from those activations.  It requires that the last call on this context
 * that used a workspace was nsm_forward_train or nsm_backward (either
 * flavour) with the same workspace, feature pointer, n, h and w, and that
 * nsm_set_weights has not been called since; otherwise it returns
 * NSM_E_INVALID_ARG and enqueues nothing.  The caller must not modify the
 * workspace or the features in between (the library cannot check that).
 * nsm_forward, nsm_autotune and nsm_set_weights forget the saved forward. */
nsm_status nsm_forward_train(nsm_ctx *ctx, const float *feat, int n, int h, int w, float *vis_out,
                             void *workspace, size_t ws_bytes, void *stream);
nsm_status nsm_backward_saved(nsm_ctx *ctx, const float *feat, const float *dvis, int n, int h, int w,
                              float *dw_out, int accumulate, float *dfeat_out, void *workspace,
                              size_t ws_bytes, void *stream);

/* --------------------------------------------------- temporal stability
 * nsm_perturbation_loss -- the perturbation loss of paper Sec. 3.3, Eq. 2,
 * with its per-pixel term L(y, y~) = alpha * mean |y - y~| (the perceptual
 * term is not part of this library).  For each of n samples, x_0 is the
 * network output on the unperturbed input, x_1..x_p the outputs on p
 * perturbed inputs and x~ the target:
 *     loss = alpha / (n h w) * sum ( |x_0 - x~| + sum_i |x_0 - x_i| )
 * and its gradient with respect to x_0 alone (x_1..x_p are held constant,
 * as in the paper only one instance back-propagates), sgn(0) taken as 0:
 *     dvis0 = alpha / (n h w) * ( sgn(x_0 - x~) + sum_i sgn(x_0 - x_i) ).
 *   vis        [n][1+p][h][w] float32 (x_0 first in every sample).
 *   target     [n][h][w] float32.
 *   p          0..16 (the paper uses 3).
 *   loss_out   [1] float64, overwritten.
 *   dvis0_out  [n][h][w] float32, overwritten; feed it to nsm_backward with
 *              the x_0 features.
 * The sums are float64 and deterministic (fixed reduction order).
 * Errors: NSM_E_SHAPE for n, p, h, w out of range; NSM_E_WORKSPACE below
 * nsm_perturbation_loss_workspace_bytes. */
nsm_status nsm_perturbation_loss_workspace_bytes(int n, int p, int h, int w, size_t *bytes);
nsm_status nsm_perturbation_loss(const float *vis, const float *target, int n, int p, int h, int w,
                                 float alpha, double *loss_out, float *dvis0_out, void *workspace,
                                 size_t ws_bytes, void *stream);

/* nsm_perturbation_loss_noalloc -- nsm_perturbation_loss for callers that
 * cannot allocate device memory or pass a workspace (code under hipGraph
 * capture, tight serving or training loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors, minus the workspace: the
 * per-block partial sums live in a 2 MiB array that the library holds on
 * each device it runs on until the process ends, so n * h * w is at most
 * 67,108,864 pixels (NSM_E_SHAPE above).  It makes no allocation of any kind;
 * the first call on a device looks up that device's copy of the array
 * (NSM_E_DEVICE if that fails).  The kernels and the reduction order are
 * those of nsm_perturbation_loss, so both give identical bits.  Every call
 * on one device shares the array: calls that may overlap on one device (two
 * streams, two threads) race and must be ordered by the caller. */
nsm_status nsm_perturbation_loss_noalloc(const float *vis, const float *target, int n, int p, int h,
                                         int w, float alpha, double *loss_out, float *dvis0_out,
                                         void *stream);

/* nsm_temporal_instability -- one frame pair of the temporal-instability
 * metric of paper Sec. 3.4, Eq. 3:
 *     E = (1/P) sum_{p,t} [exp(alpha D_t(p)) - 1],  D_t(p) = |I_t(p) - I_{t-1}(m(p))|.
 * Adds this pair's sum of exp(alpha D) - 1 to acc_out[0] and its number of
 * contributing pixels to acc_out[1] (or overwrites both when accumulate is
 * 0); call once per consecutive pair and divide acc_out[0] by P (the paper's
 * normaliser, the total pixel count, w h (T - 1) for T frames).
 * Per pixel p = (i, j) of the current frame:
 *   - background (empty key) contributes nothing;
 *   - the receiver P (pixel-centre ray / key triangle plane, float64
 *     rounded to float32) and its camera-facing face normal n;
 *   - m(p): P projected with prev->m_cam (float32, products and sums in
 *     order, as the rasteriser's vertex transform), c_w <= 1e-6 or outside
 *     [0, w) x [0, h) rejects, else the pixel (floor(sx), floor(sy));
 *   - rejected when the previous key at m(p) is empty, when the view depths
 *     of P and of the previous receiver P' along prev's camera axis differ
 *     by more than depth_tol * depth(P'), or when n . n' < cos_tol.
 * Scenes are static (camera and light move), so reprojecting P is the
 * motion-vector lookup.  The paper does not give the thresholds; 0.01 and
 * 0.9 are this library's defaults in the Python binding.
 *   tris, tri_normals  the scene, as in nsm_build_features.
 *   gbuf_prev/cur      [h][w] camera keys of the two frames (as written by
 *                      nsm_build_features).
 *   vis_prev/cur       [h][w] float32 network outputs I_{t-1}, I_t.
 *   acc_out            [2] float64 (device).
 *   d_out              [h][w] float32 or NULL: D(p) where the pixel counted,
 *                      else -1 background, -2 off-screen, -3 empty previous
 *                      pixel, -4 depth, -5 normal.
 * Deterministic. Errors: NSM_E_SHAPE for h, w out of range;
 * NSM_E_WORKSPACE below nsm_temporal_workspace_bytes. */
nsm_status nsm_temporal_workspace_bytes(int h, int w, size_t *bytes);
nsm_status nsm_temporal_instability(const float *tris, const float *tri_normals, int n_tris,
                                    const nsm_frame_params *prev, const nsm_frame_params *cur,
                                    const uint64_t *gbuf_prev, const uint64_t *gbuf_cur,
                                    const float *vis_prev, const float *vis_cur, int h, int w, float alpha,
                                    float depth_tol, float cos_tol, int accumulate, double *acc_out,
                                    float *d_out, void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------- diagnostics
 * Per-kernel timing.  While enabled (process-wide), every kernel the
 * library launches is bracketed by two hipEvents recorded on its launch
 * stream, so the measured time is the kernel's own execution.
 * nsm_trace_read waits for the recorded events, writes up to max_records
 * entries (names: max_records x 64 chars, NUL-terminated; ms: durations)
 * in launch order, stores the number of records consumed in *n_out and
 * clears the list.  Tracing adds the event records between launches, so
 * time whole calls with tracing off. */
nsm_status nsm_trace_enable(int on);
nsm_status nsm_trace_read(int max_records, char *names, float *ms, int *n_out);

#ifdef __cplusplus
}
#endif
#endif /* NSM_H */
