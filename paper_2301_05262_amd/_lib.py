"""ctypes binding of ``libnsm.so`` with the C-ABI's names.

Argument marshalling only: tensors are passed as raw device pointers and
every step of the path runs in the library's HIP kernels.  There is no
fallback: if the library has not been built the import of any entry point
raises.

With ``NSM_TRACE=1`` in the environment the library's per-kernel timing is
switched on when it is loaded, and at interpreter exit every kernel's call
count, median and total time are printed to stderr (the records accumulate
until then, so use it on bounded runs).
"""
import atexit
import ctypes
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libnsm.so")

NSM_OK = 0
STATUS_NAMES = {0: "NSM_OK", 1: "NSM_E_INVALID_ARG", 2: "NSM_E_SHAPE", 3: "NSM_E_UNSUPPORTED",
                4: "NSM_E_WORKSPACE", 5: "NSM_E_NO_WEIGHTS", 6: "NSM_E_DEVICE", 7: "NSM_E_LAUNCH"}
DTYPES = {"f32": 0, "bf16": 1, "f16": 2, "f8": 3, "f8mfma": 4}
FEATURE_SETS = {"hard6": 0, "soft8": 1, "paper4": 2}
FEATURE_CHANNELS = {"hard6": 6, "soft8": 8, "paper4": 4}
ARCHS = {"unet": 0, "paper": 1, "paper_s2d": 2}

EXPORTS = [
    "nsm_abi_version", "nsm_status_str", "nsm_features_workspace_bytes", "nsm_build_features",
    "nsm_build_features_stored", "nsm_forward_stored", "nsm_autotune_stored",
    "nsm_create", "nsm_destroy", "nsm_param_count", "nsm_set_weights", "nsm_workspace_bytes",
    "nsm_forward", "nsm_backward", "nsm_forward_train", "nsm_backward_saved", "nsm_trace_enable", "nsm_trace_read", "nsm_autotune",
    "nsm_set_stage_variant", "nsm_get_stage_variants",
    "nsm_perturbation_loss_workspace_bytes", "nsm_perturbation_loss", "nsm_perturbation_loss_noalloc",
    "nsm_temporal_workspace_bytes",
    "nsm_temporal_instability",
]


class NsmError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}")


class NetDesc(ctypes.Structure):
    _fields_ = [("arch", ctypes.c_int32), ("c_in", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("widths", ctypes.c_int32 * 8)]


class FrameParams(ctypes.Structure):
    _fields_ = [
        ("m_light", ctypes.c_float * 16), ("light_pos", ctypes.c_float * 3),
        ("light_radius", ctypes.c_float), ("light_near", ctypes.c_float),
        ("light_far", ctypes.c_float), ("light_tan_half_fov", ctypes.c_float),
        ("sm_size", ctypes.c_int32), ("m_cam", ctypes.c_float * 16),
        ("cam_pos", ctypes.c_float * 3), ("cam_fwd", ctypes.c_float * 3),
        ("cam_right", ctypes.c_float * 3), ("cam_up", ctypes.c_float * 3),
        ("cam_tan_half_x", ctypes.c_float), ("cam_tan_half_y", ctypes.c_float),
        ("cam_near", ctypes.c_float), ("cam_far", ctypes.c_float),
    ]


_lib = None


def load():
    """Load libnsm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    psz = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "nsm_abi_version": ([], i32),
        "nsm_status_str": ([i32], ctypes.c_char_p),
        "nsm_features_workspace_bytes": ([i32, i32, i32, i32, psz], i32),
        "nsm_build_features": ([vp, vp, i32, ctypes.POINTER(FrameParams), i32, i32, i32, vp, vp, vp,
                                vp, vp, vp, sz, vp], i32),
        "nsm_build_features_stored": ([vp, vp, i32, ctypes.POINTER(FrameParams), i32, i32, i32, vp, vp, vp,
                                       i32, vp, vp, vp, sz, vp], i32),
        "nsm_forward_stored": ([vp, vp, i32, i32, i32, vp, vp, vp, sz, vp], i32),
        "nsm_autotune_stored": ([vp, vp, i32, i32, i32, vp, vp, sz, i32, ctypes.POINTER(ctypes.c_int), vp], i32),
        "nsm_create": ([ctypes.POINTER(NetDesc), i32, ctypes.POINTER(vp)], i32),
        "nsm_destroy": ([vp], i32),
        "nsm_param_count": ([vp, psz], i32),
        "nsm_set_weights": ([vp, vp, sz, vp], i32),
        "nsm_workspace_bytes": ([vp, i32, i32, i32, i32, psz], i32),
        "nsm_forward": ([vp, vp, i32, i32, i32, vp, vp, vp, sz, vp], i32),
        "nsm_backward": ([vp, vp, vp, i32, i32, i32, vp, i32, vp, vp, sz, vp], i32),
        "nsm_forward_train": ([vp, vp, i32, i32, i32, vp, vp, sz, vp], i32),
        "nsm_backward_saved": ([vp, vp, vp, i32, i32, i32, vp, i32, vp, vp, sz, vp], i32),
        "nsm_trace_enable": ([i32], i32),
        "nsm_autotune": ([vp, vp, i32, i32, i32, vp, vp, sz, i32, ctypes.POINTER(ctypes.c_int), vp], i32),
        "nsm_set_stage_variant": ([vp, i32, i32], i32),
        "nsm_get_stage_variants": ([vp, ctypes.POINTER(ctypes.c_int), i32, ctypes.POINTER(ctypes.c_int)], i32),
        "nsm_perturbation_loss_workspace_bytes": ([i32, i32, i32, i32, psz], i32),
        "nsm_perturbation_loss": ([vp, vp, i32, i32, i32, i32, ctypes.c_float, vp, vp, vp, sz, vp], i32),
        "nsm_perturbation_loss_noalloc": ([vp, vp, i32, i32, i32, i32, ctypes.c_float, vp, vp, vp], i32),
        "nsm_temporal_workspace_bytes": ([i32, i32, psz], i32),
        "nsm_temporal_instability": ([vp, vp, i32, ctypes.POINTER(FrameParams), ctypes.POINTER(FrameParams),
                                      vp, vp, vp, vp, i32, i32, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, i32, vp, vp, vp, sz, vp], i32),
        "nsm_trace_read": ([i32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_float),
                            ctypes.POINTER(ctypes.c_int)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    if os.environ.get("NSM_TRACE") == "1":
        _check(L.nsm_trace_enable(1), "nsm_trace_enable")
        atexit.register(_trace_report)
    return L


def _trace_report():
    """Per-kernel summary of the trace records (NSM_TRACE=1), to stderr."""
    per = {}
    for name, ms in nsm_trace_read(1 << 18):
        per.setdefault(name, []).append(ms)
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        v = sorted(v)
        print(f"nsm trace: {name}: {len(v)} calls, median {1e3 * v[len(v) // 2]:.2f} us, "
              f"total {1e3 * sum(v):.1f} us", file=sys.stderr)


def _ptr(t):
    """Device pointer of a tensor (or None)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _check(status, where):
    if status != NSM_OK:
        raise NsmError(status, where)


# ------------------------------------------------------------ entry points
def nsm_abi_version():
    return load().nsm_abi_version()


def nsm_status_str(status):
    return load().nsm_status_str(int(status)).decode()


def nsm_features_workspace_bytes(n_tris, h, w, sm_size):
    out = ctypes.c_size_t()
    _check(load().nsm_features_workspace_bytes(n_tris, h, w, sm_size, ctypes.byref(out)),
           "nsm_features_workspace_bytes")
    return out.value


def frame_params(fr):
    """ctypes FrameParams from an nsm_synth FrameParams."""
    p = FrameParams()
    p.m_light[:] = [float(v) for v in fr.m_light.reshape(-1)]
    p.light_pos[:] = [float(v) for v in fr.light_pos]
    p.light_radius = fr.light_radius
    p.light_near = fr.light_near
    p.light_far = fr.light_far
    p.light_tan_half_fov = fr.light_tan_half_fov
    p.sm_size = fr.sm_size
    p.m_cam[:] = [float(v) for v in fr.m_cam.reshape(-1)]
    p.cam_pos[:] = [float(v) for v in fr.cam_pos]
    p.cam_fwd[:] = [float(v) for v in fr.cam_fwd]
    p.cam_right[:] = [float(v) for v in fr.cam_right]
    p.cam_up[:] = [float(v) for v in fr.cam_up]
    p.cam_tan_half_x = fr.cam_tan_half_x
    p.cam_tan_half_y = fr.cam_tan_half_y
    p.cam_near = fr.cam_near
    p.cam_far = fr.cam_far
    return p


def nsm_build_features(tris, tri_normals, n_tris, fp, h, w, fs, gbuf_in, gbuf_out, sm_out, feat_out,
                       mask_out, workspace, ws_bytes, stream=None):
    if not isinstance(fp, FrameParams):
        fp = frame_params(fp)
    fs = FEATURE_SETS.get(fs, fs)
    _check(load().nsm_build_features(_ptr(tris), _ptr(tri_normals), n_tris, ctypes.byref(fp), h, w,
                                     fs, _ptr(gbuf_in), _ptr(gbuf_out), _ptr(sm_out), _ptr(feat_out),
                                     _ptr(mask_out), _ptr(workspace), ws_bytes, _stream(stream)),
           "nsm_build_features")


def nsm_build_features_stored(tris, tri_normals, n_tris, fp, h, w, fs, gbuf_in, gbuf_out, sm_out, feat_dtype,
                              feat_out, mask_out, workspace, ws_bytes, stream=None):
    if not isinstance(fp, FrameParams):
        fp = frame_params(fp)
    fs = FEATURE_SETS.get(fs, fs)
    _check(load().nsm_build_features_stored(_ptr(tris), _ptr(tri_normals), n_tris, ctypes.byref(fp), h, w,
                                            fs, _ptr(gbuf_in), _ptr(gbuf_out), _ptr(sm_out),
                                            DTYPES.get(feat_dtype, feat_dtype), _ptr(feat_out), _ptr(mask_out),
                                            _ptr(workspace), ws_bytes, _stream(stream)),
           "nsm_build_features_stored")


def nsm_create(c_in, widths, dtype="f32", arch="unet"):
    d = NetDesc()
    d.arch = ARCHS.get(arch, arch)
    d.c_in = c_in
    d.levels = len(widths)
    for i, v in enumerate(widths):
        d.widths[i] = v
    h = ctypes.c_void_p()
    _check(load().nsm_create(ctypes.byref(d), DTYPES.get(dtype, dtype), ctypes.byref(h)), "nsm_create")
    return h.value


def nsm_destroy(ctx):
    _check(load().nsm_destroy(ctx), "nsm_destroy")


def nsm_param_count(ctx):
    out = ctypes.c_size_t()
    _check(load().nsm_param_count(ctx, ctypes.byref(out)), "nsm_param_count")
    return out.value


def nsm_set_weights(ctx, w, n, stream=None):
    _check(load().nsm_set_weights(ctx, _ptr(w), n, _stream(stream)), "nsm_set_weights")


def nsm_workspace_bytes(ctx, n, h, w, training=0):
    out = ctypes.c_size_t()
    _check(load().nsm_workspace_bytes(ctx, n, h, w, int(training), ctypes.byref(out)),
           "nsm_workspace_bytes")
    return out.value


def nsm_forward(ctx, feat, n, h, w, vis_out, logits_out, workspace, ws_bytes, stream=None):
    _check(load().nsm_forward(ctx, _ptr(feat), n, h, w, _ptr(vis_out), _ptr(logits_out),
                              _ptr(workspace), ws_bytes, _stream(stream)), "nsm_forward")


def nsm_forward_stored(ctx, feat, n, h, w, vis_out, logits_out, workspace, ws_bytes, stream=None):
    _check(load().nsm_forward_stored(ctx, _ptr(feat), n, h, w, _ptr(vis_out), _ptr(logits_out),
                                     _ptr(workspace), ws_bytes, _stream(stream)), "nsm_forward_stored")


def nsm_backward(ctx, feat, dvis, n, h, w, dw_out, accumulate, dfeat_out, workspace, ws_bytes,
                 stream=None):
    _check(load().nsm_backward(ctx, _ptr(feat), _ptr(dvis), n, h, w, _ptr(dw_out), int(accumulate),
                               _ptr(dfeat_out), _ptr(workspace), ws_bytes, _stream(stream)),
           "nsm_backward")


def nsm_forward_train(ctx, feat, n, h, w, vis_out, workspace, ws_bytes, stream=None):
    _check(load().nsm_forward_train(ctx, _ptr(feat), n, h, w, _ptr(vis_out), _ptr(workspace), ws_bytes,
                                    _stream(stream)), "nsm_forward_train")


def nsm_backward_saved(ctx, feat, dvis, n, h, w, dw_out, accumulate, dfeat_out, workspace, ws_bytes,
                       stream=None):
    _check(load().nsm_backward_saved(ctx, _ptr(feat), _ptr(dvis), n, h, w, _ptr(dw_out), int(accumulate),
                                     _ptr(dfeat_out), _ptr(workspace), ws_bytes, _stream(stream)),
           "nsm_backward_saved")


def nsm_autotune(ctx, feat, n, h, w, vis_out, workspace, ws_bytes, reps=5, stream=None):
    """Times every launch variant of every stage and keeps the fastest;
    returns the chosen variants (stages in execution order)."""
    out = (ctypes.c_int * 16)()
    _check(load().nsm_autotune(ctx, _ptr(feat), n, h, w, _ptr(vis_out), _ptr(workspace), ws_bytes, int(reps),
                               out, _stream(stream)), "nsm_autotune")
    return nsm_get_stage_variants(ctx)


def nsm_autotune_stored(ctx, feat, n, h, w, vis_out, workspace, ws_bytes, reps=5, stream=None):
    """nsm_autotune on features in the context's storage type."""
    out = (ctypes.c_int * 16)()
    _check(load().nsm_autotune_stored(ctx, _ptr(feat), n, h, w, _ptr(vis_out), _ptr(workspace), ws_bytes,
                                      int(reps), out, _stream(stream)), "nsm_autotune_stored")
    return nsm_get_stage_variants(ctx)


def nsm_set_stage_variant(ctx, stage, variant):
    _check(load().nsm_set_stage_variant(ctx, int(stage), int(variant)), "nsm_set_stage_variant")


def nsm_get_stage_variants(ctx):
    out = (ctypes.c_int * 16)()
    n = ctypes.c_int()
    _check(load().nsm_get_stage_variants(ctx, out, 16, ctypes.byref(n)), "nsm_get_stage_variants")
    return [int(out[i]) for i in range(n.value)]


def nsm_trace_enable(on=True):
    _check(load().nsm_trace_enable(int(bool(on))), "nsm_trace_enable")


def nsm_trace_read(max_records=4096):
    """[(kernel name, milliseconds)] recorded since the last read."""
    names = ctypes.create_string_buffer(64 * max_records)
    ms = (ctypes.c_float * max_records)()
    n = ctypes.c_int()
    _check(load().nsm_trace_read(max_records, names, ms, ctypes.byref(n)), "nsm_trace_read")
    out = []
    raw = names.raw
    for i in range(min(n.value, max_records)):
        out.append((raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode(), float(ms[i])))
    return out


def nsm_perturbation_loss_workspace_bytes(n, p, h, w):
    out = ctypes.c_size_t()
    _check(load().nsm_perturbation_loss_workspace_bytes(n, p, h, w, ctypes.byref(out)),
           "nsm_perturbation_loss_workspace_bytes")
    return out.value


def nsm_perturbation_loss(vis, target, n, p, h, w, alpha, loss_out, dvis0_out, workspace, ws_bytes,
                          stream=None):
    _check(load().nsm_perturbation_loss(_ptr(vis), _ptr(target), n, p, h, w, float(alpha), _ptr(loss_out),
                                        _ptr(dvis0_out), _ptr(workspace), ws_bytes, _stream(stream)),
           "nsm_perturbation_loss")


def nsm_perturbation_loss_noalloc(vis, target, n, p, h, w, alpha, loss_out, dvis0_out, stream=None):
    _check(load().nsm_perturbation_loss_noalloc(_ptr(vis), _ptr(target), n, p, h, w, float(alpha),
                                                _ptr(loss_out), _ptr(dvis0_out), _stream(stream)),
           "nsm_perturbation_loss_noalloc")


def nsm_temporal_workspace_bytes(h, w):
    out = ctypes.c_size_t()
    _check(load().nsm_temporal_workspace_bytes(h, w, ctypes.byref(out)), "nsm_temporal_workspace_bytes")
    return out.value


def nsm_temporal_instability(tris, tri_normals, n_tris, fp_prev, fp_cur, gbuf_prev, gbuf_cur, vis_prev,
                             vis_cur, h, w, alpha, depth_tol, cos_tol, accumulate, acc_out, d_out,
                             workspace, ws_bytes, stream=None):
    a, b = frame_params(fp_prev), frame_params(fp_cur)
    _check(load().nsm_temporal_instability(_ptr(tris), _ptr(tri_normals), n_tris, ctypes.byref(a),
                                           ctypes.byref(b), _ptr(gbuf_prev), _ptr(gbuf_cur), _ptr(vis_prev),
                                           _ptr(vis_cur), h, w, float(alpha), float(depth_tol),
                                           float(cos_tol), int(accumulate), _ptr(acc_out), _ptr(d_out),
                                           _ptr(workspace), ws_bytes, _stream(stream)),
           "nsm_temporal_instability")
