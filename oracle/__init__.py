"""CPU oracle for the neural shadow-mapping hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the GPU library:

* ``nsm_oracle.c`` (plain C, float32/float64 with no contraction): the
  z-buffer rasteriser, the feature gather with its depth-test mask, and the
  ray-cast visibility reference;
* ``net.py`` (numpy float64): the network forward, its exact adjoint and a
  storage-rounding emulation of the low-precision forward;
* ``paper_net.py``: the paper's own network and its space-to-depth form;
* ``temporal.py``: the perturbation loss of Eq. 2 and the temporal
  instability metric of Eq. 3 (its per-pixel part in ``nsm_oracle.c``).

Parity status of every function is recorded in its test module; all of the
functions here are pinned by the ``-m "not gpu"`` tests.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import net  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "nsm_oracle.c")
_lib = None

EMPTY_DEPTH = 0x7F800000
EMPTY_KEY = 0xFFFFFFFFFFFFFFFF


def build_lib(force=False):
    """Compile the C part with gcc (no floating-point contraction)."""
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", SRC_PATH, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build_lib()
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
        L.ora_raster.argtypes = [vp, i32, vp, i32, i32, i32, vp, vp]
        L.ora_raster.restype = i32
        L.ora_gather.argtypes = [vp, vp, i32, vp, vp, vp, i32, i32, i32, vp, vp, vp, vp]
        L.ora_gather.restype = i32
        L.ora_raycast.argtypes = [vp, i32, vp, vp, i32, vp, f32, i32, ctypes.c_uint64, i32,
                                  ctypes.c_double, vp]
        L.ora_raycast.restype = i32
        L.ora_temporal.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, i32, i32, f32, f32, f32, vp, vp, vp]
        L.ora_temporal.restype = i32
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def frame_vector(fr):
    """Pack frame parameters into the oracle's 56-float layout."""
    v = np.zeros(56, np.float32)
    v[0:16] = np.asarray(fr.m_light, np.float32).reshape(-1)
    v[16:19] = fr.light_pos
    v[19] = fr.light_radius
    v[20] = fr.light_near
    v[21] = fr.light_far
    v[22] = fr.light_tan_half_fov
    v[23] = fr.sm_size
    v[24:40] = np.asarray(fr.m_cam, np.float32).reshape(-1)
    v[40:43] = fr.cam_pos
    v[43:46] = fr.cam_fwd
    v[46:49] = fr.cam_right
    v[49:52] = fr.cam_up
    v[52] = fr.cam_tan_half_x
    v[53] = fr.cam_tan_half_y
    v[54] = fr.cam_near
    v[55] = fr.cam_far
    return v


def raster(tris, matrix, width, height, mode="depth"):
    """Rasterise a float32 [T,3,3] triangle soup.

    mode 'depth' -> uint32 [H,W] depth bits (min), empty = +inf bits;
    'key' -> uint64 [H,W] (depth bits << 32 | triangle id), empty = all ones;
    'count' -> uint32 [H,W] covering-fragment counts.
    Returns (image, stats) with stats = (dropped, zero-area, fragments)."""
    tris = np.ascontiguousarray(tris, np.float32)
    m = np.ascontiguousarray(matrix, np.float32).reshape(16)
    md = {"depth": 0, "key": 1, "count": 2}[mode]
    out = np.empty((height, width), np.uint64 if md == 1 else np.uint32)
    stats = np.zeros(3, np.int64)
    rc = lib().ora_raster(_p(tris), int(tris.shape[0]), _p(m), int(width), int(height), md,
                          _p(out), _p(stats))
    if rc:
        raise RuntimeError(f"ora_raster failed ({rc})")
    return out, tuple(int(s) for s in stats)


FEATURE_SETS = {"hard6": (0, 6), "soft8": (1, 8), "paper4": (2, 4)}


def gather(scene, fr, gbuf, sm, soft=False, fs=None):
    """Feature gather. Returns dict(feat [H,W,C] f32, mask [H,W] u8,
    pos [H,W,3] f32, aux [H,W,4] f32 = (z, z_f, beta, inside)).
    fs: 'hard6', 'soft8' or 'paper4' (default from `soft`)."""
    h, w = fr.height, fr.width
    code, C = FEATURE_SETS[fs or ("soft8" if soft else "hard6")]
    feat = np.empty((h, w, C), np.float32)
    mask = np.empty((h, w), np.uint8)
    pos = np.empty((h, w, 3), np.float32)
    aux = np.empty((h, w, 4), np.float32)
    fv = frame_vector(fr)
    tris = np.ascontiguousarray(scene.tris, np.float32)
    nrm = np.ascontiguousarray(scene.normals, np.float32)
    gbuf = np.ascontiguousarray(gbuf, np.uint64)
    sm = np.ascontiguousarray(sm, np.uint32)
    rc = lib().ora_gather(_p(tris), _p(nrm), int(tris.shape[0]), _p(fv), _p(gbuf), _p(sm),
                          w, h, code, _p(feat), _p(mask), _p(pos), _p(aux))
    if rc:
        raise RuntimeError(f"ora_gather failed ({rc})")
    return {"feat": feat, "mask": mask, "pos": pos, "aux": aux}


def build_features(scene, fr, soft=False, fs=None):
    """Shadow map, camera G-buffer and features for one frame (the oracle pipeline)."""
    sm, sm_stats = raster(scene.tris, fr.m_light, fr.sm_size, fr.sm_size, "depth")
    gb, gb_stats = raster(scene.tris, fr.m_cam, fr.width, fr.height, "key")
    out = gather(scene, fr, gb, sm, soft=soft, fs=fs)
    out.update(sm=sm, gbuf=gb, sm_stats=sm_stats, gbuf_stats=gb_stats)
    return out


def raycast(scene, pos, valid, light_pos, radius=0.0, samples=1, seed=0, use_bvh=True, eps=1e-4):
    """Visibility of the emitter from receivers ``pos`` [..., 3] (1 = lit)."""
    pos = np.ascontiguousarray(pos, np.float32)
    shape = pos.shape[:-1]
    npix = int(np.prod(shape))
    valid = None if valid is None else np.ascontiguousarray(valid, np.uint8).reshape(-1)
    vis = np.empty(npix, np.float32)
    tris = np.ascontiguousarray(scene.tris, np.float32)
    lp = np.ascontiguousarray(light_pos, np.float32)
    rc = lib().ora_raycast(_p(tris), int(tris.shape[0]), _p(pos), _p(valid), npix, _p(lp),
                           float(radius), int(samples), int(seed) & 0xFFFFFFFFFFFFFFFF,
                           int(bool(use_bvh)), float(eps), _p(vis))
    if rc:
        raise RuntimeError(f"ora_raycast failed ({rc})")
    return vis.reshape(shape)
