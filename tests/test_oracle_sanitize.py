"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/oracle_driver.c links oracle/nsm_oracle.c with
-fsanitize=address,undefined (no recovery: the first finding ends the run
with a non-zero status).  The driver reads each input from a raw file into a
buffer of exactly that size and allocates each output at exactly its size,
so a read or write past any array of the rasteriser, the gather (HARD6,
SOFT8, PAPER4), the ray caster (brute force and BVH, hard and soft) or the
temporal metric is caught.  Inputs are the synthetic scenes at small and
ragged sizes (odd screens and maps, an empty scene, triangles that leave the
guard band); every sanitized result must also equal the regular build's bit
for bit.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import nsm_synth as S
import oracle
from oracle import temporal as ot

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(os.path.dirname(HERE), "oracle", "nsm_oracle.c"),
       os.path.join(HERE, "sanitize", "oracle_driver.c")]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    d = tmp_path_factory.mktemp("sanitize")
    exe = str(d / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           *SRC, "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("the sanitizer runtimes are not available: " + r.stderr[-300:])
    return exe, d


def _run(driver, args):
    exe, _ = driver
    r = subprocess.run([exe, *[str(a) for a in args]], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0 and "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, \
        f"{args[0]} exited {r.returncode}:\n{r.stderr[-3000:]}"


def _put(d, name, a):
    p = str(d / name)
    np.ascontiguousarray(a).tofile(p)
    return p


def _raster(driver, tris, m, w, h, mode):
    _, d = driver
    tris = np.ascontiguousarray(tris, np.float32)
    _run(driver, ["raster", _put(d, "tris.bin", tris), tris.shape[0],
                  _put(d, "m.bin", np.asarray(m, np.float32).reshape(16)), w, h, mode,
                  str(d / "out.bin"), str(d / "stats.bin")])
    out = np.fromfile(str(d / "out.bin"), np.uint64 if mode == 1 else np.uint32).reshape(h, w)
    stats = tuple(int(s) for s in np.fromfile(str(d / "stats.bin"), np.int64))
    return out, stats


def _frames():
    out = []
    sc, fr = S.workload_frame("tiny_64", 3)
    out.append(("tiny_64", sc, fr))
    sc = S.make_scene("objects60", 1)
    fr = S.make_frame(sc, 37, 23, 61, (0.7, 3.1, -0.4), (2.9, 1.4, 1.7), light_radius=0.12)
    out.append(("ragged 37x23, map 61", sc, fr))
    # a scene reaching far past the screen: triangles dropped at the guard band
    big = np.concatenate([sc.tris, np.array([[[-900.0, 0.0, -900.0], [900.0, 0.0, -900.0], [0.0, 0.0, 900.0]]],
                                            np.float32)])
    out.append(("guard band", S.scenes._finish([big.astype(np.float64)]), fr))
    return out


@pytest.mark.parametrize("case", range(3))
def test_raster_and_gather_sanitized(driver, case):
    name, sc, fr = _frames()[case]
    _, d = driver
    for m, w, h, mode in ((fr.m_light, fr.sm_size, fr.sm_size, 0), (fr.m_cam, fr.width, fr.height, 1),
                          (fr.m_cam, fr.width, fr.height, 2)):
        got, gst = _raster(driver, sc.tris, m, w, h, mode)
        want, wst = oracle.raster(sc.tris, m, w, h, ("depth", "key", "count")[mode])
        assert gst == wst, name
        np.testing.assert_array_equal(got, want, err_msg=name)
    sm, _ = oracle.raster(sc.tris, fr.m_light, fr.sm_size, fr.sm_size, "depth")
    gb, _ = oracle.raster(sc.tris, fr.m_cam, fr.width, fr.height, "key")
    for fs, (code, C) in oracle.FEATURE_SETS.items():
        px = fr.width * fr.height
        _run(driver, ["gather", _put(d, "tris.bin", sc.tris), _put(d, "nrm.bin", sc.normals), sc.tris.shape[0],
                      _put(d, "fp.bin", oracle.frame_vector(fr)), _put(d, "gb.bin", gb), _put(d, "sm.bin", sm),
                      fr.width, fr.height, code, d / "feat.bin", d / "mask.bin", d / "pos.bin", d / "aux.bin"])
        want = oracle.gather(sc, fr, gb, sm, fs=fs)
        np.testing.assert_array_equal(np.fromfile(str(d / "feat.bin"), np.float32).reshape(px, C).view(np.uint32),
                                      want["feat"].reshape(px, C).view(np.uint32), err_msg=f"{name} {fs}")
        np.testing.assert_array_equal(np.fromfile(str(d / "mask.bin"), np.uint8), want["mask"].reshape(-1))


def test_empty_scene_sanitized(driver):
    _, fr = S.workload_frame("tiny_64", 0)
    none = np.zeros((0, 3, 3), np.float32)
    got, st = _raster(driver, none, fr.m_cam, fr.width, fr.height, 1)
    assert st == (0, 0, 0) and np.all(got == oracle.EMPTY_KEY)


def test_raycast_sanitized(driver):
    name, sc, fr = _frames()[1]
    _, d = driver
    feats = oracle.build_features(sc, fr, soft=True)
    pos = feats["pos"].reshape(-1, 3)
    valid = (feats["gbuf"] != oracle.EMPTY_KEY).astype(np.uint8).reshape(-1)
    lp = np.asarray(fr.light_pos, np.float32)
    for radius, samples, bvh in ((0.0, 1, 1), (0.0, 1, 0), (0.12, 16, 1), (0.12, 16, 0)):
        _run(driver, ["raycast", _put(d, "tris.bin", sc.tris), sc.tris.shape[0], _put(d, "pos.bin", pos),
                      _put(d, "valid.bin", valid), pos.shape[0], _put(d, "lp.bin", lp), radius, samples, 7, bvh,
                      1e-4, d / "vis.bin"])
        want = oracle.raycast(sc, pos, valid, lp, radius=radius, samples=samples, seed=7, use_bvh=bool(bvh))
        np.testing.assert_array_equal(np.fromfile(str(d / "vis.bin"), np.float32), want)


def test_temporal_sanitized(driver):
    _, d = driver
    sc, frs = S.make_train_window(0, 0, frames=2, width=48, height=40, sm_size=96)
    b0, b1 = (oracle.build_features(sc, fr, soft=True) for fr in frs)
    rng = S.SplitMix64(11)
    v0, v1 = (rng.uniforms(48 * 40, 0.0, 1.0).reshape(40, 48).astype(np.float32) for _ in range(2))
    _run(driver, ["temporal", _put(d, "tris.bin", sc.tris), _put(d, "nrm.bin", sc.normals), sc.tris.shape[0],
                  _put(d, "fa.bin", oracle.frame_vector(frs[0])), _put(d, "fb.bin", oracle.frame_vector(frs[1])),
                  _put(d, "ga.bin", b0["gbuf"]), _put(d, "gb.bin", b1["gbuf"]), _put(d, "va.bin", v0),
                  _put(d, "vb.bin", v1), 48, 40, 3.0, ot.DEPTH_TOL, ot.COS_TOL,
                  d / "sum.bin", d / "valid.bin", d / "dmap.bin"])
    total, valid, dmap = ot.temporal_pair(sc, frs[0], frs[1], b0["gbuf"], b1["gbuf"], v0, v1)
    assert np.fromfile(str(d / "sum.bin"), np.float64)[0] == total
    assert int(np.fromfile(str(d / "valid.bin"), np.int64)[0]) == valid
    np.testing.assert_array_equal(np.fromfile(str(d / "dmap.bin"), np.float32).reshape(40, 48), dmap)
