"""Pins for the oracle feature gather and ray-cast reference.

Features are the screen-space buffers of paper Sec. 3.1 (view depth d,
normal n, emitter-to-occluder depth z, pixel-to-emitter depth z_f, emitter
size r_e) and their compositions (Sec. 3.2: z - z_f, z / z_f, ...).  The
depth-test mask is the vanilla shadow-map test.  The ray cast is the
emitter-to-receiver visibility the paper trains against (Sec. 3.1, supp.
Sec. 5), with one ray for a point light and stratified emitter samples for a
spherical light.

Pins: geometric invariants of the gathered channels on an analytic ground
plane, no self-shadowing of a lit plane, agreement of the mask with an
independent ray cast away from shadow edges, BVH == brute force, exact
special cases of the soft ray cast (fully lit, umbra, a half-plane occluder
through the emitter centre covers exactly half of the stratified samples).
"""
import math

import numpy as np
import pytest

import oracle
from nsm_synth import scenes
from nsm_synth.scenes import make_frame, Scene, box_tris, ground_quad


def _scene(parts):
    return scenes._finish(parts)


def _clip(m, P):
    m = np.asarray(m, np.float64)
    Ph = np.concatenate([P.astype(np.float64), np.ones(P.shape[:-1] + (1,))], axis=-1)
    return Ph @ m.T


@pytest.fixture(scope="module")
def ground_only():
    sc = _scene([ground_quad(half=1.5)])
    fr = make_frame(sc, 96, 64, 512, light_pos=(0.2, 3.0, 0.1),
                    eye=(2.8, 1.4, 1.1), target=(0.0, -1.0, 0.0))
    return sc, fr, oracle.build_features(sc, fr)


def test_ground_plane_channels(ground_only):
    sc, fr, o = ground_only
    fg = o["gbuf"] != oracle.EMPTY_KEY
    assert fg.mean() > 0.3
    f, P = o["feat"], o["pos"]
    # normal of the ground facing the camera is +y exactly
    np.testing.assert_array_equal(f[fg][:, 1:4], np.tile([0, 1, 0], (fg.sum(), 1)))
    # receivers lie on the plane
    assert np.abs(P[fg][:, 1] + 1.0).max() < 2e-6
    # P reprojects to its own pixel centre
    c = _clip(fr.m_cam, P[fg])
    sx = (c[:, 0] / c[:, 3] * 0.5 + 0.5) * fr.width
    sy = (c[:, 1] / c[:, 3] * 0.5 + 0.5) * fr.height
    jj, ii = np.nonzero(fg)
    assert np.abs(sx - (ii + 0.5)).max() < 1e-3 and np.abs(sy - (jj + 0.5)).max() < 1e-3
    # view depth channel = camera-axis depth / far
    np.testing.assert_allclose(f[fg][:, 0] * fr.cam_far, c[:, 3], rtol=2e-6)
    # pixel-to-emitter depth z_f = light-axis depth (w of the light clip)
    cl = _clip(fr.m_light, P[fg])
    np.testing.assert_allclose(o["aux"][fg][:, 1], cl[:, 3], rtol=1e-5)
    # background pixels are all zero
    assert (f[~fg] == 0).all() and (o["mask"][~fg] == 0).all()


def test_lit_plane_has_no_self_shadow(ground_only):
    sc, fr, o = ground_only
    fg = o["gbuf"] != oracle.EMPTY_KEY
    assert (o["mask"][fg] == 0).all()
    z, zf, beta = o["aux"][..., 0], o["aux"][..., 1], o["aux"][..., 2]
    inside = fg & (o["aux"][..., 3] == 1)
    # texels off the plane's edge are empty: those receivers read z = f_L (lit)
    assert inside.mean() > 0.9 * fg.mean()
    np.testing.assert_array_equal(z[fg & ~inside], np.float32(fr.light_far))
    # where the map resolves the plane itself, |z - z_f| stays within the bias
    assert (np.abs(z - zf)[inside] <= beta[inside]).all()
    # depth-test channels agree: (z - z_f)/f_L and z/f_L
    np.testing.assert_allclose(o["feat"][fg][:, 5] * fr.light_far, z[fg], rtol=1e-6)


def _eligible(rc, fg, cosl, r=2):
    """Pixels whose ray-cast value is constant within r pixels, foreground
    within r pixels, and facing the light (cos >= 0.2)."""
    h, w = rc.shape
    ok = fg & (cosl >= 0.2)
    out = np.zeros_like(ok)
    for j in range(r, h - r):
        for i in range(r, w - r):
            if not ok[j, i]:
                continue
            win = rc[j - r:j + r + 1, i - r:i + r + 1]
            fw = fg[j - r:j + r + 1, i - r:i + r + 1]
            out[j, i] = fw.all() and (win == win[r, r]).all()
    return out


def _cos_light(o, fr):
    P = o["pos"].astype(np.float64)
    n = o["feat"][..., 1:4].astype(np.float64)
    l = np.asarray(fr.light_pos, np.float64) - P
    l /= np.linalg.norm(l, axis=-1, keepdims=True) + 1e-30
    return (n * l).sum(-1)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mask_equals_hard_raycast_away_from_edges(seed):
    rng = np.random.default_rng(seed)
    boxes = [box_tris(c, h) for c, h in
             [((rng.uniform(-0.6, 0.6), -0.6, rng.uniform(-0.6, 0.6)), (0.25, 0.4, 0.2)),
              ((rng.uniform(-0.6, 0.6), -0.3, rng.uniform(-0.6, 0.6)), (0.15, 0.15, 0.3))]]
    sc = _scene([ground_quad(half=1.5)] + boxes)
    light = (rng.uniform(-2.0, -1.2), 2.2, rng.uniform(-1.0, 1.0))      # oblique: long shadows
    fr = make_frame(sc, 160, 120, 1024, light_pos=light, eye=(3.0, 1.8, 0.8), target=(0.0, -0.8, 0.0))
    o = oracle.build_features(sc, fr)
    fg = o["gbuf"] != oracle.EMPTY_KEY
    vis = oracle.raycast(sc, o["pos"], fg, fr.light_pos, use_bvh=True)
    shadow_rc = (vis < 0.5)
    elig = _eligible(shadow_rc, fg, _cos_light(o, fr))
    assert elig.sum() > 3000
    assert shadow_rc[elig].sum() > 200                     # some umbra is tested
    mism = (o["mask"].astype(bool) != shadow_rc) & elig
    assert mism.sum() == 0, f"{mism.sum()} mismatches of {elig.sum()}"


def test_bvh_equals_brute_force():
    sc, fr = scenes.workload_frame("tiny_64", 3)
    o = oracle.build_features(sc, fr)
    fg = o["gbuf"] != oracle.EMPTY_KEY
    a = oracle.raycast(sc, o["pos"], fg, fr.light_pos, use_bvh=True)
    b = oracle.raycast(sc, o["pos"], fg, fr.light_pos, use_bvh=False)
    np.testing.assert_array_equal(a, b)
    a = oracle.raycast(sc, o["pos"], fg, fr.light_pos, radius=0.15, samples=16, seed=5, use_bvh=True)
    b = oracle.raycast(sc, o["pos"], fg, fr.light_pos, radius=0.15, samples=16, seed=5, use_bvh=False)
    np.testing.assert_array_equal(a, b)


def test_soft_raycast_special_cases():
    big = box_tris((0.0, 1.0, 0.0), (0.8, 0.05, 0.8))           # slab between light and ground
    half_plane = np.array([[[-10.0, 1.0, 0.0], [10.0, 1.0, 0.0], [0.0, 1.0, -10.0]]])
    P = np.array([[0.0, 0.0, 0.0]], np.float32)
    L = np.array([0.0, 2.0, 0.0], np.float32)
    lit = oracle.raycast(_scene([ground_quad(y=-0.5)]), P, None, L, radius=0.2, samples=64)
    assert lit[0] == 1.0
    umbra = oracle.raycast(_scene([big]), P, None, L, radius=0.1, samples=64)
    assert umbra[0] == 0.0
    # an occluding half-plane whose edge passes under the emitter centre along
    # a disk axis blocks exactly the half of the 8x8 strata on one side
    for seed in range(5):
        v = oracle.raycast(_scene([half_plane]), P, None, L, radius=0.2, samples=64, seed=seed)
        assert v[0] == 0.5
    # a vanishing emitter reproduces the point-light answer
    sc, fr = scenes.workload_frame("tiny_64", 1)
    o = oracle.build_features(sc, fr)
    fg = o["gbuf"] != oracle.EMPTY_KEY
    hard = oracle.raycast(sc, o["pos"], fg, fr.light_pos)
    tiny = oracle.raycast(sc, o["pos"], fg, fr.light_pos, radius=1e-7, samples=64, seed=3)
    elig = _eligible(hard < 0.5, fg, np.ones_like(hard))
    np.testing.assert_array_equal(tiny[elig], hard[elig])


def test_soft_channels():
    sc = _scene([ground_quad(half=1.5), box_tris((0.0, 0.0, 0.0), (0.3, 0.02, 0.3))])
    fr = make_frame(sc, 64, 64, 512, light_pos=(0.0, 3.0, 0.0), eye=(2.5, 1.5, 0.5),
                    target=(0.0, -1.0, 0.0), light_radius=0.1)
    o = oracle.build_features(sc, fr, soft=True)
    f = o["feat"]
    fg = o["gbuf"] != oracle.EMPTY_KEY
    np.testing.assert_array_equal(f[fg][:, 6], np.float32(np.float32(0.1) / np.float32(0.2)))
    # deep in the umbra on the ground the blocker average is the slab's depth
    sh = (o["mask"] == 1) & (np.abs(o["pos"][..., 1] + 1.0) < 1e-5)
    assert sh.sum() > 20
    slab = o["aux"][sh][:, 0]                       # z of the occluder seen by the map
    # z_blk lies between the slab's min and max light depth, never at the receiver
    zb = f[sh][:, 7] * fr.light_far
    assert (zb <= o["aux"][sh][:, 1]).all()
    assert np.abs(zb - slab).max() < 0.05
    # unshadowed, unblocked receivers report z_blk = z_f
    lit = (o["mask"] == 0) & fg & (np.abs(o["pos"][..., 1] + 1.0) < 1e-5)
    far_lit = lit & (np.hypot(o["pos"][..., 0], o["pos"][..., 2]) > 0.9)
    np.testing.assert_allclose(f[far_lit][:, 7] * fr.light_far, o["aux"][far_lit][:, 1], rtol=1e-6)


def test_paper4_channels_on_ground_plane():
    """The paper's feature set (Sec. 3.2): c_e + size code, z/z_f, z - z_f, c_c/d,
    checked against the cosines computed directly from the receiver positions."""
    sc = _scene([ground_quad(half=1.5)])
    fr = make_frame(sc, 96, 64, 512, light_pos=(0.2, 3.0, 0.1), eye=(2.8, 1.4, 1.1),
                    target=(0.0, -1.0, 0.0), light_radius=0.125)
    o = oracle.build_features(sc, fr, fs="paper4")
    hard = oracle.build_features(sc, fr)
    fg = o["gbuf"] != oracle.EMPTY_KEY
    inside = fg & (o["aux"][..., 3] == 1)
    f, P = o["feat"].astype(np.float64), o["pos"].astype(np.float64)
    L, E = np.asarray(fr.light_pos, np.float64), np.asarray(fr.cam_pos, np.float64)
    l = L - P
    c_e = l[..., 1] / np.linalg.norm(l, axis=-1)                 # n = +y on the ground
    v = E - P
    c_c = v[..., 1] / np.linalg.norm(v, axis=-1)
    d = hard["feat"][..., 0].astype(np.float64) * fr.cam_far       # view depth
    np.testing.assert_allclose(f[fg][:, 0], c_e[fg] + 2.0, rtol=0, atol=2e-6)
    np.testing.assert_allclose(f[fg][:, 3], (c_c / d)[fg], rtol=2e-6)
    z, zf = o["aux"][..., 0].astype(np.float64), o["aux"][..., 1].astype(np.float64)
    np.testing.assert_allclose(f[inside][:, 1], (z / zf)[inside], rtol=1e-6)
    # same depth-test channel as the 6-channel set
    np.testing.assert_array_equal(o["feat"][..., 2], hard["feat"][..., 4])
    assert (o["mask"] == hard["mask"]).all()
