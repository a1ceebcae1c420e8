"""Pins for the oracle of the temporal-stability parts (Sec. 3.3, Eq. 2;
Sec. 3.4, Eq. 3).

Eq. 2 (per-pixel L1 term): against torch autograd with the perturbed outputs
detached, against its p = 0 special case (plain L1) and central differences.
Eq. 3: zero for a static sequence; the closed form for a constant change
of intensity; an exact two-pixel camera shift over a fronto-parallel plane
(every pixel must find its shifted partner); and, on a scene with an
occluder, agreement of the depth rejection with visibility from the
previous camera computed by the BVH ray cast."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import nsm_synth as S
import oracle
from oracle import temporal as ot


# ------------------------------------------------------------------ Eq. 2
def _batch(seed, n=2, p=3, h=9, w=7):
    r = S.SplitMix64(seed)
    vis = r.uniforms(n * (1 + p) * h * w, 0, 1).reshape(n, 1 + p, h, w)
    tgt = r.uniforms(n * h * w, 0, 1).reshape(n, h, w)
    return vis, tgt


def test_perturbation_loss_matches_autograd():
    vis, tgt = _batch(1)
    loss, g = ot.perturbation_loss(vis, tgt, alpha=0.9)
    v = torch.from_numpy(vis).requires_grad_(True)
    t = torch.from_numpy(tgt)
    x0 = v[:, 0]
    L = F.l1_loss(x0, t) + sum(F.l1_loss(x0, v[:, i].detach()) for i in range(1, 4))
    (0.9 * L).backward()
    assert loss == pytest.approx(0.9 * L.item(), rel=1e-12)
    np.testing.assert_allclose(g, v.grad[:, 0].numpy(), atol=1e-15)
    assert np.all(v.grad[:, 1:].numpy() == 0)          # nothing flows into x_1..x_p


def test_perturbation_loss_special_cases():
    vis, tgt = _batch(2, p=0)
    loss, g = ot.perturbation_loss(vis, tgt, alpha=1.0)
    assert loss == pytest.approx(np.abs(vis[:, 0] - tgt).mean(), rel=1e-12)
    np.testing.assert_array_equal(g, np.sign(vis[:, 0] - tgt) / tgt.size)
    # perturbed outputs equal to x_0: the extra terms and their gradients vanish
    vis3, _ = _batch(3)
    vis3[:, 1:] = vis3[:, :1]
    l3, g3 = ot.perturbation_loss(vis3, tgt, alpha=0.9)
    l0, g0 = ot.perturbation_loss(vis3[:, :1], tgt, alpha=0.9)
    assert l3 == l0
    np.testing.assert_array_equal(g3, g0)


def test_perturbation_loss_finite_differences():
    vis, tgt = _batch(4)
    _, g = ot.perturbation_loss(vis, tgt)
    rng = S.SplitMix64(5)
    for _ in range(20):
        n, y, x = int(rng.uniform(0, 2)), int(rng.uniform(0, 9)), int(rng.uniform(0, 7))
        h = 1e-7
        a, b = vis.copy(), vis.copy()
        a[n, 0, y, x] += h
        b[n, 0, y, x] -= h
        fd = (ot.perturbation_loss(a, tgt)[0] - ot.perturbation_loss(b, tgt)[0]) / (2 * h)
        # loss ~1.5, step 1e-7: float64 roundoff of the quotient is ~3e-9
        assert fd == pytest.approx(g[n, y, x], rel=1e-5, abs=1e-8)


# ------------------------------------------------------------------ Eq. 3
def _frames(scene, eyes, target, w=96, h=64, light=(1.0, 1.5, 5.0)):
    return [S.make_frame(scene, w, h, 256, light, e, target=t) for e, t in zip(eyes, target)]


def _gbuf(scene, fr):
    return oracle.raster(scene.tris, fr.m_cam, fr.width, fr.height, "key")[0]


def test_static_sequence_gives_zero():
    sc, frames = S.make_train_window(0, 1, width=96, height=64, sm_size=256)
    fr = frames[0]
    g = _gbuf(sc, fr)
    # intensities on a 1/1024 grid below 7/8, so that adding 1/8 is exact in float32
    vis = (np.floor(S.SplitMix64(6).uniforms(64 * 96, 0, 896)) / 1024).reshape(64, 96).astype(np.float32)
    total, valid, dmap = ot.temporal_pair(sc, fr, fr, g, g, vis, vis)
    fg = g != oracle.EMPTY_KEY
    assert total == 0.0
    assert valid == int(fg.sum()) and valid > 1000
    assert np.all(dmap[fg] == 0.0) and np.all(dmap[~fg] == -1.0)
    # a constant change of intensity delta: every passed pixel adds exp(3 delta) - 1
    d = np.float32(0.125)
    t2, v2, _ = ot.temporal_pair(sc, fr, fr, g, g, vis + d, vis)
    assert v2 == valid
    assert t2 == pytest.approx(valid * (math.exp(3.0 * float(d)) - 1.0), rel=1e-12)
    assert ot.instability([t2], 96, 64) == pytest.approx(t2 / (96 * 64))


def _plane(z=0.0, half=10.0):
    v = np.array([[-half, -half, z], [half, -half, z], [half, half, z], [-half, half, z]], np.float64)
    tris = np.array([[v[0], v[1], v[2]], [v[0], v[2], v[3]]])
    return tris


def _scene(tri_list):
    tris = np.concatenate(tri_list).astype(np.float64)
    e1, e2 = tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]
    n = np.cross(e1, e2)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return S.Scene(tris=tris.astype(np.float32), normals=n.astype(np.float32))


def test_exact_pixel_shift_over_a_plane():
    """Camera translated along its right axis by exactly two pixels' width at
    the plane's depth: pixel (i, j) of the new frame is (i + 2, j) of the old."""
    sc = _scene([_plane()])
    w, h = 96, 64
    fr0 = S.make_frame(sc, w, h, 256, (1.0, 1.5, 5.0), (0.0, 0.0, 4.0), target=(0.0, 0.0, 0.0))
    px = 2.0 * 4.0 * float(fr0.cam_tan_half_x) / w             # world width of one pixel at depth 4
    right = fr0.cam_right.astype(np.float64)
    dlt = 2.0 * px * right
    fr1 = S.make_frame(sc, w, h, 256, (1.0, 1.5, 5.0), dlt + [0.0, 0.0, 4.0], target=dlt)
    g0, g1 = _gbuf(sc, fr0), _gbuf(sc, fr1)
    ii, jj = np.meshgrid(np.arange(w), np.arange(h))
    ramp = (1e-3 * ii + 1e-5 * jj).astype(np.float32)
    cur = np.zeros_like(ramp)
    cur[:, : w - 2] = ramp[:, 2:]
    total, valid, dmap = ot.temporal_pair(sc, fr0, fr1, g0, g1, ramp, cur)
    assert valid == (w - 2) * h
    assert np.all(dmap[:, : w - 2] == 0.0)
    assert np.all(dmap[:, w - 2:] == -2.0)
    assert total == 0.0


def test_depth_rejection_matches_visibility_from_previous_camera():
    """A box on a ground plane; the camera moves sideways.  Passed pixels must
    be visible from the previous eye, and pixels the previous camera could
    not see must be rejected.  Both up to silhouettes, where the nearest-pixel
    lookup can land on the other surface (0.04% and 2.3% of the pixels here)."""
    box = S.scenes.box_tris((0.0, 0.0, 0.5), (0.5, 0.5, 0.5))
    sc = _scene([_plane(0.0, 4.0), box.astype(np.float64)])
    w, h = 128, 96
    eyes = [np.array([0.0, -0.6, 4.0]), np.array([0.6, -0.6, 4.0])]
    fr0, fr1 = (S.make_frame(sc, w, h, 256, (1.0, 1.5, 6.0), e, target=(0.0, 0.0, 0.0)) for e in eyes)
    b0, b1 = oracle.build_features(sc, fr0), oracle.build_features(sc, fr1)
    vis = np.zeros((h, w), np.float32)
    _, valid, dmap = ot.temporal_pair(sc, fr0, fr1, b0["gbuf"], b1["gbuf"], vis, vis)
    fg = b1["gbuf"] != oracle.EMPTY_KEY
    seen = oracle.raycast(sc, b1["pos"], fg, fr0.cam_pos) > 0.5     # unoccluded towards the old eye
    passed = dmap >= 0
    rej_depth = dmap == -4.0
    assert passed.sum() == valid and rej_depth.sum() > 50
    assert np.mean(seen[passed]) >= 0.995
    assert np.mean(~passed[fg & ~seen]) >= 0.95
    assert np.mean(~seen[rej_depth]) >= 0.75     # the rest sit next to the box's silhouette
    # the thresholds order the tests: no normal can pass cos >= 1.01
    _, v_none, d_none = ot.temporal_pair(sc, fr0, fr1, b0["gbuf"], b1["gbuf"], vis, vis, cos_tol=1.01)
    assert v_none == 0 and np.all(d_none[passed] == -5.0)
