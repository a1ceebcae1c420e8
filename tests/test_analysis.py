"""Pins for the design-time tools: penumbra model special cases (closed forms),
the receptive-field rule against the values Table 1 prints, and the
sensitivity of a channel the network cannot see."""
import json
import math
import os

import numpy as np
import pytest

from paper_2301_05262_amd import analysis as A

GOLD = os.path.join(os.path.dirname(__file__), "golden", "receptive_field_table1.json")


def test_point_light_has_no_penumbra():
    zf = np.linspace(1.5, 4.0, 11)
    w = A.penumbra_width(0.8, 1.2, zf, 0.0)
    np.testing.assert_allclose(w, 0.0, atol=1e-14)


def test_point_occluder_reduces_to_pcss():
    # r_s = 0 (z_min = z_max): both extents equal the PCSS estimate r_e (z_f - z_b) / z_b
    z_b, r_e = 1.3, 0.25
    zf = np.linspace(1.5, 5.0, 8)
    x_a, x_b = A.penumbra_extents(z_b, z_b, zf, r_e)
    pcss = r_e * (zf - z_b) / z_b
    np.testing.assert_allclose(x_a, pcss, rtol=1e-12)
    np.testing.assert_allclose(x_b, pcss, rtol=1e-12)


def test_width_grows_with_emitter_and_receiver_distance():
    w1 = A.penumbra_width(1.0, 1.4, 3.0, 0.1)
    w2 = A.penumbra_width(1.0, 1.4, 3.0, 0.2)
    w3 = A.penumbra_width(1.0, 1.4, 4.0, 0.2)
    assert 0 < w1 < w2 < w3


def test_receptive_field_matches_table1():
    g = json.load(open(GOLD))
    for layers, rf in g["layers_to_receptive_field"].items():
        assert A.receptive_field(int(layers)) == rf
    avail = [int(k) for k in g["layers_to_receptive_field"]]
    for w in g["p95_width_px"]:
        need = A.levels_for_width(w, avail)
        for l in avail:
            fails = [w, l] in g["failing_pairs_width_layers"]
            # a net fails exactly when it has fewer levels than the rule asks for
            assert fails == (l < need), (w, l, need)
    assert A.levels_for_width(24) == 3 and A.levels_for_width(25) == 4
    assert A.levels_for_width(3 * 2 ** 5) == 5


def test_pixel_conversion():
    # at depth d with vertical fov 2*atan(t), one pixel spans 2 d t / H
    assert A.width_in_pixels(2 * 3.0 * 0.5 / 1080, 3.0, 0.5, 1080) == pytest.approx(1.0)
    assert A.p95_width(np.arange(1, 101)) == pytest.approx(np.quantile(np.arange(1, 101), 0.95))


def _plate_case(radius):
    """Ground y = -1 over [-1.5, 1.5]^2 and a square plate y = 0 over
    [-0.3, 0.3]^2, light straight above at (0, 3, 0): the plate is a flat
    blocker at light depth 3 over receivers at light depth 4."""
    import oracle
    import torch

    import nsm_synth as S
    from nsm_synth import scenes as SC
    sc = SC._finish([SC.ground_quad(), SC.ground_quad(y=0.0, half=0.3)])
    fr = S.make_frame(sc, 320, 240, 512, (0.0, 3.0, 0.0), (0.0, 1.2, 2.8), target=(0.0, -1.0, 0.6),
                      light_radius=radius)
    o = oracle.build_features(sc, fr)
    g = torch.from_numpy(o["gbuf"].view(np.int64))
    sm = torch.from_numpy(o["sm"].view(np.int32))
    tris, nrm = torch.from_numpy(sc.tris), torch.from_numpy(sc.normals)
    w, zmin, zmax, _ = A.penumbra_widths(g, sm, tris, nrm, fr)
    P, _, fg = A._receivers(g, tris, nrm, fr)
    return fr, w.numpy(), zmin.numpy(), zmax.numpy(), P.numpy(), fg.numpy()


def test_penumbra_widths_of_a_flat_blocker():
    """A flat blocker at light depth z_b = 3 over receivers at z_f = 4 with
    r_e = 0.1: z_min = z_max = 3, so the model's width is the PCSS estimate
    2 r_e (z_f - z_b) / z_b = 1/15 world units at every receiver whose cone
    to the emitter meets the plate (inside |x|, |z| <= (0.3 + 0.025) * 4/3,
    the plate's shadow widened by the cone's radius 0.025 at the plate), and
    0 well outside it; a point light gives 0 everywhere."""
    fr, w, zmin, zmax, P, fg = _plate_case(0.1)
    ground = fg & (np.abs(P[..., 1] + 1.0) < 1e-4)
    linf = np.maximum(np.abs(P[..., 0]), np.abs(P[..., 2]))
    inner, outer = ground & (linf <= 0.40), ground & (linf >= 0.46)
    assert inner.sum() > 1000 and outer.sum() > 10000
    assert np.abs(zmin[inner] - 3.0).max() < 1e-6 and np.abs(zmax[inner] - 3.0).max() < 1e-6
    view = ((P - fr.cam_pos.astype(np.float64)) * fr.cam_fwd.astype(np.float64)).sum(-1)
    world = w * (2.0 * view * fr.cam_tan_half_y / fr.height)
    np.testing.assert_allclose(world[inner], 2 * 0.1 * (4.0 - 3.0) / 3.0, rtol=1e-6)
    assert (w[outer] == 0).all()
    _, w0, *_ = _plate_case(0.0)
    assert (w0 == 0).all()
    rep = A.level_report([w])
    assert rep["penumbra_pixels"] == int((w > 0).sum()) and rep["levels"] == A.levels_for_width(rep["p95_width_px"],
                                                                                                 (2, 3, 4, 5))
