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
