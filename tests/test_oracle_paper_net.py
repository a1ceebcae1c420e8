"""Pins for the oracle of the paper's own network (Sec. 3.5).

The channel plan is pinned by the numbers the paper prints in its
layer-wise table (supplemental Sec. 3) and cost table (supplemental
Sec. 4.1); the forward is pinned against a torch float64 model of the same
plan (library convolutions, avg-pool and bilinear interpolation)."""
import json
import os

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from nsm_synth import SplitMix64
from oracle import paper_net as pn

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables_s2_s4.json")))


def test_layer_table_matches_table_s2():
    rows = pn.layer_table(G["c_in"], G["widths_5"], G["height"], G["width"])
    t = G["table_s2"]
    for l, (macs, params, io) in enumerate(rows):
        assert round(macs / 1e9, 2) == pytest.approx(t["gflops"][l], abs=0.006)
        want_p = t["params_k"][l]
        assert abs(params / 1e3 - want_p) <= 0.05 + 1e-9, (l, params, want_p)
        assert abs(io / 1e6 - t["temp_io_mpx"][l]) <= 0.1, (l, io, t["temp_io_mpx"][l])


def test_costs_match_table_s4():
    for name, widths in (("3-layer", G["widths_5"][:2] + [64]), ("5-layer", G["widths_5"])):
        want = G["table_s4"][name]
        assert pn.macs_per_pixel(4, widths) == want["flops_per_pixel"]
        weights = sum(co * k * k * ci for _, co, k, ci, _ in pn.conv_list(4, widths))
        assert abs(weights / 1e3 - want["params_k"]) <= 0.06          # printed to 0.05-0.1K


class TorchPNet(torch.nn.Module):
    def __init__(self, c_in, widths, flat):
        super().__init__()
        self.widths = widths
        self.m = torch.nn.ModuleDict()
        for name, (w, b) in pn.split(c_in, widths, flat).items():
            k = w.shape[1]
            c = torch.nn.Conv2d(w.shape[3], w.shape[0], k, padding=k // 2).double()
            c.weight.data = torch.from_numpy(w.transpose(0, 3, 1, 2).copy())
            c.bias.data = torch.from_numpy(b.copy())
            self.m[name.replace(".", "_")] = c

    def forward(self, x):
        L = len(self.widths)
        c = lambda n, t: self.m[n.replace(".", "_")](t)
        skips = []
        for l in range(L - 1):
            x = F.relu(c(f"E{l}.1", F.relu(c(f"E{l}.3", x))))
            skips.append(x)
            x = F.avg_pool2d(x, 2)
        x = F.relu(c("B.1", F.relu(c("B.3", x))))
        for l in range(L - 2, -1, -1):
            x = F.interpolate(x, scale_factor=2, mode="bilinear", align_corners=False)
            if l >= 1:
                x = x + skips[l]
            x = F.relu(c(f"D{l}.1", F.relu(c(f"D{l}.3", x))))
        return c("OUT", x)[:, 0]


@pytest.mark.parametrize("widths", [(16, 32, 64), (16, 32, 64, 128, 256)])
def test_forward_matches_torch(widths):
    n = pn.n_params(4, widths)
    flat = (SplitMix64(3).normals(n) * 0.2).astype(np.float32)
    feat = SplitMix64(4).uniforms(2 * 32 * 48 * 4, -1, 1).reshape(2, 32, 48, 4).astype(np.float32)
    got = pn.forward(4, widths, flat, feat)
    ref = TorchPNet(4, widths, flat)(torch.from_numpy(feat.astype(np.float64).transpose(0, 3, 1, 2).copy()))
    np.testing.assert_allclose(got["logits"], ref.detach().numpy(), atol=1e-11)


# ------------------------------------------------------- space-to-depth form
def test_space_to_depth_brute_force():
    x = SplitMix64(5).uniforms(2 * 4 * 6 * 3, -1, 1).reshape(2, 4, 6, 3)
    y = pn.space_to_depth(x)
    assert y.shape == (2, 2, 3, 12)
    for n in range(2):
        for i in range(2):
            for j in range(3):
                for dy in range(2):
                    for dx in range(2):
                        for c in range(3):
                            assert y[n, i, j, (2 * dy + dx) * 3 + c] == x[n, 2 * i + dy, 2 * j + dx, c]
    np.testing.assert_array_equal(pn.depth_to_space(y), x)
    # torch's pixel_unshuffle orders channels c * 4 + (2 dy + dx); permuted, it is the same map
    t = F.pixel_unshuffle(torch.from_numpy(x.transpose(0, 3, 1, 2).copy()), 2).numpy()
    perm = [c * 4 + k for k in range(4) for c in range(3)]
    np.testing.assert_array_equal(t[:, perm].transpose(0, 2, 3, 1), y)


def test_s2d_layer_table_against_table_s2():
    """Dropping level 0 keeps the printed rows of levels 1..4; the only new
    convolution is the w_0 -> 4 output conv at level 1."""
    h, w, wd = G["height"], G["width"], G["widths_5"]
    plain = pn.layer_table(4, wd, h, w)
    rows = pn.layer_table(4, wd, h, w, s2d=True)
    assert len(rows) == 4
    px1 = (h // 2) * (w // 2)
    assert rows[0][0] == plain[1][0] + px1 * 4 * wd[0]
    assert rows[0][1] == plain[1][1] + 4 * wd[0]
    assert rows[1:] == plain[2:]
    t = G["table_s2"]["gflops"]
    assert abs(sum(r[0] for r in rows) / 1e9 - (sum(t[1:]) + px1 * 64 / 1e9)) <= 0.02
    # the first layer's cost is what the form removes: 16208 - 3408 + 64 / 4 MAC per pixel
    assert pn.macs_per_pixel(4, wd, s2d=True) == G["table_s4"]["5-layer"]["flops_per_pixel"] - 3408 + 16
    assert sum(r[0] for r in plain[:1]) == 3408 * h * w


class TorchPNetS2D(TorchPNet):
    def __init__(self, c_in, widths, flat):
        torch.nn.Module.__init__(self)
        self.widths = widths
        self.c_in = c_in
        self.m = torch.nn.ModuleDict()
        for name, (w, b) in pn.split(c_in, widths, flat, s2d=True).items():
            k = w.shape[1]
            c = torch.nn.Conv2d(w.shape[3], w.shape[0], k, padding=k // 2).double()
            c.weight.data = torch.from_numpy(w.transpose(0, 3, 1, 2).copy())
            c.bias.data = torch.from_numpy(b.copy())
            self.m[name.replace(".", "_")] = c

    def forward(self, x):
        L, ci = len(self.widths), self.c_in
        c = lambda n, t: self.m[n.replace(".", "_")](t)
        x = F.pixel_unshuffle(x, 2)[:, [cc * 4 + k for k in range(4) for cc in range(ci)]]
        skips = {}
        for l in range(1, L - 1):
            x = F.relu(c(f"E{l}.1", F.relu(c(f"E{l}.3", x))))
            skips[l] = x
            x = F.avg_pool2d(x, 2)
        x = F.relu(c("B.1", F.relu(c("B.3", x))))
        for l in range(L - 2, 0, -1):
            x = F.interpolate(x, scale_factor=2, mode="bilinear", align_corners=False) + skips[l]
            x = F.relu(c(f"D{l}.1", F.relu(c(f"D{l}.3", x))))
        y = c("OUT", x)
        base = F.interpolate(y[:, :1], scale_factor=2, mode="bilinear", align_corners=False)
        detail = F.pixel_shuffle(torch.cat([torch.zeros_like(y[:, :1]), y[:, 1:]], 1), 2)
        return (base + detail)[:, 0], y


@pytest.mark.parametrize("widths", [(16, 32, 64), (16, 32, 64, 128, 256)])
def test_s2d_forward_matches_torch(widths):
    n = pn.n_params(4, widths, s2d=True)
    flat = (SplitMix64(6).normals(n) * 0.2).astype(np.float32)
    feat = SplitMix64(7).uniforms(2 * 32 * 48 * 4, -1, 1).reshape(2, 32, 48, 4).astype(np.float32)
    got = pn.forward_s2d(4, widths, flat, feat)
    ref, y = TorchPNetS2D(4, widths, flat)(torch.from_numpy(feat.astype(np.float64).transpose(0, 3, 1, 2).copy()))
    np.testing.assert_allclose(got["logits"], ref.detach().numpy(), atol=1e-11)
    np.testing.assert_allclose(got["out4"], y.detach().numpy().transpose(0, 2, 3, 1), atol=1e-11)


def test_d2s_head_special_cases():
    y = SplitMix64(8).uniforms(1 * 5 * 7 * 4, -2, 2).reshape(1, 5, 7, 4)
    lg = pn.d2s_head(y)
    # no details: plain bilinear x2 of channel 0 (align_corners=False, clamped edges)
    z = y.copy()
    z[..., 1:] = 0
    up = F.interpolate(torch.from_numpy(y[..., 0][:, None].copy()), scale_factor=2, mode="bilinear",
                       align_corners=False)[:, 0].numpy()
    np.testing.assert_allclose(pn.d2s_head(z), up, atol=1e-14)
    # constant channel 0: the base is that constant everywhere
    k = y.copy()
    k[..., 0] = 0.75
    np.testing.assert_allclose(pn.d2s_head(k)[:, 0::2, 0::2], 0.75, atol=1e-15)
    np.testing.assert_allclose(pn.d2s_head(k)[:, 0::2, 1::2], 0.75 + y[..., 1], atol=1e-15)
    np.testing.assert_allclose(pn.d2s_head(k)[:, 1::2, 0::2], 0.75 + y[..., 2], atol=1e-15)
    np.testing.assert_allclose(pn.d2s_head(k)[:, 1::2, 1::2], 0.75 + y[..., 3], atol=1e-15)
    # interior output pixel (2i+1, 2j+1): 9/16, 3/16, 3/16, 1/16 of its four nearest low-res values
    i, j = 2, 3
    want = (9 * y[0, i, j, 0] + 3 * y[0, i + 1, j, 0] + 3 * y[0, i, j + 1, 0] + y[0, i + 1, j + 1, 0]) / 16
    assert lg[0, 2 * i + 1, 2 * j + 1] == pytest.approx(want + y[0, i, j, 3], abs=1e-14)
