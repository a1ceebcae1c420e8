"""Pins for the oracle of the paper's own network (Sec. 4.5).

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
