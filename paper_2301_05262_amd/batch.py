"""Batched multi-frame inference captured in one HIP graph.

Frames of mixed sizes are grouped by resolution; each group's features are
built into one [N, H, W, C] tensor (one nsm_build_features call per frame)
and the network runs once per group (one launch per stage for all frames of
that size).  The whole sequence is captured into a single graph and replayed.
The library makes no allocation and no memset inside these calls, so the
capture holds only kernel nodes.
"""
from collections import OrderedDict

import torch

from .api import FeatureBuilder, ShadowNet


class BatchedPipeline:
    def __init__(self, frames, c_in, widths, weights, dtype="bf16", soft=True, device=None):
        """frames: list of (scene, frame params)."""
        self.device = torch.device(device if device is not None else "cuda")
        self.soft = soft
        self.frames = frames
        self.builders = [FeatureBuilder(sc, self.device) for sc, _ in frames]
        C = 8 if soft else 6
        groups = OrderedDict()
        for i, (_, fr) in enumerate(frames):
            groups.setdefault((fr.height, fr.width), []).append(i)
        self.groups = []
        for (h, w), idx in groups.items():
            feat = torch.empty((len(idx), h, w, C), dtype=torch.float32, device=self.device)
            vis = torch.empty((len(idx), h, w), dtype=torch.float32, device=self.device)
            bufs = []
            for k, i in enumerate(idx):
                S = frames[i][1].sm_size
                bufs.append({
                    "feat": feat[k],
                    "mask": torch.empty((h, w), dtype=torch.uint8, device=self.device),
                    "sm": torch.empty((S, S), dtype=torch.int32, device=self.device),
                    "gbuf": torch.empty((h, w), dtype=torch.int64, device=self.device),
                })
            self.groups.append({"hw": (h, w), "idx": idx, "feat": feat, "vis": vis, "bufs": bufs})
        self.net = ShadowNet(c_in, widths, dtype, self.device)
        self.net.set_weights(weights)
        for g in self.groups:                       # workspaces sized before any capture
            n = len(g["idx"])
            self.net.workspace(n, *g["hw"])
        self.graph = None

    def run(self):
        """Eager pass over all frames (same launches as the graph)."""
        for g in self.groups:
            for k, i in enumerate(g["idx"]):
                self.builders[i](self.frames[i][1], soft=self.soft, out=g["bufs"][k])
            self.net.forward(g["feat"], vis_out=g["vis"])

    def capture(self):
        self.run()                                  # warm-up: every workspace exists
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()

    def visibility(self):
        """[(frame index, vis [H, W])] in input order."""
        out = [None] * len(self.frames)
        for g in self.groups:
            for k, i in enumerate(g["idx"]):
                out[i] = g["vis"][k]
        return out
