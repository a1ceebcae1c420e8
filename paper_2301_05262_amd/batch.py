"""Batched multi-frame inference captured in HIP graphs.

Frames of mixed sizes are grouped by resolution.  Each group's features are
built into one [N, H, W, C] tensor (one nsm_build_features call per frame;
for BF16 and FP16 networks nsm_build_features_stored, [N, H, W, 8] in the
network's storage type) and the network runs once per group: one launch per stage for all frames of
that size, each stage in the launch variant (one workgroup per tile or a
persistent grid, default or alternative tile height) that nsm_autotune found
fastest for the group's shape.  Each group is captured into its own graph;
a batch is the groups' graphs replayed in order, so the frames of a group
are complete when its graph is.  The library makes no allocation and no
memset inside these calls, so the captures hold only kernel nodes.
"""
from collections import OrderedDict

import torch

from .api import FeatureBuilder, ShadowNet


class BatchedPipeline:
    def __init__(self, frames, c_in, widths, weights, dtype="bf16", soft=True, device=None, side_streams=4,
                 stored=True):
        """frames: list of (scene, frame params).  The frames' feature builds
        (one builder, so one workspace, per frame) are spread over
        `side_streams` streams forked from the current one and joined before
        the group's network; in a capture they become parallel branches of
        the group's graph.  0 builds them in order on the current stream.
        stored: hand BF16 / FP16 networks their features in the storage type
        (same visibility bits, half the feature bytes); float32 otherwise."""
        self.device = torch.device(device if device is not None else "cuda")
        self.soft = soft
        self.stored = dtype if stored and dtype in ("bf16", "f16") else None
        self.frames = frames
        self.builders = [FeatureBuilder(sc, self.device) for sc, _ in frames]
        with torch.cuda.device(self.device):
            self.side = [torch.cuda.Stream() for _ in range(side_streams)]
        C = 8 if soft or self.stored else 6
        ft = {None: torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[self.stored]
        groups = OrderedDict()
        for i, (_, fr) in enumerate(frames):
            groups.setdefault((fr.height, fr.width), []).append(i)
        self.groups = []
        for (h, w), idx in groups.items():
            feat = torch.empty((len(idx), h, w, C), dtype=ft, device=self.device)
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
            net = ShadowNet(c_in, widths, dtype, self.device)    # one context per shape: its own variants
            net.set_weights(weights)
            net.workspace(len(idx), h, w)                        # sized before any capture
            self.groups.append({"hw": (h, w), "idx": idx, "feat": feat, "vis": vis, "bufs": bufs, "net": net,
                                "graph": None, "variants": net.variants()})

    def run_group(self, g):
        if self.side:
            main = torch.cuda.current_stream(self.device)
            fork = main.record_event()
            for s in self.side:
                s.wait_event(fork)
            for k, i in enumerate(g["idx"]):
                s = self.side[k % len(self.side)]
                self.builders[i](self.frames[i][1], soft=self.soft, out=g["bufs"][k], stream=s,
                                 stored=self.stored)
            for s in self.side:
                main.wait_event(s.record_event())
        else:
            for k, i in enumerate(g["idx"]):
                self.builders[i](self.frames[i][1], soft=self.soft, out=g["bufs"][k], stored=self.stored)
        g["net"].forward(g["feat"], vis_out=g["vis"])

    def run(self):
        """Eager pass over all frames (the same launches as the graphs)."""
        for g in self.groups:
            self.run_group(g)

    def autotune(self, reps=5):
        """Fastest launch variant per stage for every group (blocking)."""
        self.run()
        torch.cuda.synchronize()
        for g in self.groups:
            g["variants"] = g["net"].autotune(g["feat"], reps=reps)
        return [g["variants"] for g in self.groups]

    def capture(self, tune=True):
        if tune:
            self.autotune()
        self.run()                                  # warm-up: every workspace and variant is set up
        torch.cuda.synchronize()
        for g in self.groups:
            g["graph"] = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g["graph"]):
                self.run_group(g)
        torch.cuda.synchronize()

    def replay(self):
        for g in self.groups:
            g["graph"].replay()

    def replay_timed(self):
        """Replays one batch; returns (batch ms, [completion ms of every frame
        since the batch started], input order)."""
        ev0 = torch.cuda.Event(enable_timing=True)
        ends = [torch.cuda.Event(enable_timing=True) for _ in self.groups]
        ev0.record()
        for g, e in zip(self.groups, ends):
            g["graph"].replay()
            e.record()
        ends[-1].synchronize()
        done = [0.0] * len(self.frames)
        for g, e in zip(self.groups, ends):
            t = ev0.elapsed_time(e)
            for i in g["idx"]:
                done[i] = t
        return ev0.elapsed_time(ends[-1]), done

    def visibility(self):
        """[(frame index, vis [H, W])] in input order."""
        out = [None] * len(self.frames)
        for g in self.groups:
            for k, i in enumerate(g["idx"]):
                out[i] = g["vis"][k]
        return out
