"""Seeded synthetic inputs for the neural shadow-mapping hot path.

This module produces *inputs only*: triangle soups, per-triangle face
normals, camera and light parameters (matrices built in float64 and rounded
to float32), network weights and training targets' random draws.  It holds
none of the method's arithmetic (no rasterisation, no feature composition,
no network evaluation), so both the CPU oracle and the GPU path can consume
the same bytes without sharing any computation.

Random numbers come from SplitMix64 (Steele, Lea and Flood 2014; the
constants are the published ones) so that every workload is reproducible
from an integer seed.
"""
from .rng import SplitMix64
from .scenes import (
    WORKLOADS,
    Scene,
    FrameParams,
    make_frame,
    make_scene,
    make_train_window,
    make_batched_frames,
    perturb_frame,
    workload_frame,
)
from .nets import NetDesc, U2, U3, U3_SOFT, layer_shapes, n_params, he_weights

__all__ = [
    "SplitMix64",
    "WORKLOADS",
    "Scene",
    "FrameParams",
    "make_frame",
    "make_scene",
    "make_train_window",
    "make_batched_frames",
    "workload_frame",
    "NetDesc",
    "U2",
    "U3",
    "U3_SOFT",
    "layer_shapes",
    "n_params",
    "he_weights",
]
