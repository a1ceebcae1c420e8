"""Network descriptors (shapes only) and seeded He-normal weights.

A descriptor names the input channel count and the per-level widths of a
U-Net whose stages are one 3x3 convolution each (the paper trims every level
to a single 3x3 convolution, Sec. 3.5), 2x2 max-pool between encoder levels,
bilinear x2 upsampling, skip concat [skip, up] and a 1x1 head with a sigmoid.

The flat parameter vector lists the stages in execution order
E0 .. E(L-2), B, D(L-2) .. D0, H; each stage stores its weights in OHWI order
[C_out][k][k][C_in] followed by its biases [C_out].
"""
from dataclasses import dataclass

import numpy as np

from .rng import SplitMix64


@dataclass(frozen=True)
class NetDesc:
    c_in: int
    widths: tuple

    @property
    def levels(self):
        return len(self.widths)


U2 = NetDesc(6, (8, 16))          # tiny 64x64 parity workload
U3 = NetDesc(6, (16, 32, 64))     # hard shadows, 6 channels
U3_SOFT = NetDesc(8, (16, 32, 64))  # soft shadows, 8 channels


def layer_shapes(desc):
    """[(name, C_out, k, C_in)] in flat-vector order."""
    w, L = desc.widths, desc.levels
    out = []
    for l in range(L - 1):
        out.append((f"E{l}", w[l], 3, desc.c_in if l == 0 else w[l - 1]))
    out.append(("B", w[L - 1], 3, w[L - 2] if L > 1 else desc.c_in))
    for l in range(L - 2, -1, -1):
        out.append((f"D{l}", w[l], 3, w[l] + w[l + 1]))
    out.append(("H", 1, 1, w[0]))
    return out


def n_params(desc):
    return sum(co * k * k * ci + co for _, co, k, ci in layer_shapes(desc))


def he_weights(desc, seed, bias_scale=0.0):
    """He-normal weights N(0, 2 / fan_in), fan_in = k*k*C_in (He et al. 2015).

    Biases are zero unless ``bias_scale`` > 0, in which case they are
    U[-bias_scale, bias_scale].  Returned as one float32 flat vector.
    """
    rng = SplitMix64(seed).fork(0x3E16)
    parts = []
    for _, co, k, ci in layer_shapes(desc):
        fan_in = k * k * ci
        parts.append(rng.normals(co * k * k * ci) * np.sqrt(2.0 / fan_in))
        if bias_scale > 0:
            parts.append(rng.uniforms(co, -bias_scale, bias_scale))
        else:
            parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
