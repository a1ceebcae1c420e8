"""Design-time analysis tools (host side): penumbra width, network depth and
channel sensitivity.

* Penumbra width (supplemental Sec. 4, the model of the "network depth
  optimization" section): a spherical emitter of radius r_e, an occluder
  bounded by a sphere spanning emitter distances [z_min, z_max] and a
  receiver at distance z_f.  With z_m the sphere centre's distance and r_s
  its radius, the inner / outer penumbra extents are
  x_{a,b} = z_f tan(theta -/+ theta_delta) - r_e with
  theta_delta = asin(r_s / sqrt(z_m^2 + r_e^2)) and
  theta = atan((r_e (z_f - z_m) / z_m + r_e) / z_f); the width is x_a + x_b.
* Depth rule (Sec. 3.6): halving the resolution per level with 3x3 kernels
  gives an effective receptive field of 3 * 2^l pixels for l levels, so
  l = log2(p_w / 3) levels cover a penumbra of p_w pixels; p_w is taken as
  the 95th percentile of the per-pixel screen-space widths.
* Sensitivity (Sec. 3.2, Eq. 1): S_i = E[|phi(f_i + eps_i) - phi(f_i)|] /
  (0.1 sigma_i) with eps_i ~ N(0, (0.1 sigma_i)^2) added to channel i only,
  and relative sensitivity s_i = S_i / sum_j S_j.  The expectation is taken
  over pixels and repeated draws; the absolute value is the reading used
  here (a signed mean would cancel).
"""
import math

import numpy as np


def penumbra_extents(z_min, z_max, z_f, r_e):
    """(x_a, x_b) in world units; arrays broadcast."""
    z_min, z_max, z_f, r_e = (np.asarray(v, np.float64) for v in (z_min, z_max, z_f, r_e))
    z_m = 0.5 * (z_max + z_min)
    r_s = 0.5 * (z_max - z_min)
    am = np.sqrt(z_m * z_m + r_e * r_e)
    theta_d = np.arcsin(np.clip(r_s / am, -1.0, 1.0))
    bq = r_e * (z_f - z_m) / z_m
    theta = np.arctan((bq + r_e) / z_f)
    x_a = z_f * np.tan(theta - theta_d) - r_e
    x_b = z_f * np.tan(theta + theta_d) - r_e
    return x_a, x_b


def penumbra_width(z_min, z_max, z_f, r_e):
    x_a, x_b = penumbra_extents(z_min, z_max, z_f, r_e)
    return x_a + x_b


def width_in_pixels(width_world, view_depth, tan_half_fov_y, height_px):
    """World-space width at a receiver of the given view depth -> screen pixels."""
    pixel_world = 2.0 * np.asarray(view_depth, np.float64) * tan_half_fov_y / height_px
    return np.asarray(width_world, np.float64) / pixel_world


def receptive_field(levels):
    """Effective receptive field (pixels) of a `levels`-level network."""
    return 3 * 2 ** int(levels)


def levels_for_width(p_w, available=None):
    """Smallest level count whose receptive field covers p_w pixels
    (l = ceil(log2(p_w / 3))); with `available`, the smallest allowed >= l."""
    l = max(1, math.ceil(math.log2(max(float(p_w), 3.0) / 3.0) - 1e-12))
    if available:
        ok = [a for a in sorted(available) if a >= l]
        return ok[0] if ok else max(available)
    return l


def p95_width(widths_px):
    w = np.asarray(widths_px, np.float64)
    w = w[np.isfinite(w) & (w > 0)]
    return float(np.quantile(w, 0.95)) if w.size else 0.0


def sensitivity(phi, feat, sigma=None, repeats=4, seed=0):
    """Relative sensitivity of each input channel of `phi`.

    phi: callable mapping a float32 torch tensor [N,H,W,C] on the GPU to the
    visibility [N,H,W] (e.g. ShadowNet.forward).  feat: [N,H,W,C] tensor.
    Returns (S [C], s [C])."""
    import torch

    C = feat.shape[-1]
    if sigma is None:
        sigma = feat.reshape(-1, C).double().std(dim=0).float()
    gen = torch.Generator(device=feat.device).manual_seed(seed)
    base = phi(feat).double()
    S = np.zeros(C)
    for i in range(C):
        if float(sigma[i]) == 0.0:
            continue
        acc = 0.0
        for _ in range(repeats):
            pert = feat.clone()
            eps = torch.randn(feat.shape[:-1], generator=gen, device=feat.device) * (0.1 * float(sigma[i]))
            pert[..., i] += eps
            acc += float((phi(pert).double() - base).abs().mean())
        S[i] = acc / repeats / (0.1 * float(sigma[i]))
    tot = S.sum()
    return S, (S / tot if tot > 0 else S)
