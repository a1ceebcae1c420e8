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
* Per-pixel penumbra widths of a rendered frame (Sec. 3.6, supplemental
  Sec. 4): for every receiver, the blockers are the shadow-map texels in
  front of it (beyond the receiver's own surface) that lie inside the cone
  from the receiver to the emitter disk; their nearest and farthest depths
  are z_min and z_max, the receiver's own light depth is z_f, and the model
  above gives the world width, converted to screen pixels at the
  receiver's view depth.  The P95 of the widths over a set of frames picks
  the level count.
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


def _receivers(gbuf, tris, normals, fr):
    """World positions (float64) of the pixels' receivers -- the pixel-centre
    camera ray meets the plane of the key's triangle -- their camera-facing
    normals and the foreground mask.  gbuf: [H, W] int64 camera keys."""
    import torch

    dev = gbuf.device
    h, w = gbuf.shape
    key = gbuf.to(torch.int64)
    tid = key & 0xFFFFFFFF
    fg = (key != -1) & (tid < tris.shape[0])
    t = torch.where(fg, tid, torch.zeros_like(tid))
    V0 = tris[t, 0].double()
    N = normals[t].double()
    j = torch.arange(h, device=dev, dtype=torch.float64)[:, None]
    i = torch.arange(w, device=dev, dtype=torch.float64)[None, :]
    ndcx = (2.0 * (i + 0.5)) / w - 1.0
    ndcy = (2.0 * (j + 0.5)) / h - 1.0
    f64 = lambda v: torch.as_tensor(np.asarray(v, np.float64), device=dev)
    E, fwd, right, up = f64(fr.cam_pos), f64(fr.cam_fwd), f64(fr.cam_right), f64(fr.cam_up)
    D = (fwd + (ndcx * fr.cam_tan_half_x)[..., None] * right + (ndcy * fr.cam_tan_half_y)[..., None] * up)
    den = (N * D).sum(-1)
    fg = fg & (den != 0)
    tt = ((N * (V0 - E)).sum(-1)) / torch.where(den != 0, den, torch.ones_like(den))
    P = E + tt[..., None] * D
    Nf = torch.where(((N * (E - P)).sum(-1) < 0)[..., None], -N, N)
    return P, Nf, fg


def penumbra_widths(gbuf, sm_bits, tris, normals, fr, max_radius=48, chunk=64):
    """Per-pixel screen-space penumbra width (pixels) of one rendered frame
    under the penumbra model: 0 where the receiver has no blocker (and on
    background pixels).  gbuf [H, W] int64 keys and sm_bits [S, S] int32
    (float32 ndc depth bits) as nsm_build_features writes them; tris
    [T, 3, 3] and normals [T, 3] float32 tensors on the same device.

    A texel at distance rho (texels) from the receiver's own map position,
    with linear depth z_t, blocks part of the emitter disk when it is in
    front of the receiver's surface (by more than the depth change of the
    receiver's own plane over that distance, plus a texel) and when
    rho * texel(z_t) <= r_e (z_f - z_t) / z_f + texel(z_t) / sqrt 2, with
    texel(z) = 2 z tan(fov_L / 2) / S the texel's width at depth z: inside
    the cone from the receiver to the disk of radius r_e.  The search window
    is capped at `max_radius` texels.  Returns (widths [H, W] float64,
    z_min, z_max, z_f)."""
    import torch

    dev = gbuf.device
    h, w = gbuf.shape
    S = int(fr.sm_size)
    r_e = float(fr.light_radius)
    nl, fl, tanl = float(fr.light_near), float(fr.light_far), float(fr.light_tan_half_fov)
    P, N, fg = _receivers(gbuf, tris, normals, fr)
    M = torch.as_tensor(np.asarray(fr.m_light, np.float64).reshape(4, 4), device=dev)
    c = P @ M[:, :3].T + M[:, 3]
    cw = torch.where(c[..., 3] > 1e-6, c[..., 3], torch.ones_like(c[..., 3]))
    ndc = c[..., :3] / cw[..., None]
    sx = (ndc[..., 0] * 0.5 + 0.5) * S
    sy = (ndc[..., 1] * 0.5 + 0.5) * S
    lin = lambda q: (nl * fl) / (fl - q * (fl - nl))
    zf = lin(ndc[..., 2])
    inside = fg & (c[..., 3] > 1e-6) & (sx >= 0) & (sx < S) & (sy >= 0) & (sy < S) & (ndc[..., 2] >= 0) & (
        ndc[..., 2] <= 1)
    smf = sm_bits.view(torch.float32).double()
    smlin = torch.where(torch.isfinite(smf), lin(smf), torch.full_like(smf, float("inf")))
    # slope of the receiver's own plane against the light direction
    L = torch.as_tensor(np.asarray(fr.light_pos, np.float64), device=dev)
    l = L - P
    cosn = ((N * l).sum(-1) / l.norm(dim=-1)).clamp(min=1e-3)
    slope = (torch.sqrt((1 - cosn * cosn).clamp(min=0)) / cosn).clamp(max=10.0)
    ti = sx.floor().clamp(0, S - 1).long()
    tj = sy.floor().clamp(0, S - 1).long()
    tex_f = 2.0 * zf * tanl / S
    R = int(min(max_radius, math.ceil(r_e * S / (2.0 * tanl * nl)) + 1)) if r_e > 0 else 1
    offs = [(du, dv) for dv in range(-R, R + 1) for du in range(-R, R + 1) if du * du + dv * dv <= (R + 1) ** 2]
    sel = inside.reshape(-1)
    idx = torch.nonzero(sel).squeeze(1)
    zmin = torch.full((idx.numel(),), float("inf"), dtype=torch.float64, device=dev)
    zmax = torch.full((idx.numel(),), -float("inf"), dtype=torch.float64, device=dev)
    qi, qj = ti.reshape(-1)[idx], tj.reshape(-1)[idx]
    qsx, qsy = sx.reshape(-1)[idx], sy.reshape(-1)[idx]
    qzf, qtex, qslope = zf.reshape(-1)[idx], tex_f.reshape(-1)[idx], slope.reshape(-1)[idx]
    for k0 in range(0, len(offs), chunk):
        o = torch.as_tensor(offs[k0:k0 + chunk], device=dev, dtype=torch.int64)
        ci = qi[None, :] + o[:, 0:1]
        cj = qj[None, :] + o[:, 1:2]
        ok = (ci >= 0) & (ci < S) & (cj >= 0) & (cj < S)
        zt = smlin[cj.clamp(0, S - 1), ci.clamp(0, S - 1)]
        rho = torch.sqrt((ci.double() + 0.5 - qsx[None]) ** 2 + (cj.double() + 0.5 - qsy[None]) ** 2)
        front = zt < qzf[None] - (rho + 1.0) * qtex[None] * (1.0 + qslope[None])
        tex_t = 2.0 * zt * tanl / S
        cone = rho * tex_t <= r_e * (qzf[None] - zt) / qzf[None] + tex_t / math.sqrt(2.0)
        hit = ok & front & cone & torch.isfinite(zt)
        zmin = torch.minimum(zmin, torch.where(hit, zt, torch.full_like(zt, float("inf"))).min(0).values)
        zmax = torch.maximum(zmax, torch.where(hit, zt, torch.full_like(zt, -float("inf"))).max(0).values)
    has = torch.isfinite(zmin)
    out_w = torch.zeros(h * w, dtype=torch.float64, device=dev)
    zmin_full = torch.full((h * w,), float("nan"), dtype=torch.float64, device=dev)
    zmax_full = zmin_full.clone()
    if bool(has.any()):
        zm, zx, zq = zmin[has], zmax[has], qzf[has]
        ww = torch.as_tensor(penumbra_width(zm.cpu().numpy(), zx.cpu().numpy(), zq.cpu().numpy(), r_e), device=dev)
        view = ((P.reshape(-1, 3)[idx][has] - torch.as_tensor(np.asarray(fr.cam_pos, np.float64), device=dev))
                * torch.as_tensor(np.asarray(fr.cam_fwd, np.float64), device=dev)).sum(-1)
        px = torch.as_tensor(width_in_pixels(ww.cpu().numpy(), view.cpu().numpy(), fr.cam_tan_half_y, h),
                             device=dev)
        out_w[idx[has]] = px
        zmin_full[idx[has]] = zm
        zmax_full[idx[has]] = zx
    return (out_w.reshape(h, w), zmin_full.reshape(h, w), zmax_full.reshape(h, w), zf)


def level_report(width_maps, available=(2, 3, 4, 5)):
    """P95 of the per-pixel widths (pixels with a penumbra, i.e. width > 0)
    over a set of frames, the level count the rule picks, and the share of
    penumbra pixels each level count's receptive field covers."""
    allw = np.concatenate([np.asarray(m).reshape(-1) for m in width_maps])
    pen = allw[np.isfinite(allw) & (allw > 0)]
    p95 = p95_width(pen)
    return {"penumbra_pixels": int(pen.size), "p95_width_px": p95,
            "levels": levels_for_width(p95, available) if pen.size else min(available),
            "covered_share": {int(l): float((pen <= receptive_field(l)).mean()) if pen.size else 1.0
                              for l in available}}


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
