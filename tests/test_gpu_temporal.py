"""GPU parity of the temporal-stability entry points.

nsm_perturbation_loss (Eq. 2, per-pixel L1 term): dvis0 bit-exact and the
loss to 1e-12 relative against the oracle on the same inputs (both take the
same float64 steps; only the summation order differs), with planted ties
x_0 == x_i, ragged sizes and p = 0; a short training run with the loss.
nsm_temporal_instability (Eq. 3): the per-pixel outcome (rejection code or
D) bit-exact, the number of contributing pixels exact and the sum to 1e-12
relative, on consecutive frames of spline camera/light paths at a ragged
small size and at 1920x1080, for a static pair and an all-empty key buffer,
and accumulated over a sequence."""
import numpy as np
import pytest
import torch

import nsm_synth as S
import oracle
from oracle import temporal as ot

pytestmark = pytest.mark.gpu

ALPHA2 = float(np.float32(0.9))     # the ABI takes alpha as float32


def _loss_inputs(seed, n, p, h, w, ties=True):
    r = S.SplitMix64(seed)
    vis = r.uniforms(n * (1 + p) * h * w, 0, 1).reshape(n, 1 + p, h, w).astype(np.float32)
    tgt = r.uniforms(n * h * w, 0, 1).reshape(n, h, w).astype(np.float32)
    if ties and p > 0:
        vis[:, 1, ::3, ::5] = vis[:, 0, ::3, ::5]       # x_1 == x_0 on a lattice
        tgt[:, 1::7, ::2] = vis[:, 0, 1::7, ::2]        # target == x_0 on another
    return vis, tgt


@pytest.mark.parametrize("n,p,h,w", [(2, 3, 70, 130), (1, 0, 33, 17), (3, 1, 1, 1), (8, 3, 512, 512)])
def test_perturbation_loss_matches_oracle(n, p, h, w):
    from paper_2301_05262_amd.api import perturbation_loss
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    vis, tgt = _loss_inputs(10 + n, n, p, h, w)
    ref_loss, ref_g = ot.perturbation_loss(vis, tgt, alpha=ALPHA2)
    loss, g = perturbation_loss(torch.from_numpy(vis).cuda(), torch.from_numpy(tgt).cuda(), alpha=ALPHA2)
    torch.cuda.synchronize()
    got = float(loss.cpu()[0])
    print(f"[Eq.2 n{n} p{p} {h}x{w}] loss {got:.9f} vs {ref_loss:.9f}", flush=True)
    assert got == pytest.approx(ref_loss, rel=1e-12)
    np.testing.assert_array_equal(g.cpu().numpy(), ref_g.astype(np.float32))


def test_training_with_perturbation_loss():
    """Eq. 2 end to end on the GPU: features of an unperturbed frame and three
    perturbed copies, one forward over all four, the loss, and the backward
    through x_0 only; Adam on the weights must lower the loss."""
    from paper_2301_05262_amd.api import FeatureBuilder, ShadowNet, perturbation_loss
    sc, frames = S.make_train_window(2, 0, width=64, height=64, sm_size=256)
    fb = FeatureBuilder(sc)
    feats, targets = [], []
    for k, fr in enumerate(frames[:2]):
        group = [fr] + [S.perturb_frame(sc, fr, 100 * k + i) for i in range(3)]
        for g in group:
            feats.append(fb(g, fs="soft8")["feat"].clone())
        o = oracle.build_features(sc, fr, soft=True)
        fg = o["gbuf"] != oracle.EMPTY_KEY
        targets.append(oracle.raycast(sc, o["pos"], fg, fr.light_pos, radius=fr.light_radius, samples=16, seed=3))
    feat = torch.stack(feats)                                  # [2*4, H, W, 8], x_0 first per sample
    target = torch.from_numpy(np.stack(targets)).cuda()
    net = ShadowNet(8, S.U3_SOFT.widths, "f32")
    wts = torch.from_numpy(S.he_weights(S.U3_SOFT, 4)).cuda()
    m = torch.zeros_like(wts)
    v = torch.zeros_like(wts)
    losses = []
    for it in range(1, 41):
        net.set_weights(wts)
        vis = net.forward(feat).reshape(2, 4, 64, 64).contiguous()
        loss, dvis0 = perturbation_loss(vis, target)
        dw, _ = net.backward(feat.reshape(2, 4, 64, 64, 8)[:, 0].contiguous(), dvis0, want_dfeat=False)
        m = 0.9 * m + 0.1 * dw
        v = 0.999 * v + 0.001 * dw * dw
        wts = wts - 3e-3 * (m / (1 - 0.9 ** it)) / (torch.sqrt(v / (1 - 0.999 ** it)) + 1e-8)
        losses.append(float(loss.cpu()[0]))
    print(f"[Eq.2 training] loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert losses[-1] < 0.8 * losses[0]


def _gpu_pair(metric, fb, fr_prev, fr_cur, vis_prev, vis_cur):
    a = fb(fr_prev)["gbuf"].clone()
    b = fb(fr_cur)["gbuf"].clone()
    d = torch.empty((fr_cur.height, fr_cur.width), dtype=torch.float32, device="cuda")
    metric.add(fr_prev, fr_cur, a, b, vis_prev, vis_cur, d_out=d)
    torch.cuda.synchronize()
    return a.cpu().numpy().view(np.uint64), b.cpu().numpy().view(np.uint64), d.cpu().numpy()


@pytest.mark.parametrize("w,h", [(160, 96), (1920, 1080)])
def test_temporal_pair_matches_oracle(w, h):
    from paper_2301_05262_amd.api import FeatureBuilder, TemporalMetric
    sc, frames = S.make_train_window(3, 1, frames=2, width=w, height=h, sm_size=512)
    fb = FeatureBuilder(sc)
    r = S.SplitMix64(31)
    vp = r.uniforms(h * w, 0, 1).reshape(h, w).astype(np.float32)
    vc = np.clip(vp + r.uniforms(h * w, -0.2, 0.2).reshape(h, w), 0, 1).astype(np.float32)
    metric = TemporalMetric(sc, h, w)
    ga, gb, d = _gpu_pair(metric, fb, frames[0], frames[1], torch.from_numpy(vp).cuda(),
                          torch.from_numpy(vc).cuda())
    ra = oracle.raster(sc.tris, frames[0].m_cam, w, h, "key")[0]
    rb = oracle.raster(sc.tris, frames[1].m_cam, w, h, "key")[0]
    np.testing.assert_array_equal(ga, ra)
    np.testing.assert_array_equal(gb, rb)
    total, valid, dref = ot.temporal_pair(sc, frames[0], frames[1], ra, rb, vp, vc)
    s, k = metric.acc.tolist()
    codes, counts = np.unique(dref[dref < 0], return_counts=True)
    print(f"[Eq.3 {w}x{h}] sum {s:.6f} vs {total:.6f}, passed {int(k)} vs {valid}, "
          f"rejections {dict(zip(codes.tolist(), counts.tolist()))}", flush=True)
    np.testing.assert_array_equal(d, dref)
    assert int(k) == valid and valid > 0.3 * w * h
    assert s == pytest.approx(total, rel=1e-12)


def test_temporal_sequence_and_empty_scene():
    from paper_2301_05262_amd.api import FeatureBuilder, TemporalMetric
    w, h = 128, 72
    sc, frames = S.make_train_window(4, 2, frames=4, width=w, height=h, sm_size=256)
    fb = FeatureBuilder(sc)
    r = S.SplitMix64(41)
    vis = [r.uniforms(h * w, 0, 1).reshape(h, w).astype(np.float32) for _ in frames]
    metric = TemporalMetric(sc, h, w)
    sums = []
    for t in range(1, 4):
        _gpu_pair(metric, fb, frames[t - 1], frames[t], torch.from_numpy(vis[t - 1]).cuda(),
                  torch.from_numpy(vis[t]).cuda())
        ra = oracle.raster(sc.tris, frames[t - 1].m_cam, w, h, "key")[0]
        rb = oracle.raster(sc.tris, frames[t].m_cam, w, h, "key")[0]
        sums.append(ot.temporal_pair(sc, frames[t - 1], frames[t], ra, rb, vis[t - 1], vis[t])[0])
    e, _ = metric.value()
    assert e == pytest.approx(ot.instability(sums, w, h), rel=1e-12)
    # a static pair gives exactly zero; an empty key buffer gives no terms
    metric.reset()
    fr = frames[0]
    g = fb(fr)["gbuf"].clone()
    vt = torch.from_numpy(vis[0]).cuda()
    metric.add(fr, fr, g, g, vt, vt)
    empty = torch.full((h, w), -1, dtype=torch.int64, device="cuda")
    metric.add(fr, fr, empty, empty, vt, vt)
    s, k = metric.acc.tolist()
    assert s == 0.0 and k == float((g.cpu().numpy().view(np.uint64) != oracle.EMPTY_KEY).sum())
