"""Eq. 1 sensitivity through the GPU network: a channel whose first-layer
weights are all zero has sensitivity exactly 0; the relative sensitivities
sum to 1."""
import numpy as np
import pytest
import torch

import nsm_synth as S

pytestmark = pytest.mark.gpu


def test_sensitivity_of_ignored_channel_is_zero():
    from paper_2301_05262_amd.analysis import sensitivity
    from paper_2301_05262_amd.api import ShadowNet
    assert torch.cuda.is_available()
    flat = S.he_weights(S.U3, 31)
    w = flat[:16 * 9 * 6].reshape(16, 3, 3, 6)
    w[..., 2] = 0.0                                  # E0 ignores channel 2
    net = ShadowNet(6, S.U3.widths, "f32")
    net.set_weights(torch.from_numpy(flat))
    feat = torch.from_numpy(S.SplitMix64(32).uniforms(2 * 64 * 96 * 6, -1, 1)
                            .reshape(2, 64, 96, 6).astype(np.float32)).cuda()
    Sabs, rel = sensitivity(net.forward, feat, repeats=2, seed=1)
    print("[sensitivity]", np.round(rel, 4), flush=True)
    assert Sabs[2] == 0.0
    assert (Sabs[[0, 1, 3, 4, 5]] > 0).all()
    assert abs(rel.sum() - 1.0) < 1e-12


def test_penumbra_levels_on_training_window():
    """The penumbra-width tool on one rendered soft-shadow training window (4
    frames of 512^2, map 1024^2) from the GPU's own buffers equals the same
    tool on the oracle's buffers (the buffers are bit-identical); the level
    report and Eq. 1 on the rendered SOFT8 features are printed."""
    import oracle
    from paper_2301_05262_amd.analysis import level_report, penumbra_widths, sensitivity
    from paper_2301_05262_amd.api import FeatureBuilder, ShadowNet
    sc, frames = S.make_train_window(0, 1)
    fb = FeatureBuilder(sc)
    tris, nrm = torch.from_numpy(sc.tris).cuda(), torch.from_numpy(sc.normals).cuda()
    maps, feats = [], []
    for k, fr in enumerate(frames):
        out = fb(fr, soft=True)
        w_gpu = penumbra_widths(out["gbuf"], out["sm"], tris, nrm, fr)[0].cpu().numpy()
        if k == 0:      # the host evaluation of the same tool on the oracle's buffers (one frame: it is slow)
            o = oracle.build_features(sc, fr, soft=True)
            w_cpu = penumbra_widths(torch.from_numpy(o["gbuf"].view(np.int64)),
                                    torch.from_numpy(o["sm"].view(np.int32)), torch.from_numpy(sc.tris),
                                    torch.from_numpy(sc.normals), fr, max_radius=16)[0].numpy()
            w16 = penumbra_widths(out["gbuf"], out["sm"], tris, nrm, fr, max_radius=16)[0].cpu().numpy()
            assert ((w16 > 0) == (w_cpu > 0)).mean() > 0.9999
            both = (w16 > 0) & (w_cpu > 0)
            assert np.abs(w16[both] - w_cpu[both]).max() <= 1e-9 * max(1.0, np.abs(w_cpu).max())
        maps.append(w_gpu)
        feats.append(out["feat"])
    rep = level_report(maps)
    print(f"[penumbra] r_e {frames[0].light_radius:.3f}: {rep}", flush=True)
    assert rep["penumbra_pixels"] > 0 and rep["levels"] in (2, 3, 4, 5)
    net = ShadowNet(8, S.U3_SOFT.widths, "f32")
    net.set_weights(torch.from_numpy(S.he_weights(S.U3_SOFT, 5)))
    Sabs, rel = sensitivity(net.forward, torch.stack(feats).contiguous(), repeats=2, seed=3)
    print("[sensitivity, rendered SOFT8]", np.round(rel, 4), flush=True)
    assert abs(rel.sum() - 1.0) < 1e-12 and (Sabs >= 0).all()
