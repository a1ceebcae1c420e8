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
