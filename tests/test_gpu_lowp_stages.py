"""Precision forms (BF16, FP16 and 8-bit storage) against the oracle's model
of the form, stored tensor by stored tensor (tests/lowp_stages.py explains
the bound): every stored activation equals the model's or, where float32
accumulation puts it within reach of a rounding midpoint, the neighbouring
code; pooled tensors are exact max-pools; logits and visibility agree to the
float32 error of the head.  Shapes span several tiles with ragged tails, the
phase-form interior and border bands, batches, the widest screen, and the
rendered 1080p frame the benchmark times."""
import numpy as np
import pytest
import torch

import nsm_synth as S

from lowp_stages import check_stages

pytestmark = pytest.mark.gpu


def _run(desc, flat, feat, dtype):
    from paper_2301_05262_amd.api import ShadowNet
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m = ShadowNet(desc.c_in, desc.widths, dtype)
    m.set_weights(torch.from_numpy(flat))
    vis, lg = m.forward(torch.from_numpy(np.ascontiguousarray(feat, np.float32)).cuda(), logits=True)
    torch.cuda.synchronize()
    return m._ws, lg.cpu().numpy().astype(np.float64), vis.cpu().numpy().astype(np.float64)


def _rand(desc, shape, seed):
    n, h, w = shape
    flat = S.he_weights(desc, seed, bias_scale=0.1)
    feat = S.SplitMix64(seed + 1).uniforms(n * h * w * desc.c_in, -1, 1).reshape(n, h, w, desc.c_in)
    return flat, feat.astype(np.float32)


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f8", "f8mfma"])
@pytest.mark.parametrize("desc,shape", [(S.U2, (2, 64, 96)), (S.U3, (2, 72, 200)), (S.U3_SOFT, (1, 136, 264)),
                                        (S.U3, (1, 20, 4096))])
def test_stages_random_features(desc, shape, dtype):
    if dtype == "f8mfma" and desc is S.U2:
        pytest.skip("the FP8 compute form needs 16-channel tensors (U2 has 8)")
    flat, feat = _rand(desc, shape, 61)
    print(f"[stages] {desc.widths} {shape} {dtype}", flush=True)
    ws, lg, vis = _run(desc, flat, feat, dtype)
    check_stages(desc.c_in, desc.widths, flat, feat, dtype, ws, lg, vis, f"{desc.widths} {shape}")


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f8", "f8mfma"])
def test_stages_1080p_rendered_features(dtype):
    import oracle
    sc, fr = S.workload_frame("hard_1080p", 0)
    feat = oracle.build_features(sc, fr)["feat"][None]
    flat = S.he_weights(S.U3, 0)
    print(f"[stages] hard_1080p {dtype}", flush=True)
    ws, lg, vis = _run(S.U3, flat, feat, dtype)
    check_stages(6, S.U3.widths, flat, feat, dtype, ws, lg, vis, "hard_1080p")
