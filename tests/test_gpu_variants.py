"""Launch variants of the forward stages (one workgroup per tile or a
persistent grid; default or alternative tile height) must all give the same
bits -- visibility, logits and every stored activation in the workspace --
and nsm_autotune must pick valid variants without changing any result."""
import itertools

import numpy as np
import pytest
import torch

import nsm_synth as S

pytestmark = pytest.mark.gpu


def _net(desc, dtype, flat):
    from paper_2301_05262_amd.api import ShadowNet
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m = ShadowNet(desc.c_in, desc.widths, dtype)
    m.set_weights(torch.from_numpy(flat))
    return m


def _run(m, f):
    vis, lg = m.forward(f, logits=True)
    torch.cuda.synchronize()
    n, h, w, _ = f.shape
    return vis.cpu().numpy().copy(), lg.cpu().numpy().copy(), m._ws.cpu().numpy().copy()


@pytest.mark.parametrize("dtype", ["bf16", "f32", "f8", "f16", "f8mfma"])
@pytest.mark.parametrize("desc,shape", [(S.U3, (2, 72, 200)), (S.U2, (1, 64, 96)), (S.U3_SOFT, (1, 136, 264))])
def test_every_variant_gives_the_same_bits(desc, shape, dtype):
    if dtype == "f8mfma" and desc is S.U2:
        pytest.skip("the FP8 compute form needs 16-channel tensors (U2 has 8)")
    n, h, w = shape
    flat = S.he_weights(desc, 71, bias_scale=0.1)
    feat = S.SplitMix64(72).uniforms(n * h * w * desc.c_in, -1, 1).reshape(n, h, w, desc.c_in).astype(np.float32)
    f = torch.from_numpy(feat).cuda()
    m = _net(desc, dtype, flat)
    ref = _run(m, f)
    nst = len(m.variants())
    for stage, v in itertools.product(range(nst), range(1, 4)):
        m.set_variant(stage, v)
        got = _run(m, f)
        m.set_variant(stage, 0)
        for a, b, what in zip(ref, got, ("vis", "logits", "workspace")):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (stage, v, what)
    # all stages persistent with the alternative tiles at once
    for stage in range(nst):
        m.set_variant(stage, 3)
    got = _run(m, f)
    assert all(np.array_equal(a.view(np.uint8), b.view(np.uint8)) for a, b in zip(ref, got))


def test_autotune_picks_valid_variants_and_keeps_bits():
    flat = S.he_weights(S.U3, 73)
    feat = S.SplitMix64(74).uniforms(2 * 256 * 512 * 6, -1, 1).reshape(2, 256, 512, 6).astype(np.float32)
    f = torch.from_numpy(feat).cuda()
    m = _net(S.U3, "bf16", flat)
    ref = _run(m, f)
    picked = m.autotune(f, reps=3)
    print(f"[autotune] variants {picked}", flush=True)
    assert len(picked) == 5 and all(0 <= v < 4 for v in picked)
    assert picked == m.variants()
    got = _run(m, f)
    assert all(np.array_equal(a.view(np.uint8), b.view(np.uint8)) for a, b in zip(ref, got))


def test_training_backward_with_variants():
    """The backward recomputes the forward with the context's variants: dW
    and dfeat keep their bits."""
    flat = S.he_weights(S.U3, 75, bias_scale=0.1)
    feat = torch.from_numpy(S.SplitMix64(76).uniforms(64 * 96 * 6, -1, 1).reshape(1, 64, 96, 6)
                            .astype(np.float32)).cuda()
    dvis = torch.from_numpy(S.SplitMix64(77).uniforms(64 * 96, -1, 1).reshape(1, 64, 96).astype(np.float32)).cuda()
    m = _net(S.U3, "f32", flat)
    dw0, df0 = m.backward(feat, dvis)
    dw0, df0 = dw0.cpu().numpy().copy(), df0.cpu().numpy().copy()
    for stage in range(5):
        m.set_variant(stage, 3)
    dw1, df1 = m.backward(feat, dvis)
    torch.cuda.synchronize()
    assert np.array_equal(dw0.view(np.uint32), dw1.cpu().numpy().view(np.uint32))
    assert np.array_equal(df0.view(np.uint32), df1.cpu().numpy().view(np.uint32))
