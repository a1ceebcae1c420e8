"""Features handed to the network in its storage type.

nsm_build_features_stored writes each feature channel rounded to bfloat16 or
float16 (nearest even) in [H][W][8], or to FP8 E4M3 bytes in [H][W][16], with
the channels past C zero; nsm_forward_stored reads that layout directly.
Checked here:

* the stored features equal the oracle's float32 features (bit-exact with
  the GPU's, tested elsewhere) rounded on the CPU: by torch for bfloat16 and
  float16, by the oracle's E4M3 rounding for the FP8 form; the padding
  channels are zero; G-buffer, shadow map and mask are those of
  nsm_build_features;
* the network on stored features gives the same bits as on the float32
  features (the float32 path rounds when it stages its first tile), in every
  launch variant of the first stage and after nsm_autotune_stored, and its
  visibility meets the 2e-2 bar against the FP64 oracle;
* the calls refuse what they do not support.
"""
import numpy as np
import pytest
import torch

import nsm_synth as S
import oracle
from oracle import net as onet

pytestmark = pytest.mark.gpu

TORCH_DT = {"bf16": torch.bfloat16, "f16": torch.float16, "f8mfma": torch.uint8}
WIDTH = {"bf16": 8, "f16": 8, "f8mfma": 16}


def _builder(scene):
    from paper_2301_05262_amd.api import FeatureBuilder
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return FeatureBuilder(scene)


def _net(desc, dtype, flat):
    from paper_2301_05262_amd.api import ShadowNet
    m = ShadowNet(desc.c_in, desc.widths, dtype)
    m.set_weights(torch.from_numpy(flat))
    return m


def _bits(t):
    return t.cpu().view(torch.int16).numpy()


def _frames():
    sc, fr = S.workload_frame("tiny_64", 1)
    yield "tiny_64", sc, fr, False
    sc = S.make_scene("objects60", 2)
    yield "ragged 203x117", sc, S.make_frame(sc, 203, 117, 300, (0.6, 3.3, -0.2), (2.7, 1.5, 1.9),
                                             light_radius=0.1), True
    sc, fr = S.workload_frame("hard_1080p", 0)
    yield "hard_1080p", sc, fr, False


FRAMES = list(_frames())


@pytest.mark.parametrize("case", range(len(FRAMES)))
@pytest.mark.parametrize("dt", ["bf16", "f16", "f8mfma"])
def test_stored_features_are_rounded_oracle_features(case, dt):
    name, sc, fr, soft = FRAMES[case]
    fb = _builder(sc)
    ref = oracle.build_features(sc, fr, soft=soft)
    C = ref["feat"].shape[-1]
    got = fb(fr, soft=soft, stored=dt)
    plain = fb(fr, soft=soft)
    torch.cuda.synchronize()
    assert got["feat"].dtype == TORCH_DT[dt] and tuple(got["feat"].shape) == (fr.height, fr.width, WIDTH[dt])
    gf = got["feat"].cpu()
    if dt == "f8mfma":
        # E4M3 bytes decoded exactly (no byte is the NaN pattern: the kernel saturates)
        vals = gf[..., :C].view(torch.float8_e4m3fn).to(torch.float64).numpy()
        want = onet._round_e4m3_via_f32(ref["feat"])
        n_bad = int((vals != want).sum())
        pad = gf[..., C:].numpy()
    else:
        want = torch.from_numpy(ref["feat"]).to(TORCH_DT[dt])
        n_bad = int((_bits(gf[..., :C]) != _bits(want)).sum())
        pad = _bits(gf[..., C:])
    print(f"[{name} {dt}] stored feature mismatches {n_bad} of {ref['feat'].size}", flush=True)
    assert n_bad == 0
    assert int((pad != 0).sum()) == 0
    for k in ("gbuf", "sm", "mask"):
        assert torch.equal(got[k], plain[k]), k


@pytest.mark.parametrize("desc,name,dt", [(S.U3, "hard_1080p", "bf16"), (S.U3, "hard_1080p", "f16"),
                                          (S.U3, "hard_1080p", "f8mfma"), (S.U2, "tiny_64", "bf16"),
                                          (S.U3_SOFT, "soft", "bf16"), (S.U3_SOFT, "soft", "f8mfma")])
def test_forward_on_stored_features_same_bits(desc, name, dt):
    if name == "soft":
        sc = S.make_scene("objects60", 3)
        fr = S.make_frame(sc, 200, 120, 256, (0.6, 3.3, -0.2), (2.7, 1.5, 1.9), light_radius=0.12)
    else:
        sc, fr = S.workload_frame(name, 0)
    soft = desc.c_in == 8
    fb = _builder(sc)
    f32 = fb(fr, soft=soft)["feat"].clone()
    st = fb(fr, soft=soft, stored=dt)["feat"].clone()
    m = _net(desc, dt, S.he_weights(desc, 21, bias_scale=0.1))
    v_ref, l_ref = m.forward(f32, logits=True)
    v_ref, l_ref = v_ref.clone(), l_ref.clone()
    for variant in range(4):
        m.set_variant(0, variant)
        v, lg = m.forward(st, logits=True)
        torch.cuda.synchronize()
        assert torch.equal(v, v_ref) and torch.equal(lg, l_ref), f"first-stage variant {variant}"
    picked = m.autotune(st.unsqueeze(0), reps=2)
    assert len(picked) == len(m.variants()) and all(0 <= v < 4 for v in picked)
    v = m.forward(st)
    torch.cuda.synchronize()
    assert torch.equal(v, v_ref)
    if name == "tiny_64":
        # against the FP64 network on the oracle's features
        ref = oracle.build_features(sc, fr, soft=soft)
        want = onet.forward(desc.c_in, desc.widths, S.he_weights(desc, 21, bias_scale=0.1),
                            ref["feat"][None].astype(np.float32), keep=False)["vis"]
        err = float(np.abs(v.cpu().numpy().astype(np.float64) - want).max())
        print(f"[{name} {dt}] stored-path vis max abs err vs FP64 {err:.3e}", flush=True)
        assert err <= 2e-2


def test_stored_calls_refuse_unsupported():
    from paper_2301_05262_amd import _lib
    from paper_2301_05262_amd.api import ShadowNet
    sc, fr = S.workload_frame("tiny_64", 0)
    fb = _builder(sc)
    with pytest.raises(_lib.NsmError) as e:
        fb(fr, fs="paper4", stored="bf16")
    assert e.value.status == 3
    feat = torch.zeros((1, 64, 64, 8), dtype=torch.float32, device="cuda")
    m32 = ShadowNet(S.U2.c_in, S.U2.widths, "f32")
    m32.set_weights(torch.from_numpy(S.he_weights(S.U2, 1)))
    ws = m32.workspace(1, 64, 64)
    vis = torch.empty((1, 64, 64), device="cuda")
    with pytest.raises(_lib.NsmError) as e:
        _lib.nsm_forward_stored(m32.ctx, feat, 1, 64, 64, vis, None, ws, ws.numel())
    assert e.value.status == 3
    with pytest.raises(_lib.NsmError) as e:
        _lib.nsm_autotune_stored(m32.ctx, feat, 1, 64, 64, vis, ws, ws.numel(), 1)
    assert e.value.status == 3
    mb = ShadowNet(S.U2.c_in, S.U2.widths, "bf16")
    with pytest.raises(ValueError):
        mb.forward(torch.zeros((1, 64, 64, 8), dtype=torch.float16, device="cuda"))
    # a caller's buffer of another type or shape is refused before any launch
    plain = fb(fr)
    with pytest.raises(ValueError):
        fb(fr, out=plain, stored="bf16")
    st = fb(fr, stored="f8mfma")
    with pytest.raises(ValueError):
        fb(fr, out=st, stored="bf16")
    with pytest.raises(ValueError):
        fb(fr, out=st)
