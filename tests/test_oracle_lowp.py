"""Pins of the precision-form model in oracle/net.py (forward_lowp), which
the BF16 / FP16 / 8-bit GPU forms are compared with stored tensor by stored
tensor.

* phase_kernels: the 3x3 kernel per output phase that folds the bilinear x2
  upsampling into the conv equals, tap by tap, the response of the float64
  conv3x3(upsample2(.)) to a unit impulse at each low-resolution tap (brute
  force); phase_conv with it reproduces conv3x3(upsample2(low)) on every
  output pixel but the first and last rows and columns, and differs there
  (the zero padding of the upsampled image is not a clamp).
* forward_lowp: a pure-Python per-pixel evaluation of the same precision
  form on tiny images -- explicit loops for every conv tap, the bilinear
  weights from their half-pixel definition, phase kernels summed from those
  weights, rounding by torch's own dtype casts -- must give every stored
  tensor exactly and the logits to 1e-12.
* Each plausible misplacement of a rounding point, planted in the oracle
  (features, weights, biases, stored activations, pooled tensor, phase
  kernels, border upsampled tensor, head input, head weights, E4M3 storage),
  makes that comparison fail.
"""
import math

import numpy as np
import pytest
import torch

import nsm_synth as S
from oracle import net as onet


# --------------------------------------------------------------- phase form
def test_phase_kernels_equal_impulse_responses():
    rng = np.random.default_rng(3)
    co, cu = 3, 2
    w = rng.standard_normal((co, 3, 3, cu))
    Wp = onet.phase_kernels(w)
    hl = wl = 7
    i, j = 3, 3                    # interior low pixel: output pixels (2i + py, 2j + px)
    for t in range(3):
        for u in range(3):
            for c in range(cu):
                low = np.zeros((1, hl, wl, cu))
                low[0, i - 1 + t, j - 1 + u, c] = 1.0
                resp = onet.conv3x3(onet.upsample2(low), w, np.zeros(co))
                for py in range(2):
                    for px in range(2):
                        got = Wp[py, px, :, t, u, c]
                        assert np.array_equal(got, resp[0, 2 * i + py, 2 * j + px]), (t, u, c, py, px)


def test_phase_conv_equals_upsampled_conv_away_from_border():
    rng = np.random.default_rng(4)
    low = rng.standard_normal((2, 5, 7, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    ref = onet.conv3x3(onet.upsample2(low), w, np.zeros(4))
    got = onet.phase_conv(low, onet.phase_kernels(w))
    inner = (slice(None), slice(1, -1), slice(1, -1))
    assert np.abs(got[inner] - ref[inner]).max() <= 1e-12 * np.abs(ref).max()
    border = np.ones(ref.shape[1:3], bool)
    border[1:-1, 1:-1] = False
    assert np.abs(got[:, border] - ref[:, border]).min(axis=-1).max() > 1e-3


# ------------------------------------------------- scalar reference of the form
def _cast(x, dtype, storage):
    t = torch.from_numpy(np.asarray(x, np.float64))
    if (dtype == "f8" and storage) or dtype == "f8mfma":
        return t.to(torch.float32).clamp(-448.0, 448.0).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    tt = torch.float16 if dtype == "f16" else torch.bfloat16
    return t.to(torch.float32).to(tt).to(torch.float64).numpy()


def _bil_weight(out_idx, low_idx, n_low):
    """Weight of low sample low_idx in upsampled sample out_idx (half-pixel
    centres, taps clamped to [0, n_low))."""
    s = (out_idx + 0.5) / 2.0 - 0.5
    i0 = math.floor(s)
    fr = s - i0
    wsum = 0.0
    for tap, wt in ((i0, 1.0 - fr), (i0 + 1, fr)):
        if min(max(tap, 0), n_low - 1) == low_idx:
            wsum += wt
    return wsum


def _conv_px(x, w, b, y, xx, o):
    n_h, n_w, ci = x.shape
    acc = float(b[o])
    for ky in range(3):
        for kx in range(3):
            yy, xq = y + ky - 1, xx + kx - 1
            if 0 <= yy < n_h and 0 <= xq < n_w:
                for c in range(ci):
                    acc += float(w[o, ky, kx, c]) * float(x[yy, xq, c])
    return acc


def _conv(x, w, b):
    h, wd, _ = x.shape
    co = w.shape[0]
    return np.array([[[_conv_px(x, w, b, y, xx, o) for o in range(co)] for xx in range(wd)] for y in range(h)])


def _upsample(low):
    hl, wl, c = low.shape
    out = np.zeros((2 * hl, 2 * wl, c))
    for y in range(2 * hl):
        for x in range(2 * wl):
            for r in range(hl):
                wy = _bil_weight(y, r, hl)
                if wy == 0.0:
                    continue
                for q in range(wl):
                    wx = _bil_weight(x, q, wl)
                    if wx:
                        out[y, x] += wy * wx * low[r, q]
    return out


def _phase_px(low, wq_phase, y, x, o):
    hl, wl, cu = low.shape
    i, py, j, px = y // 2, y % 2, x // 2, x % 2
    acc = 0.0
    for t in range(3):
        for u in range(3):
            r, q = min(max(i - 1 + t, 0), hl - 1), min(max(j - 1 + u, 0), wl - 1)
            for c in range(cu):
                acc += float(wq_phase[py][px][o][t][u][c]) * float(low[r, q, c])
    return acc


def _phase_weights(w_up, dtype):
    """Phase kernels from the bilinear weights of an interior low pixel i = 10."""
    co, _, _, cu = w_up.shape
    i = 10
    wp = np.zeros((2, 2, co, 3, 3, cu))
    for py in range(2):
        for px in range(2):
            for t in range(3):
                for u in range(3):
                    cy = [_bil_weight(2 * i + py + ky - 1, i - 1 + t, 64) for ky in range(3)]
                    cx = [_bil_weight(2 * i + px + kx - 1, i - 1 + u, 64) for kx in range(3)]
                    for ky in range(3):
                        for kx in range(3):
                            if cy[ky] and cx[kx]:
                                wp[py, px, :, t, u, :] += cy[ky] * cx[kx] * w_up[:, ky, kx, :]
    return _cast(wp, dtype, False)


def _scalar_lowp(c_in, widths, flat, feat, dtype, boxes):
    P = onet.split_params(c_in, widths, flat)
    L = len(widths)
    x = _cast(feat[0], dtype, False)
    st = lambda a: _cast(a, dtype, True)
    out, skips, cur = {}, [], x
    for l in range(L - 1):
        w, b = P[f"E{l}"]
        a = np.maximum(_conv(cur, _cast(w, dtype, False), b), 0.0)
        e = st(a)
        h2, w2, c = e.shape
        pm = a.reshape(h2 // 2, 2, w2 // 2, 2, c).max(axis=(1, 3))
        skips.append(e)
        cur = st(pm)
        out[f"e{l}"], out[f"p{l}"] = e, cur
    w, b = P["B"]
    cur = st(np.maximum(_conv(cur, _cast(w, dtype, False), b), 0.0))
    out["b"] = cur
    for l in range(L - 2, -1, -1):
        w, b = P[f"D{l}"]
        skip = skips[l]
        cs = skip.shape[-1]
        wq = _cast(w, dtype, False)
        u = _cast(_upsample(cur), dtype, False)
        z = _conv(np.concatenate([skip, u], axis=-1), wq, b)
        box = boxes.get(f"D{l}")
        if box:
            wph = _phase_weights(w[..., cs:], dtype)
            r0, r1, c0, c1 = box
            for y in range(r0, r1):
                for xx in range(c0, c1):
                    for o in range(w.shape[0]):
                        z[y, xx, o] = _conv_px(skip, wq[..., :cs], b, y, xx, o) + _phase_px(cur, wph, y, xx, o)
        a = np.maximum(z, 0.0)
        if l > 0:
            cur = st(a)
            out[f"d{l}"] = cur
        else:
            cur = a
    wh, bh = P["H"]
    out["logits"] = np.array([[float(bh[0]) + sum(float(wh[0, 0, 0, c]) * float(cur[y, x, c])
                                                  for c in range(cur.shape[-1]))
                               for x in range(cur.shape[1])] for y in range(cur.shape[0])])
    return out


CASES = [
    ("U2", S.U2, (8, 12), {"D0": (1, 7, 2, 11)}),
    ("U3", S.U3, (8, 16), {"D1": (1, 3, 1, 7), "D0": (2, 7, 1, 14)}),
]


def _case(desc, hw, seed):
    h, w = hw
    flat = S.he_weights(desc, seed, bias_scale=0.1)
    feat = S.SplitMix64(seed + 1).uniforms(h * w * desc.c_in, -1, 1).reshape(1, h, w, desc.c_in)
    return flat, feat.astype(np.float32)


_REF = {}


def _reference(name, desc, hw, boxes, dtype):
    key = (name, dtype)
    if key not in _REF:
        flat, feat = _case(desc, hw, 7)
        _REF[key] = (flat, feat, _scalar_lowp(desc.c_in, desc.widths, flat, feat, dtype, boxes))
    return _REF[key]


def _mismatches(name, desc, hw, boxes, dtype):
    flat, feat, ref = _reference(name, desc, hw, boxes, dtype)
    got = onet.forward_lowp(desc.c_in, desc.widths, flat, feat, dtype, phase=boxes, keep=True)
    bad = []
    for k, v in ref.items():
        g = got[k][0]
        if k == "logits":
            if np.abs(g - v).max() > 1e-12 * max(1.0, np.abs(v).max()):
                bad.append(k)
        elif not np.array_equal(g, v):
            bad.append(k)
    return bad


@pytest.mark.parametrize("dtype", ["bf16", "f16", "f8", "f8mfma"])
@pytest.mark.parametrize("name,desc,hw,boxes", CASES)
def test_forward_lowp_equals_scalar_reference(name, desc, hw, boxes, dtype):
    assert _mismatches(name, desc, hw, boxes, dtype) == []


def _mutants():
    return {
        "features unrounded": ("_round_features", lambda x, cmp: x),
        "weights unrounded": ("_round_weights", lambda w, cmp: w),
        "biases rounded": ("_round_bias", lambda b: onet.round_bf16(b)),
        "activations unrounded": ("_store", lambda a, st: a),
        "pooled tensor unrounded": ("_store_pool", lambda a, st: onet.maxpool2(a)),
        "phase kernels unrounded": ("_phase_up", lambda low, w, cmp: onet.phase_conv(low, onet.phase_kernels(w))),
        "phase kernels of rounded weights": (
            "_phase_up", lambda low, w, cmp: onet.phase_conv(low, onet.phase_kernels(cmp(w)))),
        # the interior computed like the border: rounded weights on the rounded upsampled tensor
        "upsampled tensor rounded in the interior too": (
            "_phase_up", lambda low, w, cmp: onet.conv3x3(cmp(onet.upsample2(low)), cmp(w), np.zeros(w.shape[0]))),
        "border upsampled tensor unrounded": ("_border_up", lambda low, cmp: onet.upsample2(low)),
        "head input rounded": ("_head_input", lambda a: onet.round_bf16(a)),
        "head weights rounded": ("_head_weights", lambda w: onet.round_bf16(w)),
    }


@pytest.mark.parametrize("mutant", sorted(_mutants()))
def test_each_misplaced_rounding_point_is_caught(monkeypatch, mutant):
    attr, fn = _mutants()[mutant]
    monkeypatch.setattr(onet, attr, fn)
    caught = any(_mismatches(name, desc, hw, boxes, dt) for name, desc, hw, boxes in CASES
                 for dt in ("bf16", "f16", "f8"))
    assert caught, mutant


def test_f8_storage_rounding_is_caught(monkeypatch):
    """Storing E4M3 activations as bfloat16 (the compute type) is caught."""
    monkeypatch.setattr(onet, "_lowp_types", lambda dtype: (onet.round_bf16, onet.round_bf16))
    assert _mismatches(*CASES[1], "f8")


def test_phase_region_matters():
    """Computing every decoder pixel in the general form (no phase region) is caught."""
    name, desc, hw, boxes = CASES[1]
    flat, feat, ref = _reference(name, desc, hw, boxes, "bf16")
    got = onet.forward_lowp(desc.c_in, desc.widths, flat, feat, "bf16", phase=None, keep=True)
    assert not (np.array_equal(got["d1"][0], ref["d1"]) and
                np.abs(got["logits"][0] - ref["logits"]).max() <= 1e-12)
