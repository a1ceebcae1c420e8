"""Stage-by-stage comparison of a precision-form GPU forward (BF16, FP16 or
8-bit storage) with the oracle's model of that form (oracle/net.py).

Every stored tensor is read back from the forward workspace (its layout is
part of nsm_forward's contract) and each stage is recomputed by the oracle
from the GPU's own stored inputs, so a difference can only come from that
stage.  The GPU sums K exact products (bfloat16 / float16 operands) in
float32; with S the sum of the terms' magnitudes, its pre-activation lies
within gamma_{K+2} S of the oracle's float64 one, gamma_n = n u / (1 - n u),
u = 2^-24.  Storage rounding after ReLU is monotone, so the stored value must
lie in [st(relu(z - bound)), st(relu(z + bound))]: equal to the model's,
except where the pre-activation is within float32 accumulation error of a
rounding midpoint, where the neighbouring code is allowed.  On border
pixels of a decoder the GPU forms the upsampled tensor in float32 before
rounding it; where a value lies within 2^-22 of a rounding midpoint either
neighbour is allowed and the bound grows by the weights times that step.
Pooled tensors must equal the max-pool of the stored tensor bit for bit.
The head (float32 weights on float32 activations) is compared on logits.

The FP8 MFMA does not sum its 32 products exactly: measured on gfx950 with
operands whose products are powers of two, it aligns the products to the
largest one and keeps between 12 and 14 bits below it (a product 2^-12 of
the largest survives, 2^-14 is dropped, and so is 2^-18 after two large
products cancel; adding a product to the float32 accumulator is exact to
float32).  Each product of an MFMA is therefore off by less than 2^-12 of
the largest, so one MFMA by less than 32 * 2^-12 = 2^-7 of its sum of
magnitudes, and a stage by less than 2^-7 S.  For the 'f8mfma' form that
term is added to the bound, and more values may sit on the other side of a
rounding midpoint (up to 1% instead of 0.1%).
"""
import numpy as np
import torch

from oracle import net as onet

U = 2.0 ** -24


def gamma(n):
    return n * U / (1.0 - n * U)


def decode(raw, dtype, shape):
    t = torch.from_numpy(np.ascontiguousarray(raw))
    tt = {"bf16": torch.bfloat16, "f16": torch.float16, "f8": torch.float8_e4m3fn, "f8mfma": torch.float8_e4m3fn}[dtype]
    return t.view(tt).to(torch.float64).numpy().reshape(shape)


def workspace_tensors(ws, widths, n, h, w, dtype):
    """{name: float64 array} of the stored activations, in nsm_forward's
    documented workspace order (e_l, p_l for l < L-1; b; d_l for 1 <= l <= L-2),
    each at the next multiple of 256 bytes."""
    es = {"bf16": 2, "f16": 2, "f8": 1, "f8mfma": 1}[dtype]
    raw = ws.cpu().numpy()
    L = len(widths)
    off, out = 0, {}

    def take(name, shape):
        nonlocal off
        nb = int(np.prod(shape)) * es
        out[name] = decode(raw[off:off + nb], dtype, shape)
        off += (nb + 255) // 256 * 256

    for l in range(L - 1):
        take(f"e{l}", (n, h >> l, w >> l, widths[l]))
        take(f"p{l}", (n, h >> (l + 1), w >> (l + 1), widths[l]))
    take("b", (n, h >> (L - 1), w >> (L - 1), widths[L - 1]))
    for l in range(1, L - 1):
        take(f"d{l}", (n, h >> l, w >> l, widths[l]))
    return out


def phase_boxes(widths, h, w):
    """Output pixels of each decoder stage that the phase form computes: the
    kernel tiles the stage in bands of 16 rows (8 when the stage reads 96
    channels) by 32 columns and keeps the first and last band and tile column
    for the general form; with fewer than 3 tiles either way the whole stage
    is general."""
    L = len(widths)
    boxes = {}
    for l in range(L - 2, -1, -1):
        hl, wl = h >> l, w >> l
        band = 8 if widths[l] + widths[l + 1] >= 96 else 16
        gx, gy = -(-wl // 32), -(-hl // band)
        if gx >= 3 and gy >= 3:
            boxes[f"D{l}"] = (band, (gy - 1) * band, 32, (gx - 1) * 32)
    return boxes


def _interval_check(got, z, bound, st, tag, max_flips=1e-3):
    want = st(onet.relu(z))
    lo, hi = st(onet.relu(z - bound)), st(onet.relu(z + bound))
    ok = (got >= lo) & (got <= hi)
    neq = int((got != want).sum())
    print(f"    {tag}: {got.size} values, {neq} differ from the model "
          f"({neq / max(got.size, 1):.1e}), outside the rounding interval: {int((~ok).sum())}", flush=True)
    for k in np.argwhere(~ok)[:5]:
        k = tuple(k)
        print(f"      at {k}: stored {got[k]!r} model {want[k]!r} pre-activation {z[k]!r} "
              f"bound {bound[k]!r} interval [{lo[k]!r}, {hi[k]!r}]", flush=True)
    assert ok.all(), f"{tag}: {int((~ok).sum())} stored values outside the float32 rounding interval"
    assert neq <= max(8, max_flips * got.size), f"{tag}: too many flips ({neq})"


def _fragile_up(low, cmp):
    """Step of the rounded upsampled tensor where float32 interpolation could
    round it to the other neighbour (0 elsewhere)."""
    u = onet.upsample2(low)
    lo, hi = cmp(u * (1 - 2.0 ** -22)), cmp(u * (1 + 2.0 ** -22))
    return np.abs(hi - lo)


def check_stages(c_in, widths, flat, feat, dtype, ws, logits, vis, tag):
    n, h, w, _ = feat.shape
    L = len(widths)
    cmp, st = onet._lowp_types(dtype)
    P = onet.split_params(c_in, widths, flat)
    T = workspace_tensors(ws, widths, n, h, w, dtype)
    boxes = phase_boxes(widths, h, w)
    print(f"[{tag}] {dtype} phase boxes {boxes}", flush=True)
    mfma_rel = 2.0 ** -7 if dtype == "f8mfma" else 0.0     # FP8 MFMA product alignment (see above)
    flips = 1e-2 if dtype == "f8mfma" else 1e-3
    x = cmp(np.asarray(feat, np.float64))
    cur = x
    for l in range(L - 1):
        wgt, b = P[f"E{l}"]
        K = 9 * cur.shape[-1]
        z = onet.lowp_encoder_pre(cur, wgt, b, cmp)
        bound = (gamma(K + 2) + mfma_rel) * onet.lowp_encoder_pre(cur, wgt, b, cmp, magnitude=True)
        _interval_check(T[f"e{l}"], z, bound, st, f"E{l}", flips)
        assert np.array_equal(T[f"p{l}"], onet.maxpool2(T[f"e{l}"])), f"p{l} is not the max-pool of e{l}"
        cur = T[f"p{l}"]
    wgt, b = P["B"]
    z = onet.lowp_encoder_pre(cur, wgt, b, cmp)
    bound = (gamma(9 * cur.shape[-1] + 2) + mfma_rel) * onet.lowp_encoder_pre(cur, wgt, b, cmp, magnitude=True)
    _interval_check(T["b"], z, bound, st, "B", flips)
    low = T["b"]
    for l in range(L - 2, -1, -1):
        wgt, b = P[f"D{l}"]
        skip = T[f"e{l}"]
        cs = skip.shape[-1]
        box = boxes.get(f"D{l}")
        K = 9 * (cs + low.shape[-1])
        z = onet.lowp_decoder_pre(skip, low, wgt, b, cmp, box=box)
        mag = onet.lowp_decoder_pre(skip, low, wgt, b, cmp, box=box, magnitude=True)
        fr = np.concatenate([np.zeros_like(skip), _fragile_up(low, cmp)], axis=-1)
        extra = onet.conv3x3(fr, np.abs(cmp(wgt)), np.zeros(wgt.shape[0]))
        if box is not None:
            r0, r1, c0, c1 = box
            extra[:, r0:r1, c0:c1] = 0.0       # interior pixels do not read the upsampled tensor
        bound = (gamma(K + 2) + mfma_rel) * mag + extra
        if l > 0:
            _interval_check(T[f"d{l}"], z, bound, st, f"D{l}", flips)
            low = T[f"d{l}"]
            continue
        wh, bh = P["H"]
        a = onet.relu(z)
        ref = a @ wh[0, 0, 0, :] + bh[0]
        lb = (bound @ np.abs(wh[0, 0, 0, :]) + gamma(widths[0] + 2) * (np.abs(a) @ np.abs(wh[0, 0, 0, :])
                                                                      + abs(bh[0])))
        d = np.abs(logits - ref)
        print(f"    D0+head: max |logit - model| {d.max():.2e}, worst ratio to its bound "
              f"{(d / np.maximum(lb, 1e-30)).max():.2f}", flush=True)
        assert np.all(d <= 2.0 * lb + 1e-12), "logits outside the float32 accumulation bound"
        dv = np.abs(vis - onet.sigmoid(ref))
        assert np.all(dv <= 0.5 * lb + 2e-7), "visibility outside the bound of its logit"
