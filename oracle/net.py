"""FP64 network oracle -- TEST INFRASTRUCTURE (tests, smoke check and the
benchmark's CPU-baseline leg only; the product never calls this).

The network is the trimmed U-Net of the paper (Sec. 3.5: one 3x3
convolution per level, bilinear upsampling instead of transposed
convolutions, a sigmoid-bounded visibility output since visibility lies in
[0, 1], supplemental Sec. 3) in the variant measured here: 2x2 max-pool
between encoder levels and skip merge by channel concatenation [skip, up].

Everything is float64.  Features and weights arrive as float32 and are
promoted exactly.  Operations follow their plain definitions:

  conv3x3   y[p, o] = b[o] + sum_{ky,kx,i} w[o,ky,kx,i] * x[p + (ky-1, kx-1), i]
            with zero padding outside the image (a library matmul sums over i
            for each of the nine taps);
  relu      max(x, 0);
  maxpool   2x2 windows, stride 2;
  upsample  bilinear x2 with half-pixel centres and clamp-to-edge:
            source coordinate s = (y + 0.5) / 2 - 0.5, taps floor(s) and
            floor(s) + 1 clamped to the image, weights (1 - frac, frac);
  head      1x1 convolution to one channel, then sigmoid 1 / (1 + e^-x).

Backward (used for the differentiation form): the exact adjoint of each
step.  ReLU passes gradient where its input is > 0 (derivative 0 at 0);
max-pool routes each window's gradient to the first maximum in the order
(0,0), (0,1), (1,0), (1,1); the upsampling adjoint is the transpose of the
interpolation (scatter-add with the same weights); concat splits channels.

Low-precision model (the precision form, Sec. 3.5 runs the network in half
precision): the same forward with round-to-nearest-even applied exactly
where the GPU path holds a value in a narrower type -- features on load,
3x3 weights, every stored activation; in the decoders, the upsampled tensor
on border pixels and the four phase kernels (bilinear x2 folded into the
3x3 weights, formed in float64 and rounded once) on interior pixels --
accumulating in float64.  The 1x1 head keeps float32 weights and reads the
unrounded last activation.  The 8-bit storage form rounds stored
activations to FP8 E4M3 and the rest to bfloat16; the FP8 compute form
rounds everything the MFMAs read to E4M3 as well.
"""
import numpy as np


# ------------------------------------------------------------- descriptor
def stages(c_in, widths):
    """[(name, C_out, k, C_in)] in flat-vector order E0.., B, D(L-2)..D0, H."""
    L = len(widths)
    out = []
    for l in range(L - 1):
        out.append((f"E{l}", widths[l], 3, c_in if l == 0 else widths[l - 1]))
    out.append(("B", widths[L - 1], 3, widths[L - 2] if L > 1 else c_in))
    for l in range(L - 2, -1, -1):
        out.append((f"D{l}", widths[l], 3, widths[l] + widths[l + 1]))
    out.append(("H", 1, 1, widths[0]))
    return out


def split_params(c_in, widths, flat):
    """Flat float32 vector -> {stage: (w [Co,k,k,Ci] f64, b [Co] f64)}."""
    flat = np.asarray(flat)
    res, off = {}, 0
    for name, co, k, ci in stages(c_in, widths):
        nw = co * k * k * ci
        w = flat[off:off + nw].astype(np.float64).reshape(co, k, k, ci)
        off += nw
        b = flat[off:off + co].astype(np.float64)
        off += co
        res[name] = (w, b)
    if off != flat.size:
        raise ValueError(f"parameter vector has {flat.size} entries, descriptor needs {off}")
    return res


def join_params(c_in, widths, grads):
    parts = []
    for name, co, k, ci in stages(c_in, widths):
        gw, gb = grads[name]
        parts.append(np.asarray(gw, np.float64).reshape(-1))
        parts.append(np.asarray(gb, np.float64).reshape(-1))
    return np.concatenate(parts)


# -------------------------------------------------------------- operations
def conv3x3(x, w, b):
    n, h, wd, ci = x.shape
    co = w.shape[0]
    xp = np.zeros((n, h + 2, wd + 2, ci))
    xp[:, 1:-1, 1:-1] = x
    y = np.empty((n, h, wd, co))
    y[...] = b
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + h, kx:kx + wd, :] @ w[:, ky, kx, :].T
    return y


def conv3x3_backward(x, w, dy):
    """Adjoint of conv3x3: (dx, dw, db)."""
    n, h, wd, ci = x.shape
    xp = np.zeros((n, h + 2, wd + 2, ci))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    dy2 = dy.reshape(-1, dy.shape[-1])
    for ky in range(3):
        for kx in range(3):
            xs = xp[:, ky:ky + h, kx:kx + wd, :].reshape(-1, ci)
            dw[:, ky, kx, :] = dy2.T @ xs
            dxp[:, ky:ky + h, kx:kx + wd, :] += dy @ w[:, ky, kx, :]
    db = dy2.sum(axis=0)
    return dxp[:, 1:-1, 1:-1], dw, db


def relu(x):
    return np.maximum(x, 0.0)


def maxpool2(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).max(axis=(2, 4))


def maxpool2_backward(x, dy):
    n, h, w, c = x.shape
    win = x.reshape(n, h // 2, 2, w // 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(n, h // 2, w // 2, 4, c)
    arg = np.argmax(win, axis=3)          # first maximum in (0,0),(0,1),(1,0),(1,1) order
    dwin = np.zeros_like(win)
    np.put_along_axis(dwin, arg[:, :, :, None, :], dy[:, :, :, None, :], axis=3)
    return dwin.reshape(n, h // 2, w // 2, 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(n, h, w, c)


def _interp_taps(n_out, n_in):
    y = np.arange(n_out, dtype=np.float64)
    s = (y + 0.5) / 2.0 - 0.5
    i0 = np.floor(s)
    fr = s - i0
    i0 = i0.astype(np.int64)
    i1 = i0 + 1
    return np.clip(i0, 0, n_in - 1), np.clip(i1, 0, n_in - 1), 1.0 - fr, fr


def upsample2(x):
    n, h, w, c = x.shape
    r0, r1, rw0, rw1 = _interp_taps(2 * h, h)
    c0, c1, cw0, cw1 = _interp_taps(2 * w, w)
    t = x[:, r0] * rw0[None, :, None, None] + x[:, r1] * rw1[None, :, None, None]
    return t[:, :, c0] * cw0[None, None, :, None] + t[:, :, c1] * cw1[None, None, :, None]


def upsample2_backward(dy, h, w):
    n, _, _, c = dy.shape
    r0, r1, rw0, rw1 = _interp_taps(2 * h, h)
    c0, c1, cw0, cw1 = _interp_taps(2 * w, w)
    dt = np.zeros((n, 2 * h, w, c))
    np.add.at(dt, (slice(None), slice(None), c0), dy * cw0[None, None, :, None])
    np.add.at(dt, (slice(None), slice(None), c1), dy * cw1[None, None, :, None])
    dx = np.zeros((n, h, w, c))
    np.add.at(dx, (slice(None), r0), dt * rw0[None, :, None, None])
    np.add.at(dx, (slice(None), r1), dt * rw1[None, :, None, None])
    return dx


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


# ------------------------------------------------------------------ network
def forward(c_in, widths, flat, feat, keep=True):
    """feat [N,H,W,C_in] (float32 or float64) -> dict with 'logits', 'vis' and
    every activation (pre-activation 'z_*', post-ReLU 'a_*', pooled 'p_*')."""
    P = split_params(c_in, widths, flat)
    L = len(widths)
    x = np.asarray(feat, np.float64)
    if x.ndim == 3:
        x = x[None]
    n, h, w, c = x.shape
    if c != c_in or h % (1 << (L - 1)) or w % (1 << (L - 1)):
        raise ValueError("feature shape does not fit the descriptor")
    act = {"x": x}
    cur = x
    skips = []
    for l in range(L - 1):
        z = conv3x3(cur, *P[f"E{l}"])
        a = relu(z)
        act[f"z_E{l}"], act[f"a_E{l}"] = z, a
        skips.append(a)
        cur = maxpool2(a)
        act[f"p_E{l}"] = cur
    z = conv3x3(cur, *P["B"])
    cur = relu(z)
    act["z_B"], act["a_B"] = z, cur
    for l in range(L - 2, -1, -1):
        u = upsample2(cur)
        cat = np.concatenate([skips[l], u], axis=-1)
        z = conv3x3(cat, *P[f"D{l}"])
        cur = relu(z)
        act[f"up_D{l}"], act[f"z_D{l}"], act[f"a_D{l}"] = u, z, cur
    wh, bh = P["H"]
    logits = cur @ wh[0, 0, 0, :] + bh[0]
    act["logits"] = logits
    act["vis"] = sigmoid(logits)
    if not keep:
        return {"logits": act["logits"], "vis": act["vis"]}
    return act


def backward(c_in, widths, flat, feat, dvis):
    """Gradients of sum(dvis * vis) w.r.t. the flat parameters and the features.

    Returns (dflat float64 [n_params], dfeat float64 [N,H,W,C_in])."""
    P = split_params(c_in, widths, flat)
    L = len(widths)
    act = forward(c_in, widths, flat, feat)
    dvis = np.asarray(dvis, np.float64).reshape(act["vis"].shape)
    vis = act["vis"]
    g = dvis * vis * (1.0 - vis)                      # d logits
    wh, bh = P["H"]
    top = act["a_D0"] if L > 1 else act["a_B"]
    grads = {"H": (np.einsum("nhw,nhwc->c", g, top).reshape(1, 1, 1, -1), np.array([g.sum()]))}
    dcur = g[..., None] * wh[0, 0, 0, :][None, None, None, :]
    dskip = [None] * (L - 1)
    for l in range(0, L - 1):
        zname = f"D{l}"
        dz = dcur * (act[f"z_{zname}"] > 0)
        cat = np.concatenate([act[f"a_E{l}"], act[f"up_{zname}"]], axis=-1)
        dcat, dw, db = conv3x3_backward(cat, P[zname][0], dz)
        grads[zname] = (dw, db)
        cs = widths[l]
        dskip[l] = dcat[..., :cs]
        lower = act["a_B"] if l == L - 2 else act[f"a_D{l + 1}"]
        dcur = upsample2_backward(dcat[..., cs:], lower.shape[1], lower.shape[2])
    dz = dcur * (act["z_B"] > 0)
    inp = act[f"p_E{L - 2}"] if L > 1 else act["x"]
    dinp, dw, db = conv3x3_backward(inp, P["B"][0], dz)
    grads["B"] = (dw, db)
    for l in range(L - 2, -1, -1):
        da = dskip[l] + maxpool2_backward(act[f"a_E{l}"], dinp)
        dz = da * (act[f"z_E{l}"] > 0)
        inp = act["x"] if l == 0 else act[f"p_E{l - 1}"]
        dinp, dw, db = conv3x3_backward(inp, P[f"E{l}"][0], dz)
        grads[f"E{l}"] = (dw, db)
    return join_params(c_in, widths, grads), dinp


# ------------------------------------------------------ low-precision model
def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even), via float32."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def round_f16(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def round_e4m3(x):
    """Round to the nearest OCP FP8 E4M3 value (ties to even), saturating at
    +-448: 4 exponent bits with bias 7 and 3 mantissa bits, so normal values
    step by 2^(e-3) in the binade [2^e, 2^(e+1)), e = -6 .. 8, and the
    subnormals below 2^-6 are multiples of 2^-9."""
    x = np.asarray(x, np.float64)
    a = np.minimum(np.abs(x), 448.0)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -6)))
    step = np.exp2(e - 3)
    q = np.minimum(np.round(a / step) * step, 448.0)      # np.round: half to even
    return np.where(x < 0, -q, q)


# Rounding points of the precision forms, one helper each, so that every
# point is a single place (and a test can move any one of them).  `cmp` rounds
# to the compute type the MFMAs read (bfloat16 or float16; bfloat16 in the
# 8-bit storage form), `st` to the storage type of activations in memory.
def _round_features(x, cmp):
    return cmp(x)


def _round_weights(w, cmp):
    return cmp(w)


def _round_bias(b):
    return b                       # biases stay float32


def _store(a, st):
    return st(a)


def _store_pool(a, st):
    return st(maxpool2(a))


def _phase_up(low, w_up, cmp):
    """Interior decoder pixels: the phase kernels of the float weights,
    formed in float64 and rounded once (via float32) to the compute type,
    applied to the stored low-resolution tensor."""
    return phase_conv(low, cmp(phase_kernels(w_up)))


def _border_up(low, cmp):
    """Border decoder pixels: the upsampled tensor, rounded to the compute
    type, feeds the plain 3x3 conv."""
    return cmp(upsample2(low))


def _head_input(a):
    return a                       # the last activation stays float32


def _head_weights(w):
    return w                       # head weights stay float32


def _round_e4m3_via_f32(x):
    return round_e4m3(np.asarray(x, np.float64).astype(np.float32))


def _lowp_types(dtype):
    cmp = {"bf16": round_bf16, "f16": round_f16, "f8": round_bf16, "f8mfma": _round_e4m3_via_f32}[dtype]
    st = round_e4m3 if dtype in ("f8", "f8mfma") else cmp
    return cmp, st


def up_coupling():
    """C[p, k, t]: weight of low-resolution row i - 1 + t in row 2i + p + k - 1
    of the bilinear x2 upsampling, away from the border (read off the taps of
    upsample2 at an interior row)."""
    n_low, i = 8, 4
    r0, r1, w0, w1 = _interp_taps(2 * n_low, n_low)
    C = np.zeros((2, 3, 3))
    for p in range(2):
        for k in range(3):
            u = 2 * i + p + k - 1
            C[p, k, r0[u] - (i - 1)] += w0[u]
            C[p, k, r1[u] - (i - 1)] += w1[u]
    return C


def phase_kernels(w_up):
    """Bilinear x2 followed by a 3x3 conv is linear in the low-resolution
    input, so away from the border it is a 3x3 conv over the low-resolution
    image with one kernel per output phase (y mod 2, x mod 2):
        Wp[py, px, o, t, u, c] = sum_{ky, kx} C[py, ky, t] C[px, kx, u] W[o, ky, kx, c].
    w_up [Co, 3, 3, Cu] -> Wp [2, 2, Co, 3, 3, Cu] (float64)."""
    C = up_coupling()
    return np.einsum("pkt,qlu,oklc->pqotuc", C, C, np.asarray(w_up, np.float64))


def phase_conv(low, Wp):
    """out[n, 2i + py, 2j + px, o] = sum_{t, u, c} Wp[py, px, o, t, u, c]
    * low[n, i - 1 + t, j - 1 + u, c], low taps clamped to the image (the
    clamp of the bilinear interpolation).  Equals conv3x3(upsample2(low), W)
    except on the first and last output rows and columns, where the conv's
    zero padding of the upsampled image is not a clamp."""
    n, hl, wl, _ = low.shape
    lp = np.pad(np.asarray(low, np.float64), ((0, 0), (1, 1), (1, 1), (0, 0)), mode="edge")
    co = Wp.shape[2]
    out = np.zeros((n, 2 * hl, 2 * wl, co))
    for py in range(2):
        for px in range(2):
            acc = np.zeros((n, hl, wl, co))
            for t in range(3):
                for u in range(3):
                    acc += lp[:, t:t + hl, u:u + wl, :] @ Wp[py, px, :, t, u, :].T
            out[:, py::2, px::2, :] = acc
    return out


def lowp_encoder_pre(x, w, b, cmp, magnitude=False):
    """Pre-activation of an encoder / bottleneck stage of the precision form
    from its stored input x; with magnitude=True the same sum over absolute
    values of every term (the scale of its float32 rounding error)."""
    wq, bq = _round_weights(w, cmp), _round_bias(b)
    if magnitude:
        return conv3x3(np.abs(x), np.abs(wq), np.abs(bq))
    return conv3x3(x, wq, bq)


def lowp_decoder_pre(skip, low, w, b, cmp, box=None, magnitude=False):
    """Pre-activation of a decoder stage (concat [skip, up(low)] -> 3x3) of the
    precision form from its stored inputs.  Output pixels inside `box`
    (r0, r1, c0, c1) take the phase form (phase kernels rounded once, applied
    to `low`); the others the general form (rounded weights on the rounded
    upsampled tensor).  magnitude=True: the sum over absolute values."""
    cs = skip.shape[-1]
    wq, bq = _round_weights(w, cmp), _round_bias(b)
    f = np.abs if magnitude else (lambda v: v)
    u = _border_up(low, cmp)
    z = conv3x3(f(np.concatenate([skip, u], axis=-1)), f(wq), f(bq))
    if box is not None:
        r0, r1, c0, c1 = box
        zs = conv3x3(f(skip), f(wq[..., :cs]), f(bq))
        if magnitude:
            zp = zs + phase_conv(np.abs(low), np.abs(cmp(phase_kernels(w[..., cs:]))))
        else:
            zp = zs + _phase_up(low, w[..., cs:], cmp)
        z[:, r0:r1, c0:c1] = zp[:, r0:r1, c0:c1]
    return z


def forward_lowp(c_in, widths, flat, feat, dtype, phase=None, keep=False):
    """Forward of the precision form with storage rounding at the GPU's store
    points (a bit model up to float32 accumulation order):

      features   rounded to the compute type on load;
      3x3 weights rounded to the compute type; biases float32;
      e_l, p_l   encoder outputs and their 2x2 max-pools, stored;
      b, d_l     bottleneck and decoder outputs (l >= 1), stored;
      decoders   interior pixels (phase[name] = (r0, r1, c0, c1) in the
                 stage's output pixels): the four phase kernels of the float
                 weights, formed in float64 and rounded once, applied to the
                 stored low-resolution tensor; other pixels: rounded weights
                 on the upsampled tensor rounded to the compute type;
      head       1x1 with float32 weights on the unrounded (float32) last
                 decoder activation, then the sigmoid.

    dtype 'bf16' / 'f16': compute and storage type alike; 'f8': storage E4M3,
    compute bfloat16; 'f8mfma': E4M3 for storage and compute (features,
    weights and phase kernels rounded to E4M3, via float32).  Sums are
    float64.  phase=None computes every decoder
    pixel in the general form.  keep=True also returns every stored tensor."""
    cmp, st = _lowp_types(dtype)
    phase = phase or {}
    P = split_params(c_in, widths, flat)
    L = len(widths)
    x = _round_features(np.asarray(feat, np.float64), cmp)
    if x.ndim == 3:
        x = x[None]
    out = {}
    cur = x
    skips = []
    for l in range(L - 1):
        a = relu(lowp_encoder_pre(cur, *P[f"E{l}"], cmp))
        skips.append(_store(a, st))
        cur = _store_pool(a, st)
        out[f"e{l}"], out[f"p{l}"] = skips[-1], cur
    cur = _store(relu(lowp_encoder_pre(cur, *P["B"], cmp)), st)
    out["b"] = cur
    for l in range(L - 2, -1, -1):
        a = relu(lowp_decoder_pre(skips[l], cur, *P[f"D{l}"], cmp, box=phase.get(f"D{l}")))
        if l > 0:
            cur = _store(a, st)
            out[f"d{l}"] = cur
        else:
            cur = _head_input(a)
    wh, bh = P["H"]
    logits = cur @ _head_weights(wh[0, 0, 0, :]) + bh[0]
    res = {"logits": logits, "vis": sigmoid(logits)}
    if keep:
        res.update(out)
    return res


# ------------------------------------------------------------ closed forms
def count_macs_params(c_in, widths, height, width):
    """(MACs per frame, parameters) of the descriptor at a given resolution."""
    macs = 0
    for name, co, k, ci in stages(c_in, widths):
        if name == "H":
            lvl = 0
        elif name == "B":
            lvl = len(widths) - 1
        else:
            lvl = int(name[1:])
        px = (height >> lvl) * (width >> lvl)
        macs += px * co * k * k * ci
    params = sum(co * k * k * ci + co for _, co, k, ci in stages(c_in, widths))
    return macs, params
