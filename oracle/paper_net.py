"""FP64 oracle of the paper's own network ("P-net") -- TEST INFRASTRUCTURE.

The architecture the paper describes (Sec. 3.5): per level one 3x3 and one
1x1 convolution instead of a double 3x3; bilinear upsampling; skip merged by
an algebraic sum; average pooling; no skip connection at level 0; a 1x1
output convolution and a bounded (sigmoid) visibility.  The channel plan
that reproduces the paper's layer-wise tables (supplemental Table S2 and the
cost table S4) exactly, for widths w_0..w_{L-1} and c_in inputs:

  encoder level l < L-1:  3x3 C_{l-1} -> w_l, 1x1 w_l -> w_l   (C_{-1} = c_in)
  bottleneck  l = L-1:    3x3 w_{L-2} -> w_{L-1}, 1x1 w_{L-1} -> w_{L-2}
  decoder level l >= 1:   3x3 w_l -> w_l, 1x1 w_l -> w_{l-1}
  decoder level 0:        3x3 w_0 -> w_0, 1x1 w_0 -> w_0, output 1x1 w_0 -> 1

Every convolution is followed by a ReLU except the output one, which is
followed by the sigmoid.  Decoder level l reads up(y_{l+1}) + x_l (x_l the
encoder output at level l) for l >= 1 and up(y_1) alone at level 0.
Flat parameters: the convolutions in the order above (encoder levels, then
bottleneck, then decoder levels from L-2 down to 0, then the output conv),
each OHWI weights followed by biases.

The space-to-depth form (Sec. 3.5, the optimisation of the first level):
the level-0 convolutions are gone.  The input is rearranged into 2x2 blocks,
(H, W, c) -> (H/2, W/2, 4c), and fed straight to the level-1 encoder.  The
last decoder level (level 1) ends in a 1x1 output convolution to four
channels.  Channel 0 is bilinearly upsampled to full resolution, and channels
1..3 are added as the details of three of the four pixels of each 2x2 block.
Readings taken where the paper is silent:
  * channel order inside a block is block-major: channel (2 dy + dx) c_in + c
    holds pixel (2i + dy, 2j + dx), channel c;
  * the same order is used on the way out: detail channel k (1..3) belongs
    to the pixel (2i + k // 2, 2j + k % 2), and the pixel (2i, 2j) has no
    detail;
  * the output convolution is w_0 -> 4 at level 1, in place of w_0 -> 1 at
    level 0, and the sigmoid acts on the full-resolution sum.
"""
import numpy as np

from .net import conv3x3, relu, sigmoid, upsample2


def conv_list(c_in, widths):
    """[(name, C_out, k, C_in, level)] in flat order."""
    w, L = widths, len(widths)
    out = []
    for l in range(L - 1):
        out.append((f"E{l}.3", w[l], 3, c_in if l == 0 else w[l - 1], l))
        out.append((f"E{l}.1", w[l], 1, w[l], l))
    out.append(("B.3", w[L - 1], 3, w[L - 2], L - 1))
    out.append(("B.1", w[L - 2], 1, w[L - 1], L - 1))
    for l in range(L - 2, 0, -1):
        out.append((f"D{l}.3", w[l], 3, w[l], l))
        out.append((f"D{l}.1", w[l - 1], 1, w[l], l))
    out.append(("D0.3", w[0], 3, w[0], 0))
    out.append(("D0.1", w[0], 1, w[0], 0))
    out.append(("OUT", 1, 1, w[0], 0))
    return out


def conv_list_s2d(c_in, widths):
    """[(name, C_out, k, C_in, level)] of the space-to-depth form, flat order."""
    w, L = widths, len(widths)
    out = []
    for l in range(1, L - 1):
        out.append((f"E{l}.3", w[l], 3, 4 * c_in if l == 1 else w[l - 1], l))
        out.append((f"E{l}.1", w[l], 1, w[l], l))
    out.append(("B.3", w[L - 1], 3, w[L - 2], L - 1))
    out.append(("B.1", w[L - 2], 1, w[L - 1], L - 1))
    for l in range(L - 2, 0, -1):
        out.append((f"D{l}.3", w[l], 3, w[l], l))
        out.append((f"D{l}.1", w[l - 1], 1, w[l], l))
    out.append(("OUT", 4, 1, w[0], 1))
    return out


def _plan(c_in, widths, s2d):
    return conv_list_s2d(c_in, widths) if s2d else conv_list(c_in, widths)


def split(c_in, widths, flat, s2d=False):
    flat = np.asarray(flat)
    res, off = {}, 0
    for name, co, k, ci, _ in _plan(c_in, widths, s2d):
        n = co * k * k * ci
        res[name] = (flat[off:off + n].astype(np.float64).reshape(co, k, k, ci),
                     flat[off + n:off + n + co].astype(np.float64))
        off += n + co
    if off != flat.size:
        raise ValueError(f"expected {off} parameters, got {flat.size}")
    return res


def n_params(c_in, widths, s2d=False):
    return sum(co * k * k * ci + co for _, co, k, ci, _ in _plan(c_in, widths, s2d))


def conv1x1(x, w, b):
    return x @ w[:, 0, 0, :].T + b


def avgpool2(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def forward(c_in, widths, flat, feat):
    """feat [N,H,W,c_in] -> dict(logits, vis)."""
    P = split(c_in, widths, flat)
    L = len(widths)
    x = np.asarray(feat, np.float64)
    if x.ndim == 3:
        x = x[None]
    skips = []
    cur = x
    for l in range(L - 1):
        a = relu(conv3x3(cur, *P[f"E{l}.3"]))
        a = relu(conv1x1(a, *P[f"E{l}.1"]))
        skips.append(a)
        cur = avgpool2(a)
    cur = relu(conv3x3(cur, *P["B.3"]))
    cur = relu(conv1x1(cur, *P["B.1"]))
    for l in range(L - 2, -1, -1):
        u = upsample2(cur)
        if l >= 1:
            u = u + skips[l]
        a = relu(conv3x3(u, *P[f"D{l}.3"]))
        cur = relu(conv1x1(a, *P[f"D{l}.1"]))
    logits = conv1x1(cur, *P["OUT"])[..., 0]
    return {"logits": logits, "vis": sigmoid(logits)}


def layer_table(c_in, widths, height, width, s2d=False):
    """Per level: (MACs, weights (no biases), temp-storage IO elements).

    Temp-storage IO counts, for every convolution, its input plus output
    channels times the level's pixel count (pooling, upsampling and skip
    traffic are not counted)."""
    rows = {}
    for _, co, k, ci, lvl in _plan(c_in, widths, s2d):
        px = (height >> lvl) * (width >> lvl)
        m, p, io = rows.get(lvl, (0, 0, 0))
        rows[lvl] = (m + px * co * k * k * ci, p + co * k * k * ci, io + px * (ci + co))
    return [rows[l] for l in sorted(rows)]


def macs_per_pixel(c_in, widths, s2d=False):
    return sum(co * k * k * ci / 4.0 ** lvl for _, co, k, ci, lvl in _plan(c_in, widths, s2d))


# ------------------------------------------------------- space-to-depth form
def space_to_depth(x):
    """[N,H,W,C] -> [N,H/2,W/2,4C]; channel (2 dy + dx) C + c of block (i, j)
    is channel c of pixel (2i + dy, 2j + dx)."""
    n, h, w, c = x.shape
    if h % 2 or w % 2:
        raise ValueError("space-to-depth needs even sizes")
    return x.reshape(n, h // 2, 2, w // 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(n, h // 2, w // 2, 4 * c)


def depth_to_space(y):
    """Inverse of space_to_depth: [N,h,w,4C] -> [N,2h,2w,C]."""
    n, h, w, c4 = y.shape
    c = c4 // 4
    return y.reshape(n, h, w, 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(n, 2 * h, 2 * w, c)


def d2s_head(y):
    """Level-1 output [N,h,w,4] -> full-resolution logits [N,2h,2w]: the
    bilinear x2 upsampling of channel 0 plus channels 1..3 placed as the
    details of their 2x2-block pixels (no detail at the block's first pixel)."""
    base = upsample2(y[..., :1])[..., 0]
    detail = np.concatenate([np.zeros_like(y[..., :1]), y[..., 1:]], axis=-1)
    return base + depth_to_space(detail)[..., 0]


def forward_s2d(c_in, widths, flat, feat):
    """Space-to-depth form; feat [N,H,W,c_in] (H, W even) -> dict(logits, vis, out4)."""
    P = split(c_in, widths, flat, s2d=True)
    L = len(widths)
    x = np.asarray(feat, np.float64)
    if x.ndim == 3:
        x = x[None]
    cur = space_to_depth(x)
    skips = {}
    for l in range(1, L - 1):
        a = relu(conv3x3(cur, *P[f"E{l}.3"]))
        a = relu(conv1x1(a, *P[f"E{l}.1"]))
        skips[l] = a
        cur = avgpool2(a)
    cur = relu(conv3x3(cur, *P["B.3"]))
    cur = relu(conv1x1(cur, *P["B.1"]))
    for l in range(L - 2, 0, -1):
        u = upsample2(cur) + skips[l]
        a = relu(conv3x3(u, *P[f"D{l}.3"]))
        cur = relu(conv1x1(a, *P[f"D{l}.1"]))
    out4 = conv1x1(cur, *P["OUT"])
    logits = d2s_head(out4)
    return {"logits": logits, "vis": sigmoid(logits), "out4": out4}
