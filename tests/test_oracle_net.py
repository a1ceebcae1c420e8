"""Pins for the FP64 network oracle (trimmed U-Net, paper Sec. 3.5).

Each step is checked against something other than itself: library routines
(torch float64 conv2d, max_pool2d, bilinear interpolate with half-pixel
centres, autograd), special weights with known outputs (identity, delta,
constant input), linearity, the adjoint identity <up(a), b> = <a, up^T(b)>,
float64 central finite differences, and closed-form MAC/parameter counts.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import net
from nsm_synth import SplitMix64, U2, U3, U3_SOFT, he_weights



@pytest.fixture(autouse=True)
def _float64_default():
    """torch tensors built in these tests default to float64; restored after
    each test so that no other module sees the change."""
    old = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    yield
    torch.set_default_dtype(old)


def rnd(shape, seed, lo=-1.0, hi=1.0):
    return SplitMix64(seed).uniforms(int(np.prod(shape)), lo, hi).reshape(shape)


def t_nchw(x):
    return torch.from_numpy(np.ascontiguousarray(x.transpose(0, 3, 1, 2)))


def t_nhwc(t):
    return t.detach().numpy().transpose(0, 2, 3, 1)


# ---------------------------------------------------------------- conv3x3
@pytest.mark.parametrize("shape", [(1, 7, 9, 3, 5), (2, 8, 8, 16, 4), (1, 5, 12, 48, 16)])
def test_conv3x3_matches_torch(shape):
    n, h, w, ci, co = shape
    x = rnd((n, h, w, ci), 1)
    wt = rnd((co, 3, 3, ci), 2)
    b = rnd((co,), 3)
    y = net.conv3x3(x, wt, b)
    ref = F.conv2d(t_nchw(x), torch.from_numpy(wt.transpose(0, 3, 1, 2).copy()), torch.from_numpy(b), padding=1)
    np.testing.assert_allclose(y, t_nhwc(ref), rtol=0, atol=1e-12)


def test_conv3x3_identity_and_delta():
    x = np.abs(rnd((1, 6, 7, 4), 4))
    w = np.zeros((4, 3, 3, 4))
    for c in range(4):
        w[c, 1, 1, c] = 1.0
    np.testing.assert_array_equal(net.relu(net.conv3x3(x, w, np.zeros(4))), x)
    # a delta at (ky, kx) = (0, 2) reads the input at (y - 1, x + 1), zero outside
    w = np.zeros((4, 3, 3, 4))
    for c in range(4):
        w[c, 0, 2, c] = 1.0
    y = net.conv3x3(x, w, np.zeros(4))
    exp = np.zeros_like(x)
    exp[:, 1:, :-1] = x[:, :-1, 1:]
    np.testing.assert_array_equal(y, exp)


def test_conv3x3_linear_and_constant():
    x1, x2 = rnd((1, 6, 6, 3), 5), rnd((1, 6, 6, 3), 6)
    w = rnd((2, 3, 3, 3), 7)
    z = np.zeros(2)
    np.testing.assert_allclose(net.conv3x3(2 * x1 - 3 * x2, w, z),
                               2 * net.conv3x3(x1, w, z) - 3 * net.conv3x3(x2, w, z), atol=1e-13)
    c = np.full((1, 6, 6, 3), 0.7)
    b = np.array([0.1, -0.2])
    y = net.conv3x3(c, w, b)
    interior = 0.7 * w.sum(axis=(1, 2, 3)) + b
    np.testing.assert_allclose(y[0, 1:-1, 1:-1], np.broadcast_to(interior, (4, 4, 2)), atol=1e-14)


def test_conv3x3_backward_matches_autograd():
    x = rnd((2, 6, 8, 5), 8)
    w = rnd((3, 3, 3, 5), 9)
    dy = rnd((2, 6, 8, 3), 10)
    dx, dw, db = net.conv3x3_backward(x, w, dy)
    xt = t_nchw(x).requires_grad_(True)
    wt = torch.from_numpy(w.transpose(0, 3, 1, 2).copy()).requires_grad_(True)
    bt = torch.zeros(3, requires_grad=True)
    (F.conv2d(xt, wt, bt, padding=1) * t_nchw(dy)).sum().backward()
    np.testing.assert_allclose(dx, t_nhwc(xt.grad), atol=1e-12)
    np.testing.assert_allclose(dw, wt.grad.numpy().transpose(0, 2, 3, 1), atol=1e-12)
    np.testing.assert_allclose(db, bt.grad.numpy(), atol=1e-12)


# ----------------------------------------------------- pool / upsample / concat
def test_pool_and_upsample_match_torch():
    x = rnd((2, 6, 10, 3), 11)
    np.testing.assert_array_equal(net.maxpool2(x), t_nhwc(F.max_pool2d(t_nchw(x), 2)))
    up = F.interpolate(t_nchw(x), scale_factor=2, mode="bilinear", align_corners=False)
    np.testing.assert_allclose(net.upsample2(x), t_nhwc(up), atol=1e-15)


def test_upsample_invariants_and_adjoint():
    c = np.full((1, 5, 7, 2), 0.3)
    np.testing.assert_allclose(net.upsample2(c), 0.3, atol=1e-16)
    # a linear ramp in x is reproduced exactly away from the clamped border
    ramp = np.broadcast_to(np.arange(7.0)[None, None, :, None], (1, 5, 7, 1)).copy()
    u = net.upsample2(ramp)
    X = np.arange(14.0)
    np.testing.assert_allclose(u[0, 3, 1:-1, 0], ((X + 0.5) / 2 - 0.5)[1:-1], atol=1e-14)
    a, b = rnd((2, 5, 7, 3), 12), rnd((2, 10, 14, 3), 13)
    lhs = (net.upsample2(a) * b).sum()
    rhs = (a * net.upsample2_backward(b, 5, 7)).sum()
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_maxpool_backward_routes_to_first_max():
    x = np.zeros((1, 2, 2, 1))
    dy = np.ones((1, 1, 1, 1))
    # all equal: routed to (0, 0)
    np.testing.assert_array_equal(net.maxpool2_backward(x, dy)[0, :, :, 0], [[1, 0], [0, 0]])
    x[0, 1, 0, 0] = x[0, 1, 1, 0] = 2.0          # tie between (1,0) and (1,1): first wins
    np.testing.assert_array_equal(net.maxpool2_backward(x, dy)[0, :, :, 0], [[0, 0], [1, 0]])
    xr = rnd((1, 4, 6, 2), 14)
    d = rnd((1, 2, 3, 2), 15)
    xt = t_nchw(xr).requires_grad_(True)
    (F.max_pool2d(xt, 2) * t_nchw(d)).sum().backward()
    np.testing.assert_array_equal(net.maxpool2_backward(xr, d), t_nhwc(xt.grad))


# --------------------------------------------------------------- whole net
class TorchUNet(torch.nn.Module):
    """The same descriptor expressed with torch float64 modules."""

    def __init__(self, c_in, widths, flat):
        super().__init__()
        self.c_in, self.widths = c_in, widths
        P = net.split_params(c_in, widths, flat)
        self.convs = torch.nn.ModuleDict()
        for name, (w, b) in P.items():
            k = w.shape[1]
            m = torch.nn.Conv2d(w.shape[3], w.shape[0], k, padding=k // 2)
            m.weight.data = torch.from_numpy(w.transpose(0, 3, 1, 2).copy())
            m.bias.data = torch.from_numpy(b.copy())
            self.convs[name] = m

    def forward(self, x):
        L = len(self.widths)
        skips = []
        for l in range(L - 1):
            x = F.relu(self.convs[f"E{l}"](x))
            skips.append(x)
            x = F.max_pool2d(x, 2)
        x = F.relu(self.convs["B"](x))
        for l in range(L - 2, -1, -1):
            x = F.interpolate(x, scale_factor=2, mode="bilinear", align_corners=False)
            x = F.relu(self.convs[f"D{l}"](torch.cat([skips[l], x], dim=1)))
        return self.convs["H"](x)[:, 0]


@pytest.mark.parametrize("desc,hw", [(U2, (16, 24)), (U3, (16, 20)), (U3_SOFT, (12, 16))])
def test_forward_backward_match_torch(desc, hw):
    flat = he_weights(desc, 3, bias_scale=0.1)
    feat = rnd((2, hw[0], hw[1], desc.c_in), 16).astype(np.float32)
    out = net.forward(desc.c_in, desc.widths, flat, feat)
    model = TorchUNet(desc.c_in, desc.widths, flat)
    x = t_nchw(feat.astype(np.float64)).requires_grad_(True)
    logits = model(x)
    np.testing.assert_allclose(out["logits"], logits.detach().numpy(), atol=1e-12)
    dvis = rnd((2, hw[0], hw[1]), 17)
    vis = torch.sigmoid(logits)
    (vis * torch.from_numpy(dvis)).sum().backward()
    dflat, dfeat = net.backward(desc.c_in, desc.widths, flat, feat, dvis)
    tgrads = []
    for name, _, _, _ in net.stages(desc.c_in, desc.widths):
        m = model.convs[name]
        tgrads += [m.weight.grad.numpy().transpose(0, 2, 3, 1).reshape(-1), m.bias.grad.numpy()]
    np.testing.assert_allclose(dflat, np.concatenate(tgrads), atol=1e-11)
    np.testing.assert_allclose(dfeat, t_nhwc(x.grad), atol=1e-11)


def test_backward_finite_differences():
    desc = U3
    flat = he_weights(desc, 4, bias_scale=0.1)
    feat = rnd((1, 8, 8, 6), 18).astype(np.float32)
    dvis = rnd((1, 8, 8), 19)
    dflat, _ = net.backward(desc.c_in, desc.widths, flat, feat, dvis)
    f64 = flat.astype(np.float64)
    rng = SplitMix64(20)
    idx = sorted({int(rng.uniform(0, flat.size)) for _ in range(25)})
    for i in idx:
        h = 1e-6 * max(1.0, abs(f64[i]))
        p, m = f64.copy(), f64.copy()
        p[i] += h
        m[i] -= h
        fd = ((net.forward(6, desc.widths, p, feat)["vis"] * dvis).sum()
              - (net.forward(6, desc.widths, m, feat)["vis"] * dvis).sum()) / (2 * h)
        assert abs(fd - dflat[i]) <= 1e-6 * max(1.0, abs(dflat[i])), (i, fd, dflat[i])


def test_closed_form_counts():
    # U3 at 1920x1080: 17,008 MAC per full-resolution pixel, 58,641 parameters
    macs, params = net.count_macs_params(6, (16, 32, 64), 1080, 1920)
    assert params == 58641
    assert macs == 17008 * 1920 * 1080
    macs, params = net.count_macs_params(6, (8, 16), 64, 64)
    assert params == 3353


# ----------------------------------------------------- low-precision rounding
def test_storage_rounding_matches_torch_casts():
    x = np.concatenate([rnd((4000,), 21, -3, 3), [0.0, -0.0, 1.0, 65504.0, 1e-8, 3.0e38],
                        np.float32([1.00390625, 1.01171875, -1.00390625]).astype(np.float64)])
    tb = torch.from_numpy(x).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(net.round_bf16(x), tb)
    th = torch.from_numpy(x).to(torch.float32).to(torch.float16).to(torch.float64).numpy()
    np.testing.assert_array_equal(net.round_f16(x), th)


def test_lowp_forward_close_to_fp64():
    flat = he_weights(U3, 5)
    feat = rnd((1, 32, 32, 6), 22).astype(np.float32)
    ref = net.forward(6, U3.widths, flat, feat)["vis"]
    for dt, tol in (("bf16", 2e-2), ("f16", 3e-3)):
        v = net.forward_lowp(6, U3.widths, flat, feat, dt)["vis"]
        assert 0 < np.abs(v - ref).max() < tol


def test_e4m3_rounding_matches_torch_cast():
    """The 8-bit storage rounding against torch's float8_e4m3fn cast (ties to
    even) on random values, every representable value and every midpoint
    between neighbours; saturation at 448 beyond the cast's range."""
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    vals = np.unique(codes[np.isfinite(codes)])
    mids = 0.5 * (vals[1:] + vals[:-1])
    mag = np.exp(rnd((6000,), 23, np.log(1e-4), np.log(460.0)))
    x = np.concatenate([vals, mids, mag, -mag, [0.0, 2.0 ** -10, 3 * 2.0 ** -10]])
    x = x[np.abs(x) < 464.0].astype(np.float32).astype(np.float64)
    want = torch.from_numpy(x).to(torch.float32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(net.round_e4m3(x), want)
    np.testing.assert_array_equal(net.round_e4m3(vals), vals)
    np.testing.assert_array_equal(net.round_e4m3([464.0, 1e6, -1e30]), [448.0, 448.0, -448.0])


def test_f8_storage_forward_error():
    """8-bit storage keeps bfloat16 weights and compute; only stored
    activations carry E4M3's 3-bit mantissa (relative step 1/8)."""
    flat = he_weights(U3, 5)
    feat = rnd((1, 32, 32, 6), 22).astype(np.float32)
    ref = net.forward(6, U3.widths, flat, feat)["vis"]
    v8 = net.forward_lowp(6, U3.widths, flat, feat, "f8")["vis"]
    vb = net.forward_lowp(6, U3.widths, flat, feat, "bf16")["vis"]
    e8, eb = np.abs(v8 - ref).max(), np.abs(vb - ref).max()
    assert eb < e8 < 0.1
