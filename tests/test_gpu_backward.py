"""GPU parity of nsm_backward (the differentiation form, float32).

Gradients of sum(dvis * vis) w.r.t. the flat parameters and the features
must match the FP64 oracle adjoint norm-wise: max |gpu - oracle| <=
1e-4 * max |oracle| per tensor (and per stage for the weights).  Also:
bitwise run-to-run determinism, `accumulate`, float32 central finite
differences on a 16x16 crop, the torch.autograd.Function, and that a short
training run on ray-traced soft-shadow targets lowers the loss.
"""
import numpy as np
import pytest
import torch

import nsm_synth as S
import oracle
from oracle import net as onet

pytestmark = pytest.mark.gpu

REL = 1e-4


def _net(desc, flat):
    from paper_2301_05262_amd.api import ShadowNet
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m = ShadowNet(desc.c_in, desc.widths, "f32")
    m.set_weights(torch.from_numpy(flat))
    return m


def _rand(shape, seed, lo=-1.0, hi=1.0):
    return S.SplitMix64(seed).uniforms(int(np.prod(shape)), lo, hi).reshape(shape).astype(np.float32)


def _gpu_grads(m, feat, dvis, want_dfeat=True):
    f = torch.from_numpy(feat).cuda()
    d = torch.from_numpy(dvis.astype(np.float32)).cuda()
    dw, df = m.backward(f, d, want_dfeat=want_dfeat)
    torch.cuda.synchronize()
    return dw.cpu().numpy().astype(np.float64), (df.cpu().numpy().astype(np.float64) if want_dfeat else None)


def _stage_errors(desc, got, ref):
    out = {}
    off = 0
    for name, co, k, ci in onet.stages(desc.c_in, desc.widths):
        n = co * k * k * ci + co
        g, r = got[off:off + n], ref[off:off + n]
        out[name] = float(np.abs(g - r).max() / max(np.abs(r).max(), 1e-30))
        off += n
    return out


@pytest.mark.parametrize("desc,shape", [(S.U2, (2, 64, 64)), (S.U3, (2, 72, 200)), (S.U3_SOFT, (1, 32, 48)),
                                        (S.U3, (1, 4, 4))])
def test_backward_matches_oracle(desc, shape):
    n, h, w = shape
    flat = S.he_weights(desc, 21, bias_scale=0.1)
    feat = _rand((n, h, w, desc.c_in), 22)
    dvis = _rand((n, h, w), 23)
    ref_w, ref_f = onet.backward(desc.c_in, desc.widths, flat, feat, dvis)
    m = _net(desc, flat)
    dw, df = _gpu_grads(m, feat, dvis)
    per = _stage_errors(desc, dw, ref_w)
    e_f = np.abs(df - ref_f).max() / np.abs(ref_f).max()
    print(f"[{desc.widths}/{shape}] dW per-stage rel err {per}  dfeat {e_f:.3e}", flush=True)
    assert max(per.values()) <= REL and e_f <= REL
    # bitwise determinism and accumulate
    dw2, df2 = _gpu_grads(m, feat, dvis)
    np.testing.assert_array_equal(dw, dw2)
    np.testing.assert_array_equal(df, df2)
    acc = torch.from_numpy(dw.astype(np.float32)).cuda()
    m.backward(torch.from_numpy(feat).cuda(), torch.from_numpy(dvis).cuda(), dw_out=acc, accumulate=True,
               want_dfeat=False)
    torch.cuda.synchronize()
    np.testing.assert_allclose(acc.cpu().numpy(), 2 * dw.astype(np.float32), rtol=1e-6, atol=0)


# A ReLU mask or a max-pool route is fixed at float32 only where the decision
# is further from a tie than float32 rounding of the pre-activation.  The bound
# used: |z| (or the gap between a window's maximum and another window value)
# at most EPS_TIE * sum |w| |x| + |b| over the conv that produced it, about
# 170 float32 ulps of the absolute sum.
EPS_TIE = 1e-5
# Level-0 pixels beyond its own footprint from which the visibility gradient
# reaches a decision (the head is 1x1; each conv adjoint spreads one pixel of
# its level, each upsampling adjoint taps [2p-1, 2p+2]): D0 0, D1 2, B 6,
# E1 14 (skip 4, through the pool 14), E0 17 (skip 1, through the pool 17),
# the routes of the E1 and E0 pools 10 and 16.  Used with a margin;
# tests/test_reach_cpu.py measures each on the oracle and checks the table.
REACH = {"D0": 1, "D1": 4, "B": 8, "E1": 16, "E0": 20, "pool1": 12, "pool0": 18}


def _clear_windows(desc, flat, feat, axis, length=8, count=8):
    """Windows along the long image axis (1 = rows, 2 = columns) whose level-0
    extent no near-tie decision of the float64 forward can reach: there the
    float32 forward takes every decision the oracle takes."""
    act = onet.forward(desc.c_in, desc.widths, flat, feat)
    P = onet.split_params(desc.c_in, desc.widths, flat)
    L = len(desc.widths)
    size = feat.shape[axis]
    blocked = np.zeros(size + 1, np.int64)

    def block(coords, level, reach):
        lo = np.clip(coords * (1 << level) - reach, 0, size)
        hi = np.clip((coords + 1) * (1 << level) + reach, 0, size)
        np.add.at(blocked, lo, 1)
        np.add.at(blocked, hi, -1)

    inputs = {"E0": act["x"], "B": act[f"p_E{L - 2}"]}
    for l in range(1, L - 1):
        inputs[f"E{l}"] = act[f"p_E{l - 1}"]
    for l in range(L - 1):
        inputs[f"D{l}"] = np.concatenate([act[f"a_E{l}"], act[f"up_D{l}"]], -1)
    level = {"B": L - 1, **{f"E{l}": l for l in range(L - 1)}, **{f"D{l}": l for l in range(L - 1)}}
    for name, x in inputs.items():
        w, b = P[name]
        A = onet.conv3x3(np.abs(x), np.abs(w), np.abs(b))
        near = np.abs(act["z_" + name]) <= EPS_TIE * A
        pos = np.nonzero(near.any(axis=(0, 3 - axis, 3)))[0]
        block(pos, level[name], REACH[name])
        if name.startswith("E"):
            n, h, w_, c = A.shape
            win = lambda t: t.reshape(n, h // 2, 2, w_ // 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(
                n, h // 2, w_ // 2, 4, c)
            a, s = win(act["a_" + name]), win(A)
            top = a.max(axis=3, keepdims=True)
            close = (top - a <= EPS_TIE * s) & (a < top) & (top > 0)
            pos = np.nonzero(close.any(axis=3).any(axis=(0, 3 - axis, 3)))[0]
            block(pos, level[name] + 1, REACH["pool" + name[1:]])
    free = np.cumsum(blocked)[:size] == 0
    runs = np.convolve(free.astype(np.int64), np.ones(length, np.int64), "valid") == length
    starts = np.nonzero(runs)[0]
    picked = sorted({int(starts[np.abs(starts - t).argmin()]) for t in np.linspace(0, size - length, count)})
    return picked, act


def _near_ties(desc, flat, act):
    """[(level, mask [N, H_l, W_l], reach)] of the float64 forward's decisions
    within float32 rounding of a tie (ReLU pre-activations and max-pool gaps,
    bound EPS_TIE * sum |w| |x| + |b|)."""
    P = onet.split_params(desc.c_in, desc.widths, flat)
    L = len(desc.widths)
    inputs = {"E0": act["x"], "B": act[f"p_E{L - 2}"]}
    for l in range(1, L - 1):
        inputs[f"E{l}"] = act[f"p_E{l - 1}"]
    for l in range(L - 1):
        inputs[f"D{l}"] = np.concatenate([act[f"a_E{l}"], act[f"up_D{l}"]], -1)
    level = {"B": L - 1, **{f"E{l}": l for l in range(L - 1)}, **{f"D{l}": l for l in range(L - 1)}}
    out = []
    for name, x in inputs.items():
        w, b = P[name]
        A = onet.conv3x3(np.abs(x), np.abs(w), np.abs(b))
        out.append((level[name], (np.abs(act["z_" + name]) <= EPS_TIE * A).any(axis=3), REACH[name]))
        if name.startswith("E"):
            n, h, w_, c = A.shape
            win = lambda t: t.reshape(n, h // 2, 2, w_ // 2, 2, c).transpose(0, 1, 3, 2, 4, 5).reshape(
                n, h // 2, w_ // 2, 4, c)
            a, sa = win(act["a_" + name]), win(A)
            top = a.max(axis=3, keepdims=True)
            close = ((top - a <= EPS_TIE * sa) & (a < top) & (top > 0)).any(axis=3).any(axis=3)
            out.append((level[name] + 1, close, REACH["pool" + name[1:]]))
    return out


def _clear_mask(desc, flat, feat):
    """Level-0 pixels that no near-tie decision of the float64 forward can
    reach (2-D form of _clear_windows): a visibility gradient confined to
    them meets only decisions that float32 takes as float64 does."""
    act = onet.forward(desc.c_in, desc.widths, flat, feat)
    n, H, W = feat.shape[:3]
    blocked = np.zeros((n, H + 1, W + 1), np.int64)
    for lev, mask, reach in _near_ties(desc, flat, act):
        f, i, j = np.nonzero(mask)
        y0 = np.clip(i * (1 << lev) - reach, 0, H)
        y1 = np.clip((i + 1) * (1 << lev) + reach, 0, H)
        x0 = np.clip(j * (1 << lev) - reach, 0, W)
        x1 = np.clip((j + 1) * (1 << lev) + reach, 0, W)
        np.add.at(blocked, (f, y0, x0), 1)
        np.add.at(blocked, (f, y1, x0), -1)
        np.add.at(blocked, (f, y0, x1), -1)
        np.add.at(blocked, (f, y1, x1), 1)
    cover = blocked.cumsum(axis=1).cumsum(axis=2)[:, :H, :W]
    return cover == 0


@pytest.mark.parametrize("shape", [(1, 20, 16384), (1, 16384, 20)])
def test_backward_maximum_extent(shape):
    """The longest image side the library takes (16384), 20 pixels across.
    Over a third of a million pixels some hundreds of ReLU and max-pool
    decisions sit within float32 rounding of a tie, and flipping one moves a
    whole gradient; the visibility gradient is therefore non-zero only on
    8-pixel windows that no such decision reaches (chosen on the float64
    oracle alone), the first and last reachable ones included.  The whole
    extent is still processed: dW and dfeat (zero outside the windows' cones,
    exactly) are compared element-wise at the usual tolerance."""
    desc = S.U3
    n, h, w = shape
    axis = 2 if w > h else 1
    flat = S.he_weights(desc, 21, bias_scale=0.1)
    feat = _rand((n, h, w, desc.c_in), 22)
    starts, _ = _clear_windows(desc, flat, feat, axis)
    size = shape[axis]
    assert len(starts) >= 4 and starts[0] < 512 and starts[-1] > size - 512, starts
    keep = np.zeros(size, bool)
    for s0 in starts:
        keep[s0:s0 + 8] = True
    mask = keep[None, None, :] if axis == 2 else keep[None, :, None]
    dvis = (_rand((n, h, w), 23) * mask).astype(np.float32)
    ref_w, ref_f = onet.backward(desc.c_in, desc.widths, flat, feat, dvis)
    dw, df = _gpu_grads(_net(desc, flat), feat, dvis)
    per = _stage_errors(desc, dw, ref_w)
    e_f = np.abs(df - ref_f).max() / np.abs(ref_f).max()
    print(f"[{shape}] windows {starts}  dW per-stage rel err {per}  dfeat {e_f:.3e}", flush=True)
    assert max(per.values()) <= REL and e_f <= REL
    assert np.all(df[ref_f == 0] == 0)


def _soft_window_case(desc, seed, frames, width, height, sm_size):
    sc, frs = S.make_train_window(0, seed, width=width, height=height, sm_size=sm_size)
    feat = np.stack([oracle.build_features(sc, fr, soft=True)["feat"] for fr in frs[:frames]])
    return feat


def _check_soft_backward(desc, flat, feat, seed, tag, min_clear, dense_rel):
    """Gradient on the oracle's clear pixels only: dW per stage and dfeat
    element-wise at the usual tolerance, and dfeat exactly zero wherever the
    oracle's is.  Dense visibility gradient: dW per stage within
    `dense_rel`.  A dense gradient meets every ReLU and max-pool decision
    that float32 rounding can flip; each flip moves a gradient contribution
    to another pixel, so over millions of pixels dW moves by more than the
    float32 accumulation error (on the 4 x 512^2 window about 1e-3 of its
    largest entry), while the clear-pixel gradient, which meets no such
    decision, agrees to 1e-4."""
    dvis = _rand(feat.shape[:3], seed)
    ref_w, _ = onet.backward(desc.c_in, desc.widths, flat, feat, dvis)
    m = _net(desc, flat)
    dw, _ = _gpu_grads(m, feat, dvis, want_dfeat=False)
    per = _stage_errors(desc, dw, ref_w)
    print(f"[{tag}] dense dvis: dW per-stage rel err {per}", flush=True)
    assert max(per.values()) <= dense_rel
    clear = _clear_mask(desc, flat, feat)
    frac = float(clear.mean())
    dvc = (dvis * clear).astype(np.float32)
    ref_w, ref_f = onet.backward(desc.c_in, desc.widths, flat, feat, dvc)
    dw, df = _gpu_grads(m, feat, dvc)
    per = _stage_errors(desc, dw, ref_w)
    e_f = np.abs(df - ref_f).max() / np.abs(ref_f).max()
    print(f"[{tag}] dvis on the {frac:.1%} clear pixels: dW per-stage rel err {per}  dfeat {e_f:.3e}",
          flush=True)
    assert frac >= min_clear
    assert max(per.values()) <= REL and e_f <= REL
    assert np.all(df[ref_f == 0] == 0)


def test_backward_on_soft_shadow_features():
    """Rendered soft-shadow features are smooth, so thousands of 2x2 pooling
    windows hold two values that differ by less than float32 accumulation
    error (1e-7..1e-6): which one is the maximum, and so where the window's
    gradient goes, is not fixed at float32.  (A float32 PyTorch CPU forward
    on this input picks a different maximum than float64 in 37 windows and
    moves 6% of the dfeat elements.)  So dfeat is compared element-wise for a
    visibility gradient on the pixels that no such decision reaches (chosen
    on the float64 oracle alone); dW also with a dense gradient."""
    feat = _soft_window_case(S.U3_SOFT, 3, 2, 128, 96, 512)
    _check_soft_backward(S.U3_SOFT, S.he_weights(S.U3_SOFT, 2, bias_scale=0.1), feat, 24, "soft 2x96x128", 0.01, REL)


def test_backward_training_window_512():
    """One full training window of the soft-shadow training step (4 consecutive
    512 x 512 frames, SOFT8 rendered features, the U-Net the step trains) --
    at this scale every wgrad block reduces ~100 tiles.  Gradient on the
    clear pixels (about 14% of them, spread over all four frames): dW and
    dfeat element-wise; dense gradient: dW per stage within 5e-3 (decision
    flips near ties, see _check_soft_backward)."""
    feat = _soft_window_case(S.U3_SOFT, 0, 4, 512, 512, 1024)
    _check_soft_backward(S.U3_SOFT, S.he_weights(S.U3_SOFT, 0, bias_scale=0.1), feat, 29, "window 4x512x512",
                         0.1, 5e-3)


def test_finite_differences_on_crop():
    """Central differences of the GPU forward against the GPU gradient on a
    16x16 crop, relative error <= 5% with no absolute floor.

    The perturbed weights are formed in float64 and rounded to the float32
    the library takes; the difference quotient divides by the step actually
    taken.  For each weight the step is the largest of 2e-2 .. 1e-3 at which
    the float64 oracle's own central difference (same rounded weights) is
    within 1% of the float64 adjoint, i.e. no ReLU kink or curvature spoils
    the quotient at that step; the float32 noise of J (about 1e-5 over 256
    pixels, so 5e-3 in the quotient at the smallest step) stays below 1% of
    the gradients tested (the largest ones, about 2 and up)."""
    desc = S.U3
    flat = S.he_weights(desc, 25, bias_scale=0.1)
    feat = _rand((1, 16, 16, 6), 26)
    dvis = _rand((1, 16, 16), 27)
    m = _net(desc, flat)
    dw, df = _gpu_grads(m, feat, dvis)
    ref_w, _ = onet.backward(desc.c_in, desc.widths, flat, feat, dvis)
    f = torch.from_numpy(feat).cuda()
    d = torch.from_numpy(dvis).cuda().double()

    def J(p32):
        m.set_weights(torch.from_numpy(p32))
        v = m.forward(f).double()
        return float((v * d).sum())

    def J64(p32):
        return float((onet.forward(desc.c_in, desc.widths, p32, feat, keep=False)["vis"] * dvis).sum())

    order = np.argsort(-np.abs(dw))
    rng = S.SplitMix64(28)
    pick = sorted({int(order[int(rng.uniform(0, 400))]) for _ in range(30)})
    assert abs(dw[pick]).min() > 1.0
    tested = 0
    for i in pick:
        for hstep in (2e-2, 1e-2, 5e-3, 2e-3, 1e-3):
            p, q = flat.astype(np.float64).copy(), flat.astype(np.float64).copy()
            p[i] += hstep
            q[i] -= hstep
            p32, q32 = p.astype(np.float32), q.astype(np.float32)
            step = (float(p32[i]) - float(q32[i])) / 2.0
            fd64 = (J64(p32) - J64(q32)) / (2 * step)
            if abs(fd64 - ref_w[i]) <= 1e-2 * abs(ref_w[i]):
                break
        else:
            continue
        fd = (J(p32) - J(q32)) / (2 * step)
        print(f"[fd] w[{i}] step {step:.3e}: fd {fd:.6f} gpu grad {dw[i]:.6f} "
              f"({abs(fd - dw[i]) / abs(dw[i]):.2e})", flush=True)
        assert abs(fd - dw[i]) <= 5e-2 * abs(dw[i]), (i, fd, dw[i])
        tested += 1
    assert tested >= 20, tested


def test_autograd_function_and_training_step():
    """NSMForward inside a torch training loop: MSE against 64-sample ray-cast
    soft visibility on a small window; the loss must go down."""
    from paper_2301_05262_amd.api import NSMForward, ShadowNet
    sc, frames = S.make_train_window(1, 0, width=64, height=64, sm_size=256)
    feats, targets = [], []
    for fr in frames:
        o = oracle.build_features(sc, fr, soft=True)
        fg = o["gbuf"] != oracle.EMPTY_KEY
        vis = oracle.raycast(sc, o["pos"], fg, fr.light_pos, radius=fr.light_radius, samples=64, seed=7)
        feats.append(o["feat"])
        targets.append(vis)
    feat = torch.from_numpy(np.stack(feats)).cuda()
    target = torch.from_numpy(np.stack(targets)).cuda()
    net = ShadowNet(8, S.U3_SOFT.widths, "f32")
    wts = torch.nn.Parameter(torch.from_numpy(S.he_weights(S.U3_SOFT, 3)).cuda())
    # one gradient against the oracle through the autograd path
    vis = NSMForward.apply(feat, wts, net)
    loss = torch.mean((vis - target) ** 2)
    loss.backward()
    dvis = (2.0 / vis.numel()) * (vis.detach() - target).cpu().numpy()
    ref_w, _ = onet.backward(8, S.U3_SOFT.widths, wts.detach().cpu().numpy(), feat.cpu().numpy(), dvis)
    g = wts.grad.detach().cpu().numpy().astype(np.float64)
    assert np.abs(g - ref_w).max() <= REL * np.abs(ref_w).max()
    opt = torch.optim.Adam([wts], lr=3e-3)
    losses = []
    for _ in range(60):
        opt.zero_grad()
        vis = NSMForward.apply(feat, wts, net)
        loss = torch.mean((vis - target) ** 2)
        loss.backward()
        opt.step()
        losses.append(float(loss))
    print(f"[train] loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert losses[-1] < 0.5 * losses[0]


def test_saved_forward_backward_same_bits():
    """nsm_forward_train + nsm_backward_saved: the visibility is nsm_forward's
    and the gradients are nsm_backward's, bit for bit; the saved forward is
    refused after nsm_set_weights, nsm_forward, or for other features."""
    import paper_2301_05262_amd as nsm
    desc, (n, h, w) = S.U3_SOFT, (2, 64, 96)
    flat = S.he_weights(desc, 17, bias_scale=0.1)
    m = _net(desc, flat)
    feat = torch.from_numpy(_rand((n, h, w, desc.c_in), 18)).cuda()
    dvis = torch.from_numpy(_rand((n, h, w), 19)).cuda()
    vis_inf = m.forward(feat).clone()
    vis_tr = m.forward_train(feat)
    dw_s, df_s = m.backward(feat, dvis, saved=True)
    dw_s, df_s = dw_s.clone(), df_s.clone()
    dw_s2, _ = m.backward(feat, dvis, saved=True)        # the adjoint leaves the activations intact
    dw_s2 = dw_s2.clone()
    dw_r, df_r = m.backward(feat, dvis)
    torch.cuda.synchronize()
    assert torch.equal(vis_inf, vis_tr)
    assert torch.equal(dw_s, dw_r) and torch.equal(df_s, df_r) and torch.equal(dw_s2, dw_r)
    # after the recomputing backward the workspace holds this forward again
    dw_s3, _ = m.backward(feat, dvis, saved=True)
    torch.cuda.synchronize()
    assert torch.equal(dw_s3, dw_r)

    def refused():
        with pytest.raises(nsm.NsmError) as ei:
            m.backward(feat, dvis, saved=True)
        assert ei.value.status == 1

    m.forward(feat)
    refused()
    m.forward_train(feat)
    m.set_weights(torch.from_numpy(flat))
    refused()
    m.forward_train(feat)
    other = feat.clone()
    with pytest.raises(nsm.NsmError):
        m.backward(other, dvis, saved=True)


def test_resume_from_checkpoint_same_bits(tmp_path):
    """A training run saved after three Adam steps and resumed in a new
    network context gives the fourth step's weight gradient and updated
    weights bit for bit (the backward is deterministic and the checkpoint
    keeps the flat weights and the optimizer state exactly)."""
    from paper_2301_05262_amd.api import NSMForward, ShadowNet, load_checkpoint, save_checkpoint
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    feat = torch.from_numpy(_rand((2, 32, 48, 8), 41)).cuda()
    target = torch.from_numpy(_rand((2, 32, 48), 42, 0.0, 1.0)).cuda()

    def step(net, wts, opt):
        opt.zero_grad()
        vis = NSMForward.apply(feat, wts, net)
        torch.mean((vis - target) ** 2).backward()
        g = wts.grad.detach().clone()
        opt.step()
        return g

    net = ShadowNet(8, S.U3_SOFT.widths, "f32")
    wts = torch.nn.Parameter(torch.from_numpy(S.he_weights(S.U3_SOFT, 4)).cuda())
    opt = torch.optim.Adam([wts], lr=3e-3)
    for _ in range(3):
        step(net, wts, opt)
    path = str(tmp_path / "ck")
    save_checkpoint(path, wts, opt)
    g_a = step(net, wts, opt)
    w_a = wts.detach().cpu()
    w0, state = load_checkpoint(path)
    net2 = ShadowNet(8, S.U3_SOFT.widths, "f32")
    wts2 = torch.nn.Parameter(w0)
    opt2 = torch.optim.Adam([wts2], lr=3e-3)
    opt2.load_state_dict(state)
    g_b = step(net2, wts2, opt2)
    torch.cuda.synchronize()
    assert torch.equal(g_a.cpu(), g_b.cpu())
    assert torch.equal(w_a, wts2.detach().cpu())

