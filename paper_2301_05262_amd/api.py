"""Convenience wrappers over the C ABI (marshalling and buffer management only).

``FeatureBuilder`` keeps a scene's triangles on the device and calls
``nsm_build_features``; ``ShadowNet`` owns a network context and its
workspace and calls ``nsm_forward`` / ``nsm_backward``; ``NSMForward`` is the
differentiation form as a ``torch.autograd.Function``.  PyTorch only
provides device memory and the current stream.  ``save_checkpoint`` /
``load_checkpoint`` keep a training run's flat weights and optimizer state.
"""
import os

import numpy as np
import torch

from . import _lib


def _dev(device):
    return torch.device(device if device is not None else "cuda")


def _torch_stream(stream):
    """The torch stream object of a `stream=` argument (None: torch's current one)."""
    if stream is None or isinstance(stream, torch.cuda.Stream):
        return stream
    return torch.cuda.ExternalStream(int(stream))


def _grow(buf, need, device, stream):
    """A workspace of at least `need` bytes.  When the library runs on a stream
    other than torch's current one, torch's caching allocator must know that
    the old and new buffers are used there, or it could hand the old buffer
    out again while kernels queued on that stream still read it."""
    if buf is not None and buf.numel() >= need:
        return buf
    ts = _torch_stream(stream)
    if buf is not None and ts is not None:
        buf.record_stream(ts)
    buf = torch.empty(max(need, 256), dtype=torch.uint8, device=device)
    if ts is not None:
        buf.record_stream(ts)
    return buf


class FeatureBuilder:
    """Builds one frame's network input from a triangle scene on the GPU."""

    def __init__(self, scene, device=None):
        dev = _dev(device)
        self.device = dev
        self.tris = torch.from_numpy(scene.tris).to(dev).contiguous()
        self.normals = torch.from_numpy(scene.normals).to(dev).contiguous()
        self.n_tris = int(scene.tris.shape[0])
        self._ws = None

    def workspace(self, h, w, sm_size, stream=None):
        need = _lib.nsm_features_workspace_bytes(self.n_tris, h, w, sm_size)
        self._ws = _grow(self._ws, need, self.device, stream)
        return self._ws

    def __call__(self, fr, soft=False, out=None, stream=None, fs=None, stored=None):
        """Returns dict(feat [H,W,C] f32, mask [H,W] u8, sm [S,S] i32 bits, gbuf [H,W] i64 keys).

        fs: 'hard6', 'soft8' or 'paper4' (default: 'soft8' if soft else 'hard6').
        stored: None, or 'bf16' / 'f16' / 'f8mfma' for features in a network's
        storage type: [H,W,8] bfloat16 / float16 or [H,W,16] E4M3 bytes (uint8),
        the channels past C zero (nsm_build_features_stored)."""
        fs = fs or ("soft8" if soft else "hard6")
        h, w, S = fr.height, fr.width, fr.sm_size
        C = _lib.FEATURE_CHANNELS[fs]
        ft = {None: (C, torch.float32), "bf16": (8, torch.bfloat16), "f16": (8, torch.float16),
              "f8mfma": (16, torch.uint8)}[stored]
        if out is not None and (tuple(out["feat"].shape) != (h, w, ft[0]) or out["feat"].dtype != ft[1]
                                or not out["feat"].is_contiguous()):
            raise ValueError(f"out['feat'] must be a contiguous {ft[1]} tensor of shape {(h, w, ft[0])}")
        if out is None:
            out = {
                "feat": torch.empty((h, w, ft[0]), dtype=ft[1], device=self.device),
                "mask": torch.empty((h, w), dtype=torch.uint8, device=self.device),
                "sm": torch.empty((S, S), dtype=torch.int32, device=self.device),
                "gbuf": torch.empty((h, w), dtype=torch.int64, device=self.device),
            }
        ws = self.workspace(h, w, S, stream)
        if stored is None:
            _lib.nsm_build_features(self.tris, self.normals, self.n_tris, fr, h, w,
                                    fs, None, out["gbuf"], out["sm"],
                                    out["feat"], out["mask"], ws, ws.numel(), stream)
        else:
            _lib.nsm_build_features_stored(self.tris, self.normals, self.n_tris, fr, h, w,
                                           fs, None, out["gbuf"], out["sm"], stored,
                                           out["feat"], out["mask"], ws, ws.numel(), stream)
        return out


class ShadowNet:
    """A network context (descriptor + dtype) with its device weights."""

    def __init__(self, c_in, widths, dtype="f32", device=None, arch="unet"):
        self.device = _dev(device)
        self.c_in, self.widths, self.dtype = int(c_in), tuple(int(v) for v in widths), dtype
        self.arch = arch
        self.ctx = _lib.nsm_create(self.c_in, self.widths, dtype, arch)
        self.n_params = _lib.nsm_param_count(self.ctx)
        self._ws = None
        self._w = None

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                _lib.nsm_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    def set_weights(self, flat, stream=None):
        flat = torch.as_tensor(flat, dtype=torch.float32).to(self.device).contiguous()
        if flat.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {flat.numel()}")
        self._w = flat          # keep alive until the stream has copied it
        _lib.nsm_set_weights(self.ctx, flat, self.n_params, stream)

    def workspace(self, n, h, w, training=False, stream=None):
        need = _lib.nsm_workspace_bytes(self.ctx, n, h, w, int(training))
        self._ws = _grow(self._ws, need, self.device, stream)
        return self._ws

    _STORED = {"bf16": (torch.bfloat16, 8), "f16": (torch.float16, 8), "f8mfma": (torch.uint8, 16)}

    def _check_feat(self, feat):
        """True for features in the storage type (nsm_forward_stored), False for float32."""
        if not feat.is_contiguous():
            raise ValueError("features must be contiguous")
        c = feat.shape[-1]
        if feat.dtype == torch.float32 and c == self.c_in:
            return False
        if (feat.dtype, c) == self._STORED.get(self.dtype):
            return True
        raise ValueError("features must be float32 [N,H,W,c_in], or in the context's storage type "
                         "([N,H,W,8] bfloat16 / float16, [N,H,W,16] E4M3 bytes)")

    def forward(self, feat, logits=False, vis_out=None, logits_out=None, stream=None):
        """Visibility [N,H,W] for float32 features [N,H,W,c_in], or for features
        in the context's storage type (FeatureBuilder(stored=...))."""
        if feat.dim() == 3:
            feat = feat.unsqueeze(0)
        n, h, w, c = feat.shape
        stored = self._check_feat(feat)
        vis = vis_out if vis_out is not None else torch.empty((n, h, w), dtype=torch.float32,
                                                              device=feat.device)
        lg = logits_out
        if logits and lg is None:
            lg = torch.empty((n, h, w), dtype=torch.float32, device=feat.device)
        ws = self.workspace(n, h, w, stream=stream)
        call = _lib.nsm_forward_stored if stored else _lib.nsm_forward
        call(self.ctx, feat, n, h, w, vis, lg, ws, ws.numel(), stream)
        return (vis, lg) if logits else vis

    def autotune(self, feat, reps=5, stream=None):
        """Picks the fastest launch variant of every stage for this input shape
        (blocking; call before graph capture).  Returns the variants."""
        if feat.dim() == 3:
            feat = feat.unsqueeze(0)
        n, h, w, _ = feat.shape
        call = _lib.nsm_autotune_stored if self._check_feat(feat) else _lib.nsm_autotune
        vis = torch.empty((n, h, w), dtype=torch.float32, device=feat.device)
        ws = self.workspace(n, h, w, stream=stream)
        return call(self.ctx, feat, n, h, w, vis, ws, ws.numel(), reps, stream)

    def set_variant(self, stage, variant):
        _lib.nsm_set_stage_variant(self.ctx, stage, variant)

    def variants(self):
        return _lib.nsm_get_stage_variants(self.ctx)

    def forward_train(self, feat, vis_out=None, stream=None):
        """FP32 forward that keeps every activation in the training workspace
        for a following backward(..., saved=True) on the same features."""
        if feat.dim() == 3:
            feat = feat.unsqueeze(0)
        n, h, w, c = feat.shape
        if c != self.c_in or feat.dtype != torch.float32 or not feat.is_contiguous():
            raise ValueError("features must be contiguous float32 [N,H,W,c_in]")
        vis = vis_out if vis_out is not None else torch.empty((n, h, w), dtype=torch.float32,
                                                              device=feat.device)
        ws = self.workspace(n, h, w, training=True, stream=stream)
        _lib.nsm_forward_train(self.ctx, feat, n, h, w, vis, ws, ws.numel(), stream)
        return vis

    def backward(self, feat, dvis, dw_out=None, accumulate=False, want_dfeat=True, saved=False, stream=None):
        """saved=True reuses the activations of the last forward_train (or
        backward) on the same features instead of recomputing them."""
        if feat.dim() == 3:
            feat = feat.unsqueeze(0)
        n, h, w, c = feat.shape
        dvis = dvis.reshape(n, h, w).contiguous()
        dw = dw_out if dw_out is not None else torch.empty(self.n_params, dtype=torch.float32,
                                                           device=feat.device)
        df = torch.empty_like(feat) if want_dfeat else None
        ws = self.workspace(n, h, w, training=True, stream=stream)
        call = _lib.nsm_backward_saved if saved else _lib.nsm_backward
        call(self.ctx, feat, dvis, n, h, w, dw, int(accumulate), df, ws, ws.numel(), stream)
        return dw, df


class NSMForward(torch.autograd.Function):
    """vis = net(feat; weights) with the hand-written backward kernels.

    Saves only the features; the backward recomputes the activations."""

    @staticmethod
    def forward(ctx, feat, weights, net):
        net.set_weights(weights.detach())
        ctx.net = net
        ctx.save_for_backward(feat, weights)
        return net.forward(feat.detach().contiguous())

    @staticmethod
    def backward(ctx, dvis):
        feat, weights = ctx.saved_tensors
        net = ctx.net
        net.set_weights(weights.detach())
        dw, df = net.backward(feat.detach().contiguous(), dvis.contiguous(),
                              want_dfeat=ctx.needs_input_grad[0])
        return (df if ctx.needs_input_grad[0] else None), dw, None


def perturbation_loss(vis, target, alpha=0.9, stream=None):
    """Perturbation loss of Eq. 2 (per-pixel L1 term) and its gradient
    through x_0 only.

    vis [N, 1+p, H, W] float32 (x_0 first), target [N, H, W] float32 ->
    (loss: float64 tensor [1], dvis0: float32 [N, H, W])."""
    if vis.dim() == 3:
        vis, target = vis.unsqueeze(0), target.unsqueeze(0)
    n, q, h, w = vis.shape
    if (vis.dtype != torch.float32 or target.dtype != torch.float32 or not vis.is_contiguous()
            or not target.is_contiguous() or tuple(target.shape) != (n, h, w)):
        raise ValueError("vis must be contiguous float32 [N,1+p,H,W] and target [N,H,W]")
    need = _lib.nsm_perturbation_loss_workspace_bytes(n, q - 1, h, w)
    ws = torch.empty(need, dtype=torch.uint8, device=vis.device)
    loss = torch.empty(1, dtype=torch.float64, device=vis.device)
    dvis0 = torch.empty((n, h, w), dtype=torch.float32, device=vis.device)
    _lib.nsm_perturbation_loss(vis, target, n, q - 1, h, w, alpha, loss, dvis0, ws, ws.numel(), stream)
    return loss, dvis0


class TemporalMetric:
    """Temporal instability of Eq. 3 over a sequence of frames of one scene,
    accumulated on the device pair by pair."""

    def __init__(self, scene, height, width, alpha=3.0, depth_tol=0.01, cos_tol=0.9, device=None):
        dev = _dev(device)
        self.tris = torch.from_numpy(scene.tris).to(dev).contiguous()
        self.normals = torch.from_numpy(scene.normals).to(dev).contiguous()
        self.n_tris = int(scene.tris.shape[0])
        self.h, self.w = int(height), int(width)
        self.alpha, self.depth_tol, self.cos_tol = alpha, depth_tol, cos_tol
        self.acc = torch.zeros(2, dtype=torch.float64, device=dev)
        self.pairs = 0
        self._ws = torch.empty(_lib.nsm_temporal_workspace_bytes(self.h, self.w), dtype=torch.uint8,
                               device=dev)

    def reset(self):
        self.acc.zero_()
        self.pairs = 0

    def add(self, fr_prev, fr_cur, gbuf_prev, gbuf_cur, vis_prev, vis_cur, d_out=None, stream=None):
        """Adds one consecutive pair; d_out ([H, W] float32) receives D or a
        negative rejection code per pixel."""
        _lib.nsm_temporal_instability(self.tris, self.normals, self.n_tris, fr_prev, fr_cur, gbuf_prev,
                                      gbuf_cur, vis_prev.contiguous(), vis_cur.contiguous(), self.h, self.w,
                                      self.alpha, self.depth_tol, self.cos_tol, 1, self.acc, d_out,
                                      self._ws, self._ws.numel(), stream)
        self.pairs += 1

    def value(self):
        """E = sum / (W H (T - 1)) and the number of contributing pixels."""
        s, k = self.acc.tolist()
        return s / (self.w * self.h * max(self.pairs, 1)), int(k)


def save_checkpoint(path, weights, optimizer=None):
    """Writes the flat float32 weight vector to ``path + ".npy"`` and, if
    given, the torch optimizer's state to ``path + ".opt.pt"``."""
    np.save(path + ".npy", weights.detach().to(torch.float32).cpu().numpy())
    if optimizer is not None:
        torch.save(optimizer.state_dict(), path + ".opt.pt")


def load_checkpoint(path, device=None):
    """-> (flat float32 weights on `device`, the optimizer state or None).
    Both files are read without executing anything from them."""
    w = torch.from_numpy(np.load(path + ".npy", allow_pickle=False)).to(_dev(device))
    opt = path + ".opt.pt"
    state = torch.load(opt, map_location=_dev(device), weights_only=True) if os.path.exists(opt) else None
    return w, state
