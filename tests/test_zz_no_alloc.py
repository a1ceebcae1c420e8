"""GPU check of the allocation-free perturbation loss
(nsm_perturbation_loss_noalloc): its scratch is a library-held device array
instead of a caller workspace, with the same kernels and reduction order, so
loss and gradient must equal the workspace entry point's bit for bit.  Two
calls in a row, the second smaller, so that stale partials of the first call
left in the shared array would show."""
import numpy as np
import pytest
import torch

import nsm_synth as S
from paper_2301_05262_amd import _lib

pytestmark = pytest.mark.gpu


def _inputs(n, p, h, w, seed):
    rng = S.SplitMix64(seed)
    vis = rng.uniforms(n * (1 + p) * h * w, 0.0, 1.0).astype(np.float32).reshape(n, 1 + p, h, w)
    # exact ties between x_0 and a perturbed output: sgn(0) = 0 must hold on both paths
    vis[:, 1, :4] = vis[:, 0, :4]
    tgt = rng.uniforms(n * h * w, 0.0, 1.0).astype(np.float32).reshape(n, h, w)
    return torch.from_numpy(vis).cuda(), torch.from_numpy(tgt).cuda()


def _workspace_form(vis, tgt, n, p, h, w):
    need = _lib.nsm_perturbation_loss_workspace_bytes(n, p, h, w)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    d = torch.empty((n, h, w), dtype=torch.float32, device="cuda")
    _lib.nsm_perturbation_loss(vis, tgt, n, p, h, w, 0.9, loss, d, ws, need)
    return loss, d


def _noalloc_form(vis, tgt, n, p, h, w):
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    d = torch.empty((n, h, w), dtype=torch.float32, device="cuda")
    _lib.nsm_perturbation_loss_noalloc(vis, tgt, n, p, h, w, 0.9, loss, d)
    return loss, d


def test_noalloc_matches_workspace_entry_point():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    for (n, p, h, w), seed in (((3, 3, 96, 160), 5), ((1, 2, 40, 72), 6)):
        print(f"[noalloc] n={n} p={p} h={h} w={w} seed={seed}", flush=True)
        vis, tgt = _inputs(n, p, h, w, seed)
        l0, d0 = _workspace_form(vis, tgt, n, p, h, w)
        l1, d1 = _noalloc_form(vis, tgt, n, p, h, w)
        torch.cuda.synchronize()
        assert l1.cpu().numpy().view(np.uint64)[0] == l0.cpu().numpy().view(np.uint64)[0]
        assert np.array_equal(d1.cpu().numpy().view(np.uint32), d0.cpu().numpy().view(np.uint32))
        # and the value itself: the mean L1 of Eq. 2 in float64, alpha as the float32 the call takes
        v = vis.cpu().numpy().astype(np.float64)
        want = float(np.float32(0.9)) * (np.abs(v[:, 0] - tgt.cpu().numpy()).sum()
                      + np.abs(v[:, :1] - v[:, 1:]).sum()) / (n * h * w)
        assert abs(float(l1.item()) - want) <= 1e-12 * max(1.0, abs(want))
