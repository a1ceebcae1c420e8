"""Checkpoint round trip on the host: the flat weights come back bit for bit
from their .npy file, the optimizer state (step counts and moment tensors)
through torch's tensor-only loader, and an Adam step from the restored state
equals the step of the optimizer that wrote it."""
import numpy as np
import torch

import nsm_synth as S
from paper_2301_05262_amd.api import load_checkpoint, save_checkpoint


def test_weights_and_adam_state_round_trip(tmp_path):
    flat = torch.from_numpy(S.he_weights(S.U3_SOFT, 5))
    w = torch.nn.Parameter(flat.clone())
    opt = torch.optim.Adam([w], lr=1e-3)
    rng = S.SplitMix64(3)
    grads = [torch.from_numpy(rng.uniforms(flat.numel(), -1, 1).astype(np.float32)) for _ in range(3)]
    for g in grads[:2]:
        w.grad = g.clone()
        opt.step()
    path = str(tmp_path / "ck")
    save_checkpoint(path, w, opt)
    w2, state = load_checkpoint(path, device="cpu")
    assert w2.dtype == torch.float32 and torch.equal(w2, w.detach())
    p2 = torch.nn.Parameter(w2)
    opt2 = torch.optim.Adam([p2], lr=1e-3)
    opt2.load_state_dict(state)
    for p, o in ((w, opt), (p2, opt2)):
        p.grad = grads[2].clone()
        o.step()
    assert torch.equal(w.detach(), p2.detach())


def test_weights_only_checkpoint(tmp_path):
    flat = torch.from_numpy(S.he_weights(S.U2, 1))
    path = str(tmp_path / "w")
    save_checkpoint(path, flat)
    w, state = load_checkpoint(path, device="cpu")
    assert state is None and torch.equal(w, flat)
