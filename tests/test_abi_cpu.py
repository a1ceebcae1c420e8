"""C-ABI contract checks that need no GPU.

The library must load, export every function ``include/nsm.h`` declares, and
reject bad arguments with the documented status before touching the device.
"""
import ctypes
import os
import re

import pytest

import paper_2301_05262_amd as nsm
from paper_2301_05262_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "nsm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nsm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTS) == names


def test_abi_version_and_status_strings(lib):
    assert nsm.nsm_abi_version() == 3
    for s in range(8):
        assert nsm.nsm_status_str(s) != "unknown status"
    assert nsm.nsm_status_str(99) == "unknown status"


def test_struct_layouts_match_header():
    # nsm_net_desc: 11 int32; nsm_frame_params: 16+3+1+3+1 + 16+3+3+3+3+4 scalars of 4 bytes
    assert ctypes.sizeof(_lib.NetDesc) == 44
    assert ctypes.sizeof(_lib.FrameParams) == 4 * (16 + 3 + 1 + 3 + 1 + 16 + 3 + 3 + 3 + 3 + 4)


def test_create_validation_and_param_counts():
    ctx = nsm.nsm_create(6, (16, 32, 64), "f32")
    try:
        assert nsm.nsm_param_count(ctx) == 58641
        assert nsm.nsm_workspace_bytes(ctx, 1, 1080, 1920) > 0
        with pytest.raises(nsm.NsmError) as e:
            nsm.nsm_workspace_bytes(ctx, 1, 1082, 1920)      # not divisible by 4
        assert e.value.status == 2
        with pytest.raises(nsm.NsmError) as e:
            nsm.nsm_workspace_bytes(ctx, 0, 64, 64)
        assert e.value.status == 2
        # forward before set_weights: NSM_E_NO_WEIGHTS, before any device call
        with pytest.raises(nsm.NsmError) as e:
            nsm.nsm_forward(ctx, 1024, 1, 64, 64, 2048, None, 4096, 1 << 30, 0)
        assert e.value.status == 5
        with pytest.raises(nsm.NsmError) as e:
            nsm.nsm_forward(ctx, None, 1, 64, 64, 2048, None, 4096, 1 << 30, 0)
        assert e.value.status == 1
        with pytest.raises(nsm.NsmError) as e:
            nsm.nsm_set_weights(ctx, 1024, 17, 0)              # wrong count
        assert e.value.status == 1
    finally:
        nsm.nsm_destroy(ctx)
    ctx = nsm.nsm_create(6, (16, 32, 64), "f32")
    assert nsm.nsm_workspace_bytes(ctx, 2, 64, 64, training=1) > nsm.nsm_workspace_bytes(ctx, 2, 64, 64)
    with pytest.raises(nsm.NsmError) as e:        # backward before set_weights
        nsm.nsm_backward(ctx, 1024, 2048, 1, 64, 64, 4096, 0, None, 8192, 1 << 30, 0)
    assert e.value.status == 5
    nsm.nsm_destroy(ctx)
    ctx = nsm.nsm_create(6, (8, 16), "bf16")
    assert nsm.nsm_param_count(ctx) == 3353
    with pytest.raises(nsm.NsmError) as e:        # the differentiation form is float32 only
        nsm.nsm_workspace_bytes(ctx, 1, 64, 64, training=1)
    assert e.value.status == 3
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_backward(ctx, 1024, 2048, 1, 64, 64, 4096, 0, None, 8192, 1 << 30, 0)
    assert e.value.status == 3
    nsm.nsm_destroy(ctx)
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_create(6, (16, 32, 48), "f32")                  # no kernels for this width set
    assert e.value.status == 3
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_create(6, (16, 32, 64), 7)
    assert e.value.status == 1
    # the paper's network: 3x3 + 1x1 per level; parameter counts of the 3- and 5-level plans
    ctx = nsm.nsm_create(4, (16, 32, 64, 128, 256), "bf16", "paper")
    assert nsm.nsm_param_count(ctx) == 653648 + 1 + sum(
        [16, 16, 32, 32, 64, 64, 128, 128, 256, 128, 128, 64, 64, 32, 32, 16, 16, 16])
    with pytest.raises(nsm.NsmError) as e:                # 5 levels: H, W divisible by 16
        nsm.nsm_workspace_bytes(ctx, 1, 1032, 2048)
    assert e.value.status == 2
    with pytest.raises(nsm.NsmError) as e:                # no backward for this architecture
        nsm.nsm_workspace_bytes(ctx, 1, 1024, 2048, training=1)
    assert e.value.status == 3
    nsm.nsm_destroy(ctx)
    ctx = nsm.nsm_create(4, (16, 32, 64), "f32", "paper")
    assert nsm.nsm_param_count(ctx) == 39248 + 1 + sum([16, 16, 32, 32, 64, 32, 32, 16, 16, 16])
    nsm.nsm_destroy(ctx)
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_create(4, (16, 32, 64, 128), "f32", "paper")  # 4 levels: no kernels
    assert e.value.status == 3


def test_features_validation():
    import nsm_synth as S
    sc, fr = S.workload_frame("tiny_64", 0)
    need = nsm.nsm_features_workspace_bytes(sc.n_tris, 64, 64, 128)
    assert need >= 64 * 64 * 8
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_features_workspace_bytes(10, 0, 64, 128)
    assert e.value.status == 2
    fp = _lib.frame_params(fr)
    args = dict(tris=1024, tri_normals=2048, n_tris=sc.n_tris, fp=fp, h=64, w=64, fs="hard6",
                gbuf_in=None, gbuf_out=None, sm_out=4096, feat_out=8192, mask_out=None,
                workspace=16384, ws_bytes=need, stream=0)
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_build_features(**{**args, "ws_bytes": need - 1})
    assert e.value.status == 4
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_build_features(**{**args, "feat_out": None})
    assert e.value.status == 1
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_build_features(**{**args, "fs": 5})
    assert e.value.status == 1


def test_stored_feature_calls_validation():
    import nsm_synth as S
    sc, fr = S.workload_frame("tiny_64", 0)
    need = nsm.nsm_features_workspace_bytes(sc.n_tris, 64, 64, 128)
    args = dict(tris=1024, tri_normals=2048, n_tris=sc.n_tris, fp=_lib.frame_params(fr), h=64, w=64,
                fs="hard6", gbuf_in=None, gbuf_out=None, sm_out=4096, feat_dtype="bf16", feat_out=8192,
                mask_out=None, workspace=16384, ws_bytes=need, stream=0)
    for bad, status in ((dict(feat_dtype="f32"), 1), (dict(feat_dtype="f8"), 1), (dict(fs="paper4"), 3),
                        (dict(feat_out=None), 1), (dict(ws_bytes=need - 1), 4)):
        with pytest.raises(nsm.NsmError) as e:
            nsm.nsm_build_features_stored(**{**args, **bad})
        assert e.value.status == status, bad
    # stored input: BF16 / FP16 U-Net contexts only (checked before any device call)
    for c_in, widths, dt, arch in ((6, (16, 32, 64), "f32", "unet"), (6, (16, 32, 64), "f8", "unet"),
                                   (4, (16, 32, 64, 128, 256), "bf16", "paper")):
        ctx = nsm.nsm_create(c_in, widths, dt, arch)
        try:
            with pytest.raises(nsm.NsmError) as e:
                nsm.nsm_forward_stored(ctx, 1024, 1, 64, 64, 2048, None, 4096, 1 << 30, 0)
            assert e.value.status == 3, (dt, arch)
            with pytest.raises(nsm.NsmError) as e:
                nsm.nsm_autotune_stored(ctx, 1024, 1, 64, 64, 2048, 4096, 1 << 30, 1, 0)
            assert e.value.status == 3, (dt, arch)
        finally:
            nsm.nsm_destroy(ctx)
    ctx = nsm.nsm_create(6, (16, 32, 64), "bf16")
    try:
        with pytest.raises(nsm.NsmError) as e:      # no weights yet
            nsm.nsm_forward_stored(ctx, 1024, 1, 64, 64, 2048, None, 4096, 1 << 30, 0)
        assert e.value.status == 5
        with pytest.raises(nsm.NsmError) as e:
            nsm.nsm_forward_stored(ctx, None, 1, 64, 64, 2048, None, 4096, 1 << 30, 0)
        assert e.value.status == 1
    finally:
        nsm.nsm_destroy(ctx)


def test_s2d_network_plan():
    from oracle import paper_net as pn
    for widths in ((16, 32, 64), (16, 32, 64, 128, 256)):
        ctx = nsm.nsm_create(4, widths, "bf16", "paper_s2d")
        assert nsm.nsm_param_count(ctx) == pn.n_params(4, widths, s2d=True)
        with pytest.raises(nsm.NsmError) as e:
            m = 1 << (len(widths) - 1)            # sizes must be multiples of 2^(L-1)
            nsm.nsm_workspace_bytes(ctx, 1, 3 * m + 2, 4 * m, training=0)
        assert e.value.status == 2
        nsm.nsm_destroy(ctx)


def test_temporal_validation():
    import nsm_synth as S
    need = nsm.nsm_perturbation_loss_workspace_bytes(2, 3, 64, 96)
    assert need >= 8 * ((2 * 64 * 96 + 255) // 256)
    for bad in ((0, 3, 64, 96), (2, 17, 64, 96), (2, -1, 64, 96), (2, 3, 0, 96), (2, 3, 64, 16385)):
        with pytest.raises(nsm.NsmError) as e:
            nsm.nsm_perturbation_loss_workspace_bytes(*bad)
        assert e.value.status == 2
    args = dict(vis=1024, target=2048, n=2, p=3, h=64, w=96, alpha=0.9, loss_out=4096, dvis0_out=8192,
                workspace=16384, ws_bytes=need, stream=0)
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_perturbation_loss(**{**args, "ws_bytes": need - 1})
    assert e.value.status == 4
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_perturbation_loss(**{**args, "dvis0_out": None})
    assert e.value.status == 1
    sc, fr = S.workload_frame("tiny_64", 0)
    tneed = nsm.nsm_temporal_workspace_bytes(64, 64)
    assert tneed >= 16 * (64 * 64 // 256)
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_temporal_workspace_bytes(64, 0)
    assert e.value.status == 2
    targs = dict(tris=1024, tri_normals=2048, n_tris=sc.n_tris, fp_prev=fr, fp_cur=fr, gbuf_prev=4096,
                 gbuf_cur=8192, vis_prev=12288, vis_cur=16384, h=64, w=64, alpha=3.0, depth_tol=0.01,
                 cos_tol=0.9, accumulate=1, acc_out=20480, d_out=None, workspace=24576, ws_bytes=tneed,
                 stream=0)
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_temporal_instability(**{**targs, "ws_bytes": tneed - 1})
    assert e.value.status == 4
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_temporal_instability(**{**targs, "acc_out": None})
    assert e.value.status == 1
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_temporal_instability(**{**targs, "h": 16385})
    assert e.value.status == 2


def test_triangle_count_cap():
    """Triangle counts above 2^28 are rejected before any device call (the
    rasteriser carries two passes of triangle indices in 32-bit ints)."""
    import nsm_synth as S
    assert nsm.nsm_features_workspace_bytes(1 << 28, 64, 64, 128) > 0
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_features_workspace_bytes((1 << 28) + 1, 64, 64, 128)
    assert e.value.status == 2
    sc, fr = S.workload_frame("tiny_64", 0)
    fp = _lib.frame_params(fr)
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_build_features(1024, 2048, (1 << 28) + 1, fp, 64, 64, "hard6", None, None, 4096, 8192,
                               None, 16384, 1 << 40, 0)
    assert e.value.status == 2
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_temporal_instability(1024, 2048, (1 << 28) + 1, fr, fr, 4096, 8192, 12288, 16384, 64, 64,
                                     3.0, 0.01, 0.9, 1, 20480, None, 24576, 1 << 30, 0)
    assert e.value.status == 2


def test_noalloc_loss_validation():
    """The allocation-free perturbation loss checks its arguments like the
    workspace form and rejects more than 2^26 pixels (its scratch limit)
    before any device call."""
    args = dict(vis=1024, target=2048, n=2, p=3, h=64, w=96, alpha=0.9, loss_out=4096, dvis0_out=8192,
                stream=0)
    with pytest.raises(nsm.NsmError) as e:
        nsm.nsm_perturbation_loss_noalloc(**{**args, "vis": None})
    assert e.value.status == 1
    for bad in (dict(n=0), dict(p=17), dict(h=16385), dict(n=4096, h=128, w=129),
                dict(n=1, h=16384, w=4097)):
        with pytest.raises(nsm.NsmError) as e:
            nsm.nsm_perturbation_loss_noalloc(**{**args, **bad})
        assert e.value.status == 2, bad
