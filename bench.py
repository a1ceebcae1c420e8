"""Benchmark: ms/frame of 1080p neural shadow-map inference on one MI355X.

One step = the whole inference path for one 1920x1080 frame of the
19,632-triangle synthetic scene with a 2048^2 shadow map: light-view
z-buffer, camera G-buffer, feature gather (HARD6) and the U-Net forward
(U3: widths 16/32/64).  `value` is the BF16 form's ms/frame for that whole
step; the network alone (nsm_forward, the paper's convention, which leaves
out the G-buffer) is `network_ms` beside it.  The FP32, FP16 and 8-bit
storage forms are timed the same way and reported beside it, each with its
visibility error against the FP64 oracle.

Rooflines: `roofline` is the dominant kernel of the BF16 step;
`roofline_classes` gives each layer class's fraction (raster + gather and
the BF16 thin convs against HBM, BF16 D1 against the BF16 MFMA peak, the
FP32 convs against the FP32 MFMA peak), each from algorithmic bytes or
FLOPs over the summed kernel times of the class.

Timing: W untimed warm-up steps, then K steps bracketed by
torch.cuda.synchronize() with events on the launch stream (the library
launches on torch's current stream).  A second, traced pass over K steps
records HIP events around every kernel (on its launch stream) to get
per-kernel durations for the roofline; the untraced pass gives `value`.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-sample frame|none]
"""
import argparse
import json
import os
import sys
import gc
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms/frame 1080p shadow-net inference, BF16 vs FP32, at stated visibility error"
HBM_PEAK = 8.0e12                         # B/s
MFMA_PEAK = {"f32": 157.3e12, "bf16": 2.5e15, "f16": 2.5e15,
             "f8": 2.5e15,    # dense FLOP/s; the 8-bit storage form computes on bf16 MFMA
             "f8mfma": 5.0e15}
WORKLOAD = "hard_1080p"
CALIB_COPY_BYTES = 256 << 20
TRAFFIC_MD = os.path.join(ROOT, "profiles", "hbm_traffic_1080p_bf16.md")

# traced kernel name (BF16 form) -> kernel symbol as the counter summary names it
KERNEL_SYMBOL = {
    "raster light+camera": "k_raster",
    "gather hard6": "k_gather<0, 0>",
    "gather hard6 stored": "k_gather<0, 1>",
}
# BF16 stages: (traced name, stage index in network order, kernel with the
# default tile rows, kernel with the alternative ones); launch variant bit 0
# selects the persistent form, bit 1 the alternative rows.  The first stage
# reads float32 features, or (stored) features already in bfloat16.
STAGE_SYMBOLS = [
    ("conv3x3 6+0->16 Pool bf16", 0, "k_conv3x3<bf16, true, 6, 0, 16, Pool, 8>",
     "k_conv3x3<bf16, true, 6, 0, 16, Pool, 16>"),
    ("conv3x3 6+0->16 Pool stored bf16", 0, "k_conv3x3<bf16, false, 6, 0, 16, Pool, 8>",
     "k_conv3x3<bf16, false, 6, 0, 16, Pool, 16>"),
    ("conv3x3 16+0->32 Pool bf16", 1, "k_conv3x3<bf16, false, 16, 0, 32, Pool, 8>",
     "k_conv3x3<bf16, false, 16, 0, 32, Pool, 16>"),
    ("conv3x3 32+0->64 Store bf16", 2, "k_conv3x3<bf16, false, 32, 0, 64, Store, 8>",
     "k_conv3x3<bf16, false, 32, 0, 64, Store, 4>"),
    ("conv3x3 32+64->32 Store phase bf16", 3, "k_conv3x3_up<bf16, 32, 64, 32, Store, 8, 4>",
     "k_conv3x3_up<bf16, 32, 64, 32, Store, 8, 4>"),
    ("conv3x3 16+32->16 Head phase bf16", 4, "k_conv3x3_up<bf16, 16, 32, 16, Head, 16, 4>",
     "k_conv3x3_up<bf16, 16, 32, 16, Head, 16, 8>"),
]
# forms whose step hands the features over in the network's storage type
STORED_FORMS = ("bf16", "f16", "f8mfma")


def kernel_symbol(name, variants):
    """Profiled kernel behind a traced BF16 launch, in the launch variants used."""
    if name in KERNEL_SYMBOL:
        return KERNEL_SYMBOL[name]
    for traced, i, sym, alt in STAGE_SYMBOLS:
        if traced == name:
            v = variants[i] if variants and i < len(variants) else 0
            sym = alt if v & 2 else sym
            if v & 1:
                sym = sym.replace("k_conv3x3_up<", "k_conv3x3_up_persist<").replace("k_conv3x3<", "k_conv3x3_persist<")
            return sym
    return ""


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-sample", default="frame", choices=["frame", "none"])
    ap.add_argument("--forms", default="bf16,f32,f16,f8,f8mfma")
    ap.add_argument("--batched", type=int, default=1, help="also time the 16-frame graph batch")
    ap.add_argument("--paper-net", type=int, default=1, help="also time the paper's 5-level net")
    ap.add_argument("--training", type=int, default=1, help="also time the 32-frame FP32 training step")
    ap.add_argument("--temporal", type=int, default=1,
                    help="also time the perturbation-loss training step and the temporal metric")
    ap.add_argument("--f4", type=int, default=1,
                    help="also run the penumbra-width level analysis and Eq. 1 on the training frames")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="end with one plain 256 MiB device copy (the scale for HBM byte counters)")
    return ap.parse_args()


def stage_costs(widths, c_in, h, w, dtype):
    """Algorithmic FLOPs and HBM bytes per frame of each conv stage (fused:
    every tensor written once and read once per consumer; weights included).
    Activations take 4, 2 or (8-bit forms) 1 byte; weights 4, 2 or (FP8 compute) 1."""
    es = {"f32": 4, "f8": 1, "f8mfma": 1}.get(dtype, 2)
    ws = {"f32": 4, "f8mfma": 1}.get(dtype, 2)
    w0, w1, w2 = widths
    L1, L2 = (h // 2) * (w // 2), (h // 4) * (w // 4)
    L0 = h * w
    out = {}

    def add(key, px, cs, cu, co, in_bytes, out_bytes):
        flops = 2.0 * px * co * 9 * (cs + cu)
        wbytes = co * 9 * (cs + cu) * ws + co * 4
        out[key] = (flops, in_bytes + out_bytes + wbytes)

    add(f"conv3x3 {c_in}+0->{w0} Pool", L0, c_in, 0, w0, L0 * c_in * 4, L0 * w0 * es + L1 * w0 * es)
    # the same stage on features stored in the storage type, whole 16-byte blocks per pixel
    add(f"conv3x3 {c_in}+0->{w0} Pool stored", L0, c_in, 0, w0, L0 * 16, L0 * w0 * es + L1 * w0 * es)
    add(f"conv3x3 {w0}+0->{w1} Pool", L1, w0, 0, w1, L1 * w0 * es, L1 * w1 * es + L2 * w1 * es)
    add(f"conv3x3 {w1}+0->{w2} Store", L2, w1, 0, w2, L2 * w1 * es, L2 * w2 * es)
    add(f"conv3x3 {w1}+{w2}->{w1} Store", L1, w1, w2, w1, L1 * w1 * es + L2 * w2 * es, L1 * w1 * es)
    add(f"conv3x3 {w0}+{w1}->{w0} Head", L0, w0, w1, w0, L0 * w0 * es + L1 * w1 * es, L0 * 4)
    k = f"conv3x3 {w0}+{w1}->{w0} Head"
    fl, by = out[k]
    out[k] = (fl + 2.0 * L0 * w0, by)          # the fused 1x1 head
    # decoder stages at these sizes run as one launch (interior tiles in the
    # phase form, border bands in the general form)
    for key in (f"conv3x3 {w1}+{w2}->{w1} Store", f"conv3x3 {w0}+{w1}->{w0} Head"):
        out[key + " phase"] = out[key]
    return out


def _base(name):
    """Traced kernel name without its trailing storage-type suffix."""
    head, _, last = name.rpartition(" ")
    return head if last in ("bf16", "f16", "f32", "f8", "f8mfma") else name


def raster_costs(n_tris, h, w, sm):
    """Algorithmic HBM bytes of the fused light + camera z-buffer: each target
    written once (u32 shadow map, u64 camera keys) and the triangles' 36-byte
    vertex triples read once per pass."""
    return {"raster light+camera": (0.0, float(sm * sm * 4 + h * w * 8 + 2 * n_tris * 36))}


def gather_costs(n_tris, h, w, channels, name):
    """Algorithmic HBM bytes of the feature gather: per pixel the 8-byte camera
    key, the 4-byte map texel, the float32 channels (16 bytes when stored in
    a 2-byte type) and the mask byte; per triangle its vertices and normal
    (48 bytes), read once."""
    return {name: (0.0, float(h * w * (8 + 4 + 4 * channels + 1) + n_tris * 48)),
            name + " stored": (0.0, float(h * w * (8 + 4 + 16 + 1) + n_tris * 48))}


def class_rooflines(results, costs_of, forms):
    """Fraction of the relevant peak per layer class, from algorithmic work over
    the summed per-kernel times of the class (one frame per launch)."""
    out = {}

    def frac(form, keys, kind, peak):
        ks = results[form]["kernels"]
        c = costs_of(form)
        t = sum(ks[k]["avg_us"] for k in keys if k in ks) * 1e-6
        work = sum(c[_base(k)][0 if kind == "flops" else 1] for k in keys if k in ks and _base(k) in c)
        if t <= 0:
            return None
        unit = "TFLOP/s" if kind == "flops" else "GB/s"
        achieved = work / t / (1e12 if kind == "flops" else 1e9)
        return {"kernels": [k for k in keys if k in ks], "us": t * 1e6, "achieved": achieved,
                "peak": peak / (1e12 if kind == "flops" else 1e9), "unit": unit, "frac": work / t / peak}

    for form in forms:
        ks = list(results[form]["kernels"])
        feat = [k for k in ks if k.split(" ")[0] in ("setup+clear", "tile_scan", "raster", "gather")]
        convs = [k for k in ks if k.startswith("conv3x3")]
        d1 = [k for k in convs if "+64->32" in k]
        thin = [k for k in convs if k not in d1]
        if form == forms[0]:
            out["raster+gather (hbm)"] = frac(form, feat, "bytes", HBM_PEAK)
        if form == "f32":
            out["fp32 convs (fp32 mfma)"] = frac(form, convs, "flops", MFMA_PEAK["f32"])
        elif form in ("bf16", "f16", "f8", "f8mfma"):
            out[f"{form} thin convs E0,E1,B,D0 (hbm)"] = frac(form, thin, "bytes", HBM_PEAK)
            out[f"{form} D1 (mfma)"] = frac(form, d1, "flops", MFMA_PEAK[form])
    return out


def batched_section(S, torch, seed, reps):
    """16 mixed-size frames (1280x720 / 1920x1080 / 2560x1440, 20k-100k triangles,
    hard and soft lights): features + SOFT8 BF16 network per size group, one
    graph per group with the launch variants autotuned for its shape, replayed
    in order.  Per-frame latency is the completion time of the frame's group
    since the batch started.  Beside it: the same graphs with the default
    variants, and one-by-one launches (features + network per frame) in BF16
    and in FP32.  BF16 runs take their features in bfloat16
    (nsm_build_features_stored), FP32 runs in float32."""
    from paper_2301_05262_amd.api import ShadowNet
    from paper_2301_05262_amd.batch import BatchedPipeline
    frames = S.make_batched_frames(seed, 16)
    flat = torch.from_numpy(S.he_weights(S.U3_SOFT, seed))
    out = {"workload": "batched_mixed", "frames": len(frames),
           "megapixels": sum(fr.width * fr.height for _, fr in frames) / 1e6,
           "tris": [sc.n_tris for sc, _ in frames]}
    for label, tune in (("graph_bf16_default", False), ("graph_bf16_tuned", True)):
        pipe = BatchedPipeline(frames, 8, S.U3_SOFT.widths, flat, "bf16")
        pipe.capture(tune=tune)
        for _ in range(3):
            pipe.replay()
        batch_ms, frame_ms = [], []
        for _ in range(reps):
            b, done = pipe.replay_timed()
            batch_ms.append(b)
            frame_ms += done
        bm, fm = np.array(batch_ms), np.array(frame_ms)
        out[label] = {"ms_per_batch_p50": float(np.median(bm)), "ms_per_batch_p99": float(np.quantile(bm, 0.99)),
                      "frames_per_s": len(frames) / (float(bm.mean()) / 1e3),
                      "frame_latency_ms_p50": float(np.median(fm)), "frame_latency_ms_p99": float(np.quantile(fm, 0.99)),
                      "variants_per_group": {f"{g['hw'][1]}x{g['hw'][0]}": g["variants"] for g in pipe.groups}}
    ev = lambda: torch.cuda.Event(enable_timing=True)
    for dt in ("bf16", "f32"):
        net = ShadowNet(8, S.U3_SOFT.widths, dt)
        net.set_weights(flat)
        st = "bf16" if dt == "bf16" else None
        slots = []
        for g in pipe.groups:
            for k, i in enumerate(g["idx"]):
                buf = g["bufs"][k] if st else dict(g["bufs"][k], feat=torch.empty(
                    g["feat"][k].shape, dtype=torch.float32, device=g["feat"].device))
                slots.append((i, buf, buf["feat"].unsqueeze(0), torch.empty_like(g["vis"][k:k + 1])))
        for i, buf, f, v in slots:                       # warm-up (workspaces)
            pipe.builders[i](frames[i][1], soft=True, out=buf, stored=st)
            net.forward(f, vis_out=v)
        torch.cuda.synchronize()
        frame_ms = []
        for _ in range(max(1, reps // 4)):
            for i, buf, f, v in slots:
                a, b = ev(), ev()
                a.record()
                pipe.builders[i](frames[i][1], soft=True, out=buf, stored=st)
                net.forward(f, vis_out=v)
                b.record()
                b.synchronize()
                frame_ms.append(a.elapsed_time(b))
        fm = np.array(frame_ms)
        out[f"one_by_one_{dt}"] = {"ms_per_frame_p50": float(np.median(fm)),
                                   "ms_per_frame_p99": float(np.quantile(fm, 0.99)),
                                   "frames_per_s": 1e3 / float(fm.mean())}
    return out


def training_section(S, torch, seed, steps):
    """One training step of the soft-shadow net (FP32, the differentiation
    form) on 8 windows x 4 frames of 512x512: SOFT8 features of all 32 frames,
    forward keeping its activations, MSE loss gradient, backward from those
    activations (dW and dfeatures).  Targets are fixed synthetic visibilities in [0, 1] (the
    64-sample ray-cast targets are data generation, not part of a step)."""
    from paper_2301_05262_amd.api import FeatureBuilder, ShadowNet
    wins = [S.make_train_window(seed, k) for k in range(8)]
    builders = [FeatureBuilder(sc) for sc, _ in wins]
    frames = [(b, fr) for b, (_, frs) in zip(builders, wins) for fr in frs]
    n = len(frames)
    feat = torch.empty((n, 512, 512, 8), dtype=torch.float32, device="cuda")
    bufs = [b(fr, soft=True) for b, fr in frames]
    for k in range(n):
        bufs[k]["feat"] = feat[k]          # each frame's features land in the batch directly
    rng = S.SplitMix64(seed + 7)
    target = torch.from_numpy(rng.uniforms(n * 512 * 512, 0.0, 1.0).reshape(n, 512, 512).astype(np.float32)).cuda()
    net = ShadowNet(8, S.U3_SOFT.widths, "f32")
    net.set_weights(torch.from_numpy(S.he_weights(S.U3_SOFT, seed)))
    dw = torch.empty(net.n_params, dtype=torch.float32, device="cuda")

    # the windows' feature builds are independent (one builder, so one
    # workspace, per window): they run on side streams, a window's frames in
    # order on one stream, and the forward waits for all of them
    side = [torch.cuda.Stream() for _ in range(4)]
    win_of = [k // 4 for k in range(n)]

    def step():
        main = torch.cuda.current_stream()
        start = main.record_event()
        for s in side:
            s.wait_event(start)
        for k, (b, fr) in enumerate(frames):
            b(fr, soft=True, out=bufs[k], stream=side[win_of[k] % len(side)])
        for s in side:
            main.wait_event(s.record_event())
        vis = net.forward_train(feat)
        dvis = (2.0 / vis.numel()) * (vis - target)
        net.backward(feat, dvis, dw_out=dw, saved=True)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    w0, w1, w2 = S.U3_SOFT.widths
    L0, L1, L2 = 512 * 512, 256 * 256, 128 * 128
    macs = 9 * (L0 * w0 * 8 + L1 * w1 * w0 + L2 * w2 * w1 + L1 * w1 * (w1 + w2) + L0 * w0 * (w0 + w1)) + L0 * w0
    flop = 2.0 * macs * n * 3        # forward + two backward GEMMs per conv
    return {"workload": "soft_train_512", "frames": n, "ms_per_step": ms, "dtype": "f32",
            "tflops_effective": flop / (ms * 1e-3) / 1e12, "flop_per_step": flop,
            "ideal_ms_at_fp32_mfma_peak": flop / MFMA_PEAK["f32"] * 1e3}


def temporal_section(S, torch, seed, steps):
    """The temporal-stability parts (Sec. 3.3-3.4).

    perturb_train: one training step with the perturbation loss of Eq. 2 on
    8 samples of 512x512: SOFT8 features of each sample's frame and of 3
    perturbed copies (32 frames), one FP32 forward over all 32, the loss and
    its gradient, and the backward through the 8 unperturbed instances only.
    metric_1080p: one consecutive frame pair of Eq. 3 at 1920x1080 (reprojection,
    depth / normal rejection, float64 sum)."""
    import paper_2301_05262_amd as nsm
    from paper_2301_05262_amd.api import FeatureBuilder, ShadowNet, TemporalMetric, perturbation_loss
    wins = [S.make_train_window(seed, k, frames=1) for k in range(8)]
    jobs = []
    for k, (sc, frs) in enumerate(wins):
        b = FeatureBuilder(sc)
        jobs += [(b, fr) for fr in [frs[0]] + [S.perturb_frame(sc, frs[0], 1000 * k + i) for i in range(3)]]
    feat = torch.empty((32, 512, 512, 8), dtype=torch.float32, device="cuda")
    bufs = [b(fr, soft=True) for b, fr in jobs]
    rng = S.SplitMix64(seed + 11)
    target = torch.from_numpy(rng.uniforms(8 * 512 * 512, 0.0, 1.0).reshape(8, 512, 512).astype(np.float32)).cuda()
    net = ShadowNet(8, S.U3_SOFT.widths, "f32")
    net.set_weights(torch.from_numpy(S.he_weights(S.U3_SOFT, seed)))
    dw = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    x0 = torch.empty((8, 512, 512, 8), dtype=torch.float32, device="cuda")

    def step():
        for k, (b, fr) in enumerate(jobs):
            b(fr, soft=True, out=bufs[k])
            feat[k].copy_(bufs[k]["feat"])
        vis = net.forward(feat).view(8, 4, 512, 512)
        _, dvis0 = perturbation_loss(vis, target)
        x0.copy_(feat.view(8, 4, 512, 512, 8)[:, 0])
        net.backward(x0, dvis0, dw_out=dw)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    torch.cuda.synchronize()
    train_ms = a.elapsed_time(b) / steps

    sc, frames = S.make_train_window(seed, 0, frames=2, width=1920, height=1080, sm_size=2048)
    fb = FeatureBuilder(sc)
    g0, g1 = fb(frames[0])["gbuf"].clone(), fb(frames[1])["gbuf"].clone()
    v0 = torch.from_numpy(rng.uniforms(1080 * 1920, 0, 1).reshape(1080, 1920).astype(np.float32)).cuda()
    v1 = torch.from_numpy(rng.uniforms(1080 * 1920, 0, 1).reshape(1080, 1920).astype(np.float32)).cuda()
    metric = TemporalMetric(sc, 1080, 1920)
    for _ in range(5):
        metric.add(frames[0], frames[1], g0, g1, v0, v1)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps * 4):
        metric.add(frames[0], frames[1], g0, g1, v0, v1)
    b.record()
    torch.cuda.synchronize()
    pair_ms = a.elapsed_time(b) / (steps * 4)
    nsm.nsm_trace_read()
    nsm.nsm_trace_enable(True)
    for _ in range(steps):
        metric.add(frames[0], frames[1], g0, g1, v0, v1)
    torch.cuda.synchronize()
    per = {}
    for name, ms in nsm.nsm_trace_read(1 << 16):
        per.setdefault(name, []).append(ms)
    nsm.nsm_trace_enable(False)
    return {"perturb_train": {"workload": "soft_perturb_train_512", "samples": 8, "perturbations": 3,
                              "forward_frames": 32, "backward_frames": 8, "ms_per_step": train_ms,
                              "dtype": "f32"},
            "metric_1080p": {"ms_per_pair": pair_ms,
                             "kernels_us": {k: 1e3 * float(np.mean(v)) for k, v in per.items()}}}


def f4_section(S, torch, seed):
    """Design-time analysis on the soft-shadow training set (8 windows x 4
    frames of 512^2, spherical lights r_e in [0.02, 0.2]): per-pixel
    penumbra widths from the rendered G-buffer and shadow map (Sec. 3.6,
    supplemental Sec. 4), their P95 and the level count the receptive-field
    rule picks, against the 3 levels the U-Net has; and Eq. 1's relative
    channel sensitivity of the (random-weight) SOFT8 U-Net on rendered
    features of one window."""
    from paper_2301_05262_amd.analysis import level_report, penumbra_widths, receptive_field, sensitivity
    from paper_2301_05262_amd.api import FeatureBuilder, ShadowNet
    t0 = time.perf_counter()
    maps, feats0 = [], []
    for k in range(8):
        sc, frames = S.make_train_window(seed, k)
        fb = FeatureBuilder(sc)
        tris, nrm = torch.from_numpy(sc.tris).cuda(), torch.from_numpy(sc.normals).cuda()
        for fr in frames:
            out = fb(fr, soft=True)
            maps.append(penumbra_widths(out["gbuf"], out["sm"], tris, nrm, fr)[0].cpu().numpy())
            if k == 0:
                feats0.append(out["feat"].clone())
    rep = level_report(maps)
    rep["receptive_field_of_u3_px"] = receptive_field(3)
    rep["u3_covers_p95"] = rep["p95_width_px"] <= receptive_field(3)
    net = ShadowNet(8, S.U3_SOFT.widths, "f32")
    net.set_weights(torch.from_numpy(S.he_weights(S.U3_SOFT, seed)))
    _, rel = sensitivity(net.forward, torch.stack(feats0).contiguous(), repeats=2, seed=seed)
    names = ["d/f_C", "n.x", "n.y", "n.z", "(z-z_f)/f_L", "z/f_L", "r_e/0.2", "z_blk/f_L"]
    return {"workload": "soft_train_512 (8 windows x 4 frames)", "penumbra": rep,
            "sensitivity_rendered_soft8": dict(zip(names, [float(v) for v in rel])),
            "seconds": time.perf_counter() - t0}


def _time_net(torch, nsm, net, feat, vis, steps):
    """Average ms per forward over `steps` launches, then per-kernel us from the trace."""
    for _ in range(10):
        net.forward(feat, vis_out=vis)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        net.forward(feat, vis_out=vis)
    b.record()
    torch.cuda.synchronize()
    nsm.nsm_trace_read()
    nsm.nsm_trace_enable(True)
    for _ in range(max(1, steps // 4)):
        net.forward(feat, vis_out=vis)
    torch.cuda.synchronize()
    per = {}
    for name, ms in nsm.nsm_trace_read(1 << 16):
        per.setdefault(name, []).append(ms)
    nsm.nsm_trace_enable(False)
    return {"network_ms": a.elapsed_time(b) / steps,
            "kernels_us": {k: 1e3 * float(np.mean(v)) for k, v in per.items()}}


def paper_net_section(S, torch, seed, steps):
    """The paper's own 5-level network (3x3 + 1x1 per level, avg-pool, sum skip)
    at 1024x2048 on PAPER4 features, before ("paper") and after ("s2d") its
    first-level optimisation: network ms per form, per-kernel times."""
    import paper_2301_05262_amd as nsm
    from paper_2301_05262_amd.api import FeatureBuilder, ShadowNet
    widths = (16, 32, 64, 128, 256)
    sc = S.make_scene("objects60", seed)
    fr = S.make_frame(sc, 2048, 1024, 2048, light_pos=(0.4, 3.2, -0.3), eye=(3.2, 1.5, 0.3),
                      target=(0.0, -1.0, 0.0), light_radius=0.1)
    fb = FeatureBuilder(sc)
    buf = fb(fr, fs="paper4")
    feat = buf["feat"].unsqueeze(0)
    vis = torch.empty((1, 1024, 2048), dtype=torch.float32, device=feat.device)
    out = {"workload": "paper5_1024x2048", "widths": list(widths), "features": "paper4",
           "macs_per_pixel": 16208, "s2d": {"macs_per_pixel": 12816}}
    for arch, dst in (("paper", out), ("paper_s2d", out["s2d"])):
        rng = S.SplitMix64(seed)
        net0 = ShadowNet(4, widths, "f32", arch=arch)
        flat = torch.from_numpy((rng.normals(net0.n_params) * 0.1).astype(np.float32))
        for f in ("bf16", "f16", "f32"):
            net = ShadowNet(4, widths, f, arch=arch)
            net.set_weights(flat)
            dst[f] = _time_net(torch, nsm, net, feat, vis, steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        fb(fr, fs="paper4", out=buf)
    torch.cuda.synchronize()
    out["features_ms"] = 1e3 * (time.perf_counter() - t0) / steps
    out["paper_context"] = ("RTX 2080Ti, FP16: 17.3 ms for this network before the first-level "
                            "optimisation and 5.84 ms after it (Sec. 3.5), 28 ms FP32")
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, fr, desc, flat, band_rows=272, reps=3):
    """The CPU oracle per stage, median of `reps` runs, at all threads the
    process may use and at one thread: the C rasteriser (light map and camera
    keys) and the C gather on the whole frame, the float64 U-Net forward on a
    band of `band_rows` full-width rows of the frame's features, scaled to the
    frame by its pixel count (its cost is linear in pixels)."""
    import threadpoolctl

    import oracle
    from oracle import net as onet
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = min(threads, int(os.environ.get("OMP_NUM_THREADS", threads)))
    H, W = fr.height, fr.width

    def stages(nt):
        med = {}
        with threadpoolctl.threadpool_limits(nt):
            runs = []
            for _ in range(reps):
                t0 = time.perf_counter()
                sm, _ = oracle.raster(scene.tris, fr.m_light, fr.sm_size, fr.sm_size, "depth")
                t1 = time.perf_counter()
                gb, _ = oracle.raster(scene.tris, fr.m_cam, W, H, "key")
                t2 = time.perf_counter()
                ofe = oracle.gather(scene, fr, gb, sm)
                t3 = time.perf_counter()
                band = ofe["feat"][None, :band_rows]
                onet.forward(desc.c_in, desc.widths, flat, band, keep=False)
                t4 = time.perf_counter()
                runs.append((t1 - t0, t2 - t1, t3 - t2, (t4 - t3) * H / band_rows))
            r = np.median(np.array(runs), axis=0) * 1e3
            med = {"light_zbuffer_ms": r[0], "camera_gbuffer_ms": r[1], "gather_ms": r[2], "forward_ms": r[3]}
        med = {k: float(v) for k, v in med.items()}
        med["ms_per_frame"] = sum(med.values())
        ofe.update(sm=sm, gbuf=gb)
        return med, ofe

    many, ofe = stages(threads)
    one, _ = stages(1)
    return ({"value": many["ms_per_frame"], "unit": "ms/frame", "cores": threads, "kind": "oracle",
             "sample": (f"one 1920x1080 frame: C rasteriser (2048^2 light map + camera keys) and C gather "
                        f"on the whole frame, numpy float64 U-Net forward on a {band_rows}-row full-width "
                        f"band scaled by {H}/{band_rows}; median of {reps} runs per stage"),
             "stages": many, "one_thread": one, "cpu_model": _cpu_model(), "nproc": os.cpu_count()},
            ofe)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library has no "
              "multi-GPU mode; frames are independent, so a caller shards them over one process "
              "per GPU", file=sys.stderr)
        sys.exit(2)
    import torch

    import nsm_synth as S
    import paper_2301_05262_amd as nsm
    from paper_2301_05262_amd.api import FeatureBuilder, ShadowNet

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    scene, fr = S.workload_frame(WORKLOAD, args.seed)
    H, W = fr.height, fr.width
    desc = S.U3
    flat = S.he_weights(desc, args.seed)
    fb = FeatureBuilder(scene, dev)
    forms = [f for f in args.forms.split(",") if f]
    nets = {}
    for f in forms:
        nets[f] = ShadowNet(desc.c_in, desc.widths, f, dev)
        nets[f].set_weights(torch.from_numpy(flat))
    # BF16 and FP16 steps take the features in the storage type (the gather
    # rounds them, as the float32 path's first stage would); the others float32
    bufs = {f: fb(fr, stored=f if f in STORED_FORMS else None) for f in forms}
    feats = {f: bufs[f]["feat"].unsqueeze(0) for f in forms}
    vis = {f: torch.empty((1, H, W), dtype=torch.float32, device=dev) for f in forms}
    # launch variants timed once for this frame size, as a deployment would at start-up
    variants = {f: nets[f].autotune(feats[f], reps=20) for f in forms}
    torch.cuda.synchronize()

    def step(f):
        fb(fr, out=bufs[f], stored=f if f in STORED_FORMS else None)
        nets[f].forward(feats[f], vis_out=vis[f])

    def net_only(f):
        nets[f].forward(feats[f], vis_out=vis[f])

    def timed(fn, f, k):
        # the host only enqueues here; a garbage-collector pass over this
        # process's heap in the middle of the loop could leave the GPU idle
        gc.collect()
        gc.disable()
        try:
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            s.record()
            for _ in range(k):
                fn(f)
            e.record()
            torch.cuda.synchronize()
        finally:
            gc.enable()
        return s.elapsed_time(e) / k

    # Sustained load first: the autotune's short synchronised launches leave
    # the GPU below its steady-state clocks, which the first timed form would
    # otherwise absorb.  A renderer runs frames back to back.
    t_end = time.perf_counter() + 0.5
    while time.perf_counter() < t_end:
        for _ in range(50):
            step(forms[0])
        torch.cuda.synchronize()

    results = {}
    for f in forms:
        for _ in range(args.warmup):
            step(f)
        ms_step = timed(step, f, args.steps)
        ms_net = timed(net_only, f, args.steps)
        # traced pass: per-kernel durations
        nsm.nsm_trace_read()
        nsm.nsm_trace_enable(True)
        for _ in range(args.steps):
            step(f)
        torch.cuda.synchronize()
        recs = nsm.nsm_trace_read(1 << 16)
        nsm.nsm_trace_enable(False)
        per = {}
        for name, ms in recs:
            per.setdefault(name, []).append(ms)
        kern = {k: {"avg_us": 1e3 * float(np.mean(v)), "launches": len(v)} for k, v in per.items()}
        results[f] = {"ms_per_frame": ms_step, "network_ms": ms_net, "features_ms": ms_step - ms_net,
                      "launch_variants": variants[f], "kernels": kern}
        print(f"[bench] {f}: step {ms_step:.4f} ms  network {ms_net:.4f} ms", file=sys.stderr, flush=True)

    # visibility error of each form against the FP64 oracle (and the CPU baseline timing)
    cpu = None
    if args.cpu_sample == "frame":
        from oracle import net as onet
        cpu, ofe = cpu_baseline(scene, fr, desc, flat)
        print(f"[bench] cpu oracle: {cpu['value']:.0f} ms/frame at {cpu['cores']} threads, "
              f"{cpu['one_thread']['ms_per_frame']:.0f} ms/frame at 1", file=sys.stderr, flush=True)
        ref = onet.forward(desc.c_in, desc.widths, flat, ofe["feat"][None], keep=False)
        for f in forms:
            v = vis[f].cpu().numpy()[0].astype(np.float64)
            d = np.abs(v - ref["vis"][0])
            results[f]["vis_err_vs_fp64"] = {"max_abs": float(d.max()), "mean_abs": float(d.mean()),
                                             "norm_rel": float(d.max() / np.abs(ref["vis"]).max())}

    # roofline of the dominant kernel of the headline (BF16) form
    head = "bf16" if "bf16" in forms else forms[0]
    def costs_of(form):
        c = stage_costs(desc.widths, desc.c_in, H, W, form)
        c.update(raster_costs(scene.n_tris, H, W, fr.sm_size))
        c.update(gather_costs(scene.n_tris, H, W, desc.c_in, "gather hard6"))
        return c

    costs = costs_of(head)
    kern = results[head]["kernels"]
    dom = max(kern, key=lambda k: kern[k]["avg_us"])
    base = _base(dom)
    roof = None
    for f in forms:
        c = costs_of(f)
        for k, v in results[f]["kernels"].items():
            b = _base(k)
            if b in c:
                fl, by = c[b]
                t = v["avg_us"] * 1e-6
                v["gflop"] = fl / 1e9
                v["mbytes"] = by / 1e6
                v["tflops"] = fl / t / 1e12
                v["gbps"] = by / t / 1e9
                v["frac_mfma"] = fl / t / MFMA_PEAK[f]
                v["frac_hbm"] = by / t / HBM_PEAK
    if base in costs:
        fl, by = costs[base]
        t = kern[dom]["avg_us"] * 1e-6
        ai = fl / by
        if ai >= MFMA_PEAK[head] / HBM_PEAK:
            roof = {"kernel": dom, "bound": "mfma", "achieved": fl / t / 1e12, "peak": MFMA_PEAK[head] / 1e12,
                    "unit": "TFLOP/s", "frac": (fl / t) / MFMA_PEAK[head]}
        else:
            roof = {"kernel": dom, "bound": "hbm", "achieved": by / t / 1e9, "peak": HBM_PEAK / 1e9,
                    "unit": "GB/s", "frac": (by / t) / HBM_PEAK}
        from paper_2301_05262_amd.profsum import recorded_traffic
        measured = (recorded_traffic(TRAFFIC_MD).get(kernel_symbol(dom, results[head]["launch_variants"]), None)
                    if head == "bf16" else None)
        roof.update({"traffic": measured, "avg_us": kern[dom]["avg_us"], "algorithmic_bytes": by,
                     "algorithmic_flops": fl})
    roof_classes = class_rooflines(results, costs_of, [head] + [f for f in forms if f != head])
    batched = None
    if args.batched:
        batched = batched_section(S, torch, args.seed, reps=20)
        print(f"[bench] batched: {batched['graph_bf16_tuned']['frames_per_s']:.0f} frames/s (tuned graphs, bf16; "
              f"{batched['graph_bf16_default']['frames_per_s']:.0f} with default variants) vs "
              f"{batched['one_by_one_bf16']['frames_per_s']:.0f} (one by one, bf16) and "
              f"{batched['one_by_one_f32']['frames_per_s']:.0f} (one by one, f32)", file=sys.stderr, flush=True)
    training = None
    if args.training:
        training = training_section(S, torch, args.seed, steps=5)
        print(f"[bench] training step (32 x 512^2, fp32): {training['ms_per_step']:.2f} ms",
              file=sys.stderr, flush=True)
    temporal = None
    if args.temporal:
        temporal = temporal_section(S, torch, args.seed, steps=5)
        print(f"[bench] perturbation-loss training step (8 x (1+3) x 512^2, fp32): "
              f"{temporal['perturb_train']['ms_per_step']:.2f} ms; Eq. 3 metric 1080p pair: "
              f"{temporal['metric_1080p']['ms_per_pair'] * 1e3:.1f} us", file=sys.stderr, flush=True)
    f4 = None
    if args.f4:
        f4 = f4_section(S, torch, args.seed)
        print(f"[bench] penumbra P95 {f4['penumbra']['p95_width_px']:.1f} px over "
              f"{f4['penumbra']['penumbra_pixels']} penumbra pixels -> {f4['penumbra']['levels']} levels "
              f"(U3's receptive field {f4['penumbra']['receptive_field_of_u3_px']} px)", file=sys.stderr, flush=True)
    paper_net = None
    if args.paper_net:
        paper_net = paper_net_section(S, torch, args.seed, steps=50)
        print(f"[bench] paper net 1024x2048: bf16 {paper_net['bf16']['network_ms']:.3f} ms, "
              f"f16 {paper_net['f16']['network_ms']:.3f} ms, f32 {paper_net['f32']['network_ms']:.3f} ms; "
              f"s2d form: bf16 {paper_net['s2d']['bf16']['network_ms']:.3f} ms, "
              f"f16 {paper_net['s2d']['f16']['network_ms']:.3f} ms, f32 {paper_net['s2d']['f32']['network_ms']:.3f} ms",
              file=sys.stderr, flush=True)
    ms = results[head]["ms_per_frame"]
    line = {
        "metric": METRIC, "value": ms, "unit": "ms/frame", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": head, "data": "synthetic",
        "config": {"workload": WORKLOAD, "width": W, "height": H, "sm_size": fr.sm_size,
                   "n_tris": scene.n_tris, "net": "U-Net 6->16/32/64 (3 levels)", "features": "hard6",
                   "feature_storage": head if head in STORED_FORMS else "f32",
                   "seed": args.seed, "step": "light z-buffer + camera G-buffer + gather + network"},
        "network_ms": results[head]["network_ms"],
        "forms": results, "roofline": roof, "roofline_classes": roof_classes, "cpu_baseline": cpu,
        "batched": batched,
        "paper_net": paper_net, "training": training, "temporal": temporal, "design_analysis": f4,
    }
    print(json.dumps(line))
    sys.stdout.flush()
    if args.calib_copy:
        src = torch.ones(CALIB_COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
