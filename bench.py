#!/usr/bin/env python3
"""Throughput and latency of the P2S hot path on one MI355X.

A step is one whole frame through the hot path (correlated Zernike fields ->
P2S network -> fused basis blur -> tilt warp) of the single512 workload:
512x512, one channel, D/r0 = 3, K = 100 basis PSFs of 33x33, network
33-100-100-100.  The input image, basis and network are resident in HBM
before timing starts; every step draws new fields (seed 1000 + step).

Printed: ONE JSON line on stdout (progress goes to stderr) with
  value        BF16 frames/s (blur and network on BF16 MFMA, FP32 accumulate)
  fp32         the same for the plain FP32 path
  fp8          the same with the blur on FP8 E4M3 MFMA (network BF16)
  latency      p50/p99 single-frame latency, each frame synchronised
  stages_us    per-stage device time (events around each ABI call); mlp_blur
               is the kernel the frame runs (network inside the blur)
  roofline     dominant kernel (network + blur, BF16) against the BF16 MFMA
               peak, with the w-reading blur kernel alone beside it
  cpu_baseline the FP64 oracle timed on this host on a bounded sample, with
               the GPU outputs' relative L2 error against it
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP8_TFLOPS = 5000.0
PEAK_HBM_GBS = 8000.0
ANCHOR_GRID = 64        # anchor grid side of the anchor-model frames (the paper's example)
ANCHOR_CORR = 2.0       # anchor correlation length, in anchor spacings


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def blur_flops(C, H, W, K, P):
    """Algorithmic flops of the fused blur: the K x P^2 tap GEMM per pixel and
    channel plus the K-term row dot with the weights."""
    return 2.0 * C * H * W * K * (P * P + 1)


def mlp_flops(H, W, dims):
    """Algorithmic flops of the P2S network at every pixel: 2 in out per layer."""
    return 2.0 * H * W * sum(dims[i] * dims[i + 1] for i in range(len(dims) - 1))


def src_digest(*paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_sources):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, only if the kernel sources still match the digest recorded with
    the counters; else None."""
    path = os.path.join(ROOT, "profiles", "blur_mlp_bf16_single512_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        if rec.get("src_digest") != src_digest(*kernel_sources):
            return None
        return float(rec["hbm_bytes_per_launch"])
    except Exception:
        return None


def copy_mode(args, torch):
    """A plain device-to-device copy of 1 GiB (larger than the last-level
    cache), args.steps times: the bytes read and written per launch are known
    exactly."""
    n = 256 << 20
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(args.warmup):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / args.steps
    print(json.dumps({"mode": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                      "avg_us": us, "GBps": 8 * n / us / 1e3}), flush=True)


def fields_mode(args, torch, p2s, fr, NZ, H, W):
    """Only the field generator of the workload, args.steps calls."""
    F = torch.empty((NZ, H, W), dtype=torch.float32, device="cuda")
    fws = torch.empty(p2s.fields_workspace_bytes(H, W, NZ), dtype=torch.uint8, device="cuda")
    for i in range(args.warmup):
        p2s.make_fields(H, W, fr.d_over_r0, NZ, 1000 + i, F, fws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        p2s.make_fields(H, W, fr.d_over_r0, NZ, 2000 + i, F, fws)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / args.steps
    print(json.dumps({"mode": "fields", "avg_us": us, "output_bytes": 4 * NZ * H * W,
                      "GBps_output": 4 * NZ * H * W / us / 1e3}), flush=True)


def anchor_fields_mode(args, torch, p2s, fr, NZ, H, W):
    """Only the anchor-grid field generator (64 x 64 anchors), args.steps calls."""
    from paper_2107_11627_amd import anchors as panch
    model = panch.anchor_model(ANCHOR_GRID, NZ, ANCHOR_CORR)
    F = torch.empty((NZ, H, W), dtype=torch.float32, device="cuda")
    aws = torch.empty(model.fields_workspace_bytes(), dtype=torch.uint8, device="cuda")
    for i in range(args.warmup):
        p2s.make_fields_anchor(model, H, W, fr.d_over_r0, 1000 + i, F, aws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        p2s.make_fields_anchor(model, H, W, fr.d_over_r0, 2000 + i, F, aws)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / args.steps
    print(json.dumps({"mode": "anchor_fields", "avg_us": us, "grid": ANCHOR_GRID,
                      "product_flops": anchor_product_flops(ANCHOR_GRID, NZ), "output_bytes": 4 * NZ * H * W}),
          flush=True)


def anchor_product_flops(G, n):
    """Algorithmic flops of the anchor product L_s B: the lower triangle of the
    G^2 x G^2 factor times n columns, one multiply-add each."""
    return G * G * (G * G + 1) // 2 * n * 2


def anchor_section(args, torch, p2s, sim, img, fr, NZ, H, W, C, stream):
    """Frames with the paper's own field model: the Zernike coefficients of a
    64 x 64 anchor grid drawn from the 4096 x 4096 correlation matrix (with
    Noll's full R_Z) and interpolated to every pixel, then the same network,
    blur and warp.  Throughput in BF16, the field generator's own time, and
    one output kept for the oracle."""
    from paper_2107_11627_amd import anchors as panch
    t0 = time.perf_counter()
    model = panch.anchor_model(ANCHOR_GRID, NZ, ANCHOR_CORR)
    setup_s = time.perf_counter() - t0
    aws = torch.empty(model.workspace_bytes(C, H, W, sim.basis.K), dtype=torch.uint8, device="cuda")
    fws = torch.empty(model.fields_workspace_bytes(), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(img)
    F = torch.empty((NZ, H, W), dtype=torch.float32, device="cuda")

    def timed(fn, n):
        for i in range(args.warmup):
            fn(1000 + i)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(n):
            fn(3000 + i)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / n

    fields_us = timed(lambda sd: p2s.make_fields_anchor(model, H, W, fr.d_over_r0, sd, F, fws), args.steps)
    res = {"grid": ANCHOR_GRID, "correlation_length_anchor_spacings": ANCHOR_CORR, "host_setup_s": setup_s,
           "fields_us": fields_us,
           "product_flops": anchor_product_flops(ANCHOR_GRID, NZ)}
    for prec in ("bf16", "fp32"):
        us = timed(lambda sd: p2s.simulate_anchor(img, fr.d_over_r0, model, sim.basis, sim.net, sd, prec, out, aws),
                   args.steps)
        res[prec] = {"frames_per_s": 1e6 / us, "ms_per_frame": us / 1e3}
    p2s.simulate_anchor(img, fr.d_over_r0, model, sim.basis, sim.net, fr.field_seed, "bf16", out, aws)
    torch.cuda.synchronize()
    kept = out.cpu().numpy().astype(np.float64)
    log(f"[bench] anchor fields ({ANCHOR_GRID}x{ANCHOR_GRID} grid): {fields_us:.1f} us per field set; frames "
        f"BF16 {res['bf16']['frames_per_s']:.0f}/s, FP32 {res['fp32']['frames_per_s']:.0f}/s")
    model.close()
    return res, kept


def spectral_section(args, torch, p2s, S, ptrain):
    """spectral512: 512 x 512 RGB frames with one wavelength per channel (450,
    540, 570 nm), each through its own basis and trained network (three fused
    network-and-blur launches per frame), fields and warp shared.  BF16 and
    FP32 throughput; one BF16 output kept for the oracle."""
    from paper_2107_11627_amd import spectral
    wl = S.workload("spectral512")
    fr = wl.frames[0]
    z, d = wl.basis_draws()
    t0 = time.perf_counter()
    bases, Ws, bs = [], [], []
    for lam in wl.extra["wavelengths_nm"]:
        B = ptrain.workload_basis(wl, lam)
        w, b, _ = ptrain.load(f"p2s_rgb{int(lam)}", B)
        bases.append(B)
        Ws.append(w)
        bs.append(b)
    setup_s = time.perf_counter() - t0
    sim = spectral.SpectralSimulator(bases, Ws, bs, n_zernike=wl.n_zernike)
    img_h = fr.image()
    img = torch.from_numpy(img_h).cuda()
    out = torch.empty_like(img)
    stream = torch.cuda.current_stream()
    res = {"workload": "spectral512: 512x512 RGB, D/r0=3, channels at 450/540/570 nm, one K=100 basis of 33x33 "
                       "and one trained network 33-100-100-100 per channel", "host_setup_s": setup_s}
    for prec in ("bf16", "fp32"):
        for i in range(args.warmup):
            sim(img, fr.d_over_r0, 1000 + i, prec, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(args.steps):
            sim(img, fr.d_over_r0, 4000 + i, prec, out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        res[prec] = {"frames_per_s": 1e3 / ms, "ms_per_frame": ms}
    sim(img, fr.d_over_r0, fr.field_seed, "bf16", out=out)
    torch.cuda.synchronize()
    kept = {"image": img_h, "out": out.cpu().numpy().astype(np.float64), "bases": bases, "Ws": Ws, "bs": bs,
            "d": fr.d_over_r0, "seed": fr.field_seed}
    log(f"[bench] spectral512: BF16 {res['bf16']['frames_per_s']:.0f} frames/s, FP32 "
        f"{res['fp32']['frames_per_s']:.0f} frames/s")
    return res, kept


def mlp_blur_mode(args, torch, p2s, sim, img, fr, NZ, H, W, K, P, C, dims):
    """Only the kernel the frame spends most time in (network inside the
    blur), args.steps launches on one frame's fields."""
    F = torch.empty((NZ, H, W), dtype=torch.float32, device="cuda")
    fws = torch.empty(p2s.fields_workspace_bytes(H, W, NZ), dtype=torch.uint8, device="cuda")
    bl = torch.empty_like(img)
    p2s.make_fields(H, W, fr.d_over_r0, NZ, fr.field_seed, F, fws)
    for _ in range(args.warmup):
        p2s.mlp_blur(sim.net, F, NZ, img, sim.basis, args.precision, bl)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        p2s.mlp_blur(sim.net, F, NZ, img, sim.basis, args.precision, bl)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / args.steps
    fl = blur_flops(C, H, W, K, P) + mlp_flops(H, W, dims)
    print(json.dumps({"mode": "mlp_blur", "precision": args.precision, "avg_us": us,
                      "TFLOPs": fl / us / 1e6, "algorithmic_flops_per_launch": fl,
                      "algorithmic_bytes_per_launch": 4 * (2 * C * H * W + (NZ - 2) * H * W)}), flush=True)


def pipeline_times(torch, p2s, sim, img, fr, NZ, H, W, prec, frames, stream, seed0=5000):
    """The network-and-blur kernel's average duration under the same
    sustained load as the frame benchmark (a kernel run alone back to back,
    or right after lighter work, runs at other clocks): the frame as its
    three stage calls (fields, network and blur in one kernel, warp), with no
    synchronisation, `frames` frames
      (a) with HIP events on the launch stream around every network-and-blur
          launch (each event adds a little time of its own),
      (b) back to back with the kernel launched twice per frame and once,
          events only around the whole loop: the difference per frame is one
          launch's duration plus the short gap between two launches, and
      (c) with the kernel once and not at all: the difference is the frame
          time the kernel adds, less than its duration, because the launch
          gaps of the short field and warp kernels hide behind a long kernel
          and are exposed without it.
    Returns (events mean us, (b) us, frame us, (c) us)."""
    F = torch.empty((NZ, H, W), dtype=torch.float32, device="cuda")
    fws = torch.empty(p2s.fields_workspace_bytes(H, W, NZ), dtype=torch.uint8, device="cuda")
    bl = torch.empty_like(img)
    out = torch.empty_like(img)

    def loop(launches, ev=None):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(frames):
            p2s.make_fields(H, W, fr.d_over_r0, NZ, seed0 + 10 + i, F, fws)
            if ev is not None:
                ev[i][0].record(stream)
            for _ in range(launches):
                p2s.mlp_blur(sim.net, F, NZ, img, sim.basis, prec, bl)
            if ev is not None:
                ev[i][1].record(stream)
            p2s.warp(bl, F, out)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3 / frames

    for i in range(3):
        p2s.make_fields(H, W, fr.d_over_r0, NZ, seed0 + i, F, fws)
        p2s.mlp_blur(sim.net, F, NZ, img, sim.basis, prec, bl)
        p2s.warp(bl, F, out)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(frames)]
    loop(1, ev)
    per = float(np.mean([a.elapsed_time(b) * 1e3 for a, b in ev]))
    full = loop(1)
    twice = loop(2)
    without = loop(0)
    full = min(full, loop(1))
    return per, twice - full, full, full - without


def pipeline_mode(args, torch, p2s, sim, img, fr, NZ, H, W, K, P, C, dims):
    """The dominant kernel timed inside the frame pipeline (pipeline_times),
    args.steps frames: the command whose kernel trace is committed beside the
    benchmark's roofline figure."""
    ev_us, us, frame_us, share_us = pipeline_times(torch, p2s, sim, img, fr, NZ, H, W, args.precision, args.steps,
                                                   torch.cuda.current_stream())
    fl = blur_flops(C, H, W, K, P) + mlp_flops(H, W, dims)
    print(json.dumps({"mode": "pipeline", "precision": args.precision, "frames": args.steps,
                      "mlp_blur_avg_us": us, "mlp_blur_events_us": ev_us, "frame_us": frame_us,
                      "frame_share_us": share_us,
                      "TFLOPs": fl / us / 1e6, "algorithmic_flops_per_launch": fl}), flush=True)


def mlp_mode(args, torch, p2s, sim, fr, NZ, H, W, K, dims):
    """Only the P2S network kernel (w written to memory), args.steps launches
    (for counter runs)."""
    F = torch.empty((NZ, H, W), dtype=torch.float32, device="cuda")
    fws = torch.empty(p2s.fields_workspace_bytes(H, W, NZ), dtype=torch.uint8, device="cuda")
    wbuf = torch.empty((H * W, K), dtype=torch.float32, device="cuda")
    p2s.make_fields(H, W, fr.d_over_r0, NZ, fr.field_seed, F, fws)
    for _ in range(args.warmup):
        p2s.mlp(sim.net, F, NZ, H, W, args.precision, wbuf)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        p2s.mlp(sim.net, F, NZ, H, W, args.precision, wbuf)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / args.steps
    fl = mlp_flops(H, W, dims)
    print(json.dumps({"mode": "mlp", "precision": args.precision, "avg_us": us, "TFLOPs": fl / us / 1e6,
                      "algorithmic_flops_per_launch": fl}), flush=True)


def warp_mode(args, torch, p2s, sim, img, fr, NZ, H, W):
    """Only the tilt warp of the workload, args.steps launches (for counter
    runs)."""
    F = torch.empty((NZ, H, W), dtype=torch.float32, device="cuda")
    fws = torch.empty(p2s.fields_workspace_bytes(H, W, NZ), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(img)
    p2s.make_fields(H, W, fr.d_over_r0, NZ, fr.field_seed, F, fws)
    for _ in range(args.warmup):
        p2s.warp(img, F, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        p2s.warp(img, F, out)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / args.steps
    nbytes = 4 * (2 * img.numel() + 2 * H * W)
    print(json.dumps({"mode": "warp", "avg_us": us, "algorithmic_bytes_per_launch": nbytes,
                      "GBps": nbytes / us / 1e3}), flush=True)


def blur_mode(args, torch, p2s, sim, img, fr, NZ, H, W, K, P, C):
    """Only the fused blur of the workload, args.steps launches, on weights
    from one network evaluation."""
    F = torch.empty((NZ, H, W), dtype=torch.float32, device="cuda")
    fws = torch.empty(p2s.fields_workspace_bytes(H, W, NZ), dtype=torch.uint8, device="cuda")
    wbuf = torch.empty((H * W, K), dtype=torch.float32, device="cuda")
    bl = torch.empty_like(img)
    p2s.make_fields(H, W, fr.d_over_r0, NZ, fr.field_seed, F, fws)
    p2s.mlp(sim.net, F, NZ, H, W, args.precision, wbuf)
    for _ in range(args.warmup):
        p2s.blur(img, sim.basis, wbuf, args.precision, bl)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        p2s.blur(img, sim.basis, wbuf, args.precision, bl)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / args.steps
    fl = blur_flops(C, H, W, K, P)
    print(json.dumps({"mode": "blur", "precision": args.precision, "avg_us": us,
                      "TFLOPs": fl / us / 1e6, "algorithmic_flops_per_launch": fl,
                      "algorithmic_bytes_per_launch": 4 * (2 * C * H * W + H * W * K)}), flush=True)


def batch_section(args, torch, p2s, S, pbasis, ptrain):
    """The two batch workloads (64 RGB 256x256 frames; 200 ragged frames) with
    the shared K=100, P=33 basis: BF16 and FP32 through the batched kernels
    (plan uploaded once, the launch captured in a HIP graph and replayed) and,
    for comparison, the same frames one p2s_simulate call at a time."""
    from paper_2107_11627_amd import autotune

    wl0 = S.workload("batch256")
    z, d = wl0.basis_draws()
    basis, _ = pbasis.learn_basis(z, d, wl0.K, wl0.P, wl0.n_zernike)
    Ws, bs, _ = ptrain.load("p2s_shared", basis)          # trained for this basis
    sim = p2s.Simulator(basis, Ws, bs, n_zernike=wl0.n_zernike)
    out = {}
    samples = {}
    for name in ("batch256", "ragged"):
        wl = S.workload(name)
        t0 = time.perf_counter()
        imgs = [torch.from_numpy(f.image()).cuda() for f in wl.frames]
        dd = [f.d_over_r0 for f in wl.frames]
        seeds = [f.field_seed for f in wl.frames]
        log(f"[bench] {name}: {len(imgs)} frames ready in {time.perf_counter() - t0:.1f} s")
        shapes = [tuple(im.shape) for im in imgs]
        mpix = sum(c * h * w for c, h, w in shapes) / 1e6
        outs = [torch.empty_like(im) for im in imgs]
        ws = sim.batch_workspace(shapes)
        rec = {"frames": len(imgs), "megapixels_x_channels": mpix, "workspace_GiB": ws.numel() / 2 ** 30}
        # frames kept for the oracle check in the CPU-baseline leg: the first 4
        # of the uniform batch; 8 of the ragged batch, one of each size and
        # channel count in order of appearance, starting with a 768 x 768 RGB one
        if name == "batch256":
            pick = list(range(4))
        else:
            first768 = next(i for i, sh in enumerate(shapes) if sh == (3, 768, 768))
            pick, seen = [first768], {shapes[first768]}
            for i, sh in enumerate(shapes):
                if len(pick) == 8:
                    break
                if sh not in seen:
                    pick.append(i)
                    seen.add(sh)
            for i in range(len(shapes)):
                if len(pick) == 8:
                    break
                if i not in pick:
                    pick.append(i)
        rec["oracle_frames"] = [{"frame": i, "shape": list(shapes[i])} for i in pick]
        samples[name] = [{"image": imgs[i].cpu().numpy(), "d": dd[i], "seed": seeds[i], "out": {}} for i in pick]
        samples[name + "_basis"] = (basis, Ws, bs)
        for prec in ("bf16", "fp32", "fp8"):
            opt = autotune.tune(sim, imgs, dd, seeds, prec, outs=outs, ws=ws)
            b = p2s.Batch(imgs, outs, dd, seeds, sim.basis, sim.net, prec, ws, sim.n_zernike, **opt)
            b.upload()
            b.launch()
            torch.cuda.synchronize()
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(s):
                with torch.cuda.graph(g, stream=s):
                    b.launch(stream=s)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            reps = args.batch_reps
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                g.replay()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            items, grid = b.info()
            for smp, i in zip(samples[name], pick):
                smp["out"][prec] = outs[i].cpu().numpy().astype(np.float64)
            # the same frames one at a time through p2s_simulate (one untimed pass
            # first, so that the workspace has reached its largest size)
            for k, im in enumerate(imgs):
                sim(im, dd[k], seeds[k], prec, out=outs[k])
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for k, im in enumerate(imgs):
                sim(im, dd[k], seeds[k], prec, out=outs[k])
            e1.record()
            torch.cuda.synchronize()
            ms_solo = e0.elapsed_time(e1)
            rec[prec] = {"batched_frames_per_s": len(imgs) / (ms / 1e3), "batch_ms": ms,
                         "per_frame_frames_per_s": len(imgs) / (ms_solo / 1e3), "per_frame_ms": ms_solo,
                         "schedule": opt, "tuner_us": autotune.last_timings(shapes, prec, sim.basis.K, sim.basis.P),
                         "items": items, "grid": grid}
            log(f"[bench] {name} {prec}: batched {rec[prec]['batched_frames_per_s']:.1f} frames/s "
                f"({ms:.2f} ms/batch, {opt}), one at a time {rec[prec]['per_frame_frames_per_s']:.1f} frames/s")
            del g
            b.close()
        rec["bf16_batched_vs_fp32_per_frame"] = (rec["bf16"]["batched_frames_per_s"] /
                                                 rec["fp32"]["per_frame_frames_per_s"])
        out[name] = rec
        del imgs, outs, ws
        torch.cuda.empty_cache()
    return out, samples


def serving_section(args, torch, p2s, S, pbasis, ptrain):
    """The serving workload: requests of 128..2048 RGB through the
    continuous-batching loop in BF16 under the HBM admission budget.  First
    all requests queued at once (the saturated request rate), then Poisson
    arrivals at a fixed fraction of that rate (latency p50/p99, on the host
    clock), then the plain FP32 per-frame path (one p2s_simulate call per
    request).  Request images and outputs are allocated before the loop runs;
    the loop itself allocates only its arena (the budget).  A few served
    requests are kept for the oracle check in the CPU-baseline leg."""
    from paper_2107_11627_amd import serving as sv

    wl = S.workload("serving")
    z, d = wl.basis_draws()
    basis, _ = pbasis.learn_basis(z, d, wl.K, wl.P, wl.n_zernike)
    Ws, bs, _ = ptrain.load("p2s_shared", basis)          # trained for this basis
    sim = p2s.Simulator(basis, Ws, bs, n_zernike=wl.n_zernike)
    frames = wl.frames[: args.serving_requests]
    t0 = time.perf_counter()
    imgs = [S.blob_image_device(f.H, f.W, f.C, f.image_seed, f.noise_std, device_noise=True) for f in frames]
    outs = [torch.empty_like(im) for im in imgs]
    torch.cuda.synchronize()
    log(f"[bench] serving: {len(imgs)} request images on the device in {time.perf_counter() - t0:.1f} s")
    budget = wl.extra["hbm_budget_bytes"]

    def requests(arrivals):
        rs = []
        for i, f in enumerate(frames):
            r = sv.Request(i, imgs[i], f.d_over_r0, f.field_seed, float(arrivals[i]))
            r.out = outs[i]
            rs.append(r)
        return rs

    res = {"requests": len(frames), "budget_GiB": budget / 2 ** 30,
           "megapixels_x_channels": sum(f.C * f.H * f.W for f in frames) / 1e6,
           "clock": "host perf_counter for arrivals and finishes (finish = first poll that sees the batch's event)"}

    def run(label, arrivals):
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        ex = sv.GpuExecutor(sim, "bf16", budget, n_slots=args.serving_slots)
        eng = sv.Engine(ex, budget, n_slots=args.serving_slots, max_batch_frames=args.serving_max_batch)
        sv.run(eng, requests(np.zeros(len(frames)))[:4])          # warm the kernels and the plan path
        eng = sv.Engine(ex, budget, n_slots=args.serving_slots, max_batch_frames=args.serving_max_batch)
        st = sv.run(eng, requests(arrivals))
        torch.cuda.synchronize()
        st["device_bytes_allocated_by_loop"] = torch.cuda.max_memory_allocated() - base   # the arena
        res[label] = st
        log(f"[bench] serving {label}: {st['frames_per_s']:.1f} frames/s, p50 {st['latency_ms']['p50']:.2f} ms, "
            f"p99 {st['latency_ms']['p99']:.2f} ms, {st['batches']} batches (mean {st['mean_batch_frames']:.2f} "
            f"frames, {st['overlapped_launches']} overlapped), peak {st['peak_hbm_bytes'] / 2 ** 30:.1f} GiB")
        del ex, eng

    run("saturated", np.zeros(len(frames)))
    frac = wl.extra["load_fraction"]
    rate = frac * res["saturated"]["frames_per_s"]
    res["arrival_rate_hz"] = rate
    res["load_fraction_of_saturated"] = frac
    run("poisson", sv.poisson_arrivals(len(frames), rate, wl.extra["arrival_seed"]))
    # oracle sample: 7 early requests and the largest one
    pick = list(range(min(7, len(frames))))
    big = max(range(len(frames)), key=lambda i: frames[i].H * frames[i].W)
    if big not in pick:
        pick.append(big)
    samples = [{"rid": i, "image": imgs[i].cpu().numpy(), "d": frames[i].d_over_r0, "seed": frames[i].field_seed,
                "out": {"bf16": outs[i].cpu().numpy().astype(np.float64)}} for i in pick]
    # one 2048 x 2048 RGB request through the same loop on its own
    f2 = S.FrameSpec(2048, 2048, 3, 4.0, 7999, 3999, 0.02)
    im2 = S.blob_image_device(f2.H, f2.W, f2.C, f2.image_seed, f2.noise_std, device_noise=True)
    r2 = sv.Request(0, im2, f2.d_over_r0, f2.field_seed, 0.0)
    r2.out = torch.empty_like(im2)
    ex = sv.GpuExecutor(sim, "bf16", budget, n_slots=1)
    st2 = sv.run(sv.Engine(ex, budget, n_slots=1), [r2])
    torch.cuda.synchronize()
    res["single_2048_rgb_latency_ms"] = st2["latency_ms"]["p50"]
    samples.append({"rid": "2048x2048", "image": im2.cpu().numpy(), "d": f2.d_over_r0, "seed": f2.field_seed,
                    "out": {"bf16": r2.out.cpu().numpy().astype(np.float64)}})
    del ex, im2, r2
    # plain FP32 per-frame path over the same requests
    lat = []
    t = time.perf_counter()
    for i, im in enumerate(imgs):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        sim(im, frames[i].d_over_r0, frames[i].field_seed, "fp32", out=outs[i])
        b.record()
        lat.append((a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    lt = np.array([a.elapsed_time(b) for a, b in lat])
    res["fp32_per_frame"] = {"frames_per_s": len(imgs) / wall,
                             "latency_ms": {"p50": float(np.percentile(lt, 50)), "p99": float(np.percentile(lt, 99))},
                             "note": "device time per p2s_simulate call, frames back to back"}
    res["bf16_serving_vs_fp32_per_frame"] = res["saturated"]["frames_per_s"] / res["fp32_per_frame"]["frames_per_s"]
    log(f"[bench] serving fp32 per-frame: {res['fp32_per_frame']['frames_per_s']:.1f} frames/s")
    del imgs, outs
    torch.cuda.empty_cache()
    return res, {"basis": basis, "Ws": Ws, "bs": bs, "requests": samples}


def oracle_error(smp, basis, Ws, bs, n_pix, seed):
    """Relative L2 error of a GPU output against the FP64 oracle: the whole
    frame when it is small, else on n_pix sampled pixels (corners, edge
    midpoints and uniform draws) evaluated one by one."""
    from oracle.simulate import simulate as osimulate
    from oracle.simulate import simulate_pixels as osimulate_pixels
    img = smp["image"]
    C, H, W = img.shape
    if H * W <= 512 * 320:
        ref = osimulate(img, smp["d"], basis, Ws, bs, seed=smp["seed"])["out"]
        return {p: float(np.linalg.norm(got - ref) / np.linalg.norm(ref)) for p, got in smp["out"].items()}, "whole"
    rng = np.random.default_rng(seed)
    pix = [(c, y, x) for c in range(C) for y in (0, H // 2, H - 1) for x in (0, W // 2, W - 1)]
    while len(pix) < n_pix:
        pix.append((int(rng.integers(C)), int(rng.integers(H)), int(rng.integers(W))))
    ref = osimulate_pixels(img, smp["d"], basis, Ws, bs, smp["seed"], pix)
    idx = tuple(np.array(pix).T)
    return ({p: float(np.linalg.norm(got[idx] - ref) / np.linalg.norm(ref)) for p, got in smp["out"].items()},
            f"{len(pix)} sampled pixels")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--settle-s", type=float, default=0.3,
                    help="untimed frames for this many seconds before each precision's warm-up (device clocks)")
    ap.add_argument("--latency-frames", type=int, default=200)
    ap.add_argument("--stage-reps", type=int, default=20)
    ap.add_argument("--pipeline-frames", type=int, default=200)
    ap.add_argument("--cpu-frames", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--no-batches", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=1000)
    ap.add_argument("--serving-slots", type=int, default=2)
    ap.add_argument("--serving-max-batch", type=int, default=16)
    ap.add_argument("--no-anchors", action="store_true")
    ap.add_argument("--no-spectral", action="store_true")
    ap.add_argument("--mode", choices=["frame", "blur", "mlp", "mlp_blur", "pipeline", "fields", "anchor_fields",
                                       "warp", "copy"],
                    default="frame",
                    help="frame: the benchmark; blur / mlp / mlp_blur / fields / anchor_fields / warp: only that "
                         "kernel of the "
                         "workload (for counter runs); pipeline: the network-and-blur kernel timed inside "
                         "back-to-back frames (the benchmark's roofline timing); "
                         "copy: a plain device copy of known size (calibrates byte counters)")
    ap.add_argument("--precision", choices=["bf16", "fp32", "fp8"], default="bf16",
                    help="precision of the single-kernel modes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (frames are independent and "
              f"would be routed across GPUs without communication, see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import p2s_synth as S
    from paper_2107_11627_amd import basis as pbasis
    from paper_2107_11627_amd import p2s
    from paper_2107_11627_amd import train as ptrain

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.mode == "copy":
        return copy_mode(args, torch)
    wl = S.workload("single512")
    fr = wl.frames[0]
    C, H, W, K, P, NZ = fr.C, fr.H, fr.W, wl.K, wl.P, wl.n_zernike

    log(f"[bench] learning the K={K} P={P} basis from {wl.n_psf} PSFs (one-time host setup)")
    t0 = time.perf_counter()
    z, d = wl.basis_draws()
    basis, _ = pbasis.learn_basis(z, d, K, P, NZ)
    log(f"[bench] basis ready in {time.perf_counter() - t0:.1f} s")
    Ws, bs, net_meta = ptrain.load("p2s_single512", basis)   # the P2S network trained for this basis
    img_h = fr.image()
    sim = p2s.Simulator(basis, Ws, bs, n_zernike=NZ)
    img = torch.from_numpy(img_h).cuda()
    out = torch.empty_like(img)
    ws = sim.workspace(C, H, W)
    stream = torch.cuda.current_stream()

    def frame(seed, prec):
        p2s.simulate(img, fr.d_over_r0, sim.basis, sim.net, seed, prec, out, ws, NZ)

    if args.mode == "blur":
        return blur_mode(args, torch, p2s, sim, img, fr, NZ, H, W, K, P, C)
    if args.mode == "fields":
        return fields_mode(args, torch, p2s, fr, NZ, H, W)
    if args.mode == "anchor_fields":
        return anchor_fields_mode(args, torch, p2s, fr, NZ, H, W)
    if args.mode == "mlp_blur":
        return mlp_blur_mode(args, torch, p2s, sim, img, fr, NZ, H, W, K, P, C, wl.mlp_dims)
    if args.mode == "pipeline":
        return pipeline_mode(args, torch, p2s, sim, img, fr, NZ, H, W, K, P, C, wl.mlp_dims)
    if args.mode == "warp":
        return warp_mode(args, torch, p2s, sim, img, fr, NZ, H, W)
    if args.mode == "mlp":
        return mlp_mode(args, torch, p2s, sim, fr, NZ, H, W, K, wl.mlp_dims)

    res = {}
    outs = {}
    for prec in ("bf16", "fp32", "fp8"):
        # The device raises its clocks over the first ~0.1 s of sustained work
        # after an idle spell (here: the host-side basis set-up); untimed
        # frames for args.settle_s seconds bring it to its steady state, then
        # the args.warmup warm-up frames, then the timed frames.
        t_settle = time.perf_counter()
        i = 0
        while time.perf_counter() - t_settle < args.settle_s:
            frame(900000 + i, prec)
            i += 1
            if i % 50 == 0:
                torch.cuda.synchronize()
        for i in range(args.warmup):
            frame(1000 + i, prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for i in range(args.steps):
            frame(1000 + i, prec)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        res[prec] = {"frames_per_s": args.steps / (ms / 1e3), "ms_per_frame": ms / args.steps,
                     "wall_frames_per_s": args.steps / wall}
        log(f"[bench] {prec}: {res[prec]['frames_per_s']:.1f} frames/s ({ms / args.steps * 1e3:.1f} us/frame)")

        # latency: one frame at a time, synchronised
        lat_dev, lat_wall = [], []
        for i in range(args.latency_frames):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t = time.perf_counter()
            a.record(stream)
            frame(wl.extra["latency_field_seeds"][i % 200], prec)
            b.record(stream)
            b.synchronize()
            lat_wall.append((time.perf_counter() - t) * 1e3)
            lat_dev.append(a.elapsed_time(b))
        res[prec]["latency_ms"] = {"p50": float(np.percentile(lat_dev, 50)), "p99": float(np.percentile(lat_dev, 99)),
                                   "wall_p50": float(np.percentile(lat_wall, 50)),
                                   "wall_p99": float(np.percentile(lat_wall, 99))}

        # per-stage device time through the stage-level ABI calls
        F = ws[:NZ * H * W * 4].view(torch.float32).view(NZ, H, W)
        wbuf = torch.empty((H * W, K), dtype=torch.float32, device="cuda")
        fws = torch.empty(p2s.fields_workspace_bytes(H, W, NZ), dtype=torch.uint8, device="cuda")
        bl = torch.empty_like(img)
        fused = prec != "fp32"
        # each stage call back to back (args.stage_reps calls between two events,
        # after two untimed ones), so that every call runs at the clock a busy
        # device holds, as inside a stream of frames
        def stage_time(fn):
            for i in range(2):
                fn(i)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for i in range(args.stage_reps):
                fn(2 + i)
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) * 1e3 / args.stage_reps

        stages = {"fields": stage_time(lambda i: p2s.make_fields(H, W, fr.d_over_r0, NZ, 1000 + i, F, fws)),
                  "mlp": stage_time(lambda i: p2s.mlp(sim.net, F, NZ, H, W, prec, wbuf)),
                  "blur": stage_time(lambda i: p2s.blur(img, sim.basis, wbuf, prec, bl))}
        if fused:                            # network and blur in one kernel, as the frame runs them
            stages["mlp_blur"] = stage_time(lambda i: p2s.mlp_blur(sim.net, F, NZ, img, sim.basis, prec, bl))
        stages["warp"] = stage_time(lambda i: p2s.warp(bl, F, out))
        res[prec]["stages_us"] = stages
        if fused:
            # the dominant kernel's average duration inside the frame pipeline
            ev_us, us, frame_us, share_us = pipeline_times(torch, p2s, sim, img, fr, NZ, H, W, prec,
                                                           args.pipeline_frames, stream)
            res[prec]["mlp_blur_loop_us"] = us
            res[prec]["mlp_blur_events_us"] = ev_us
            res[prec]["pipeline_frame_us"] = frame_us
            res[prec]["mlp_blur_frame_share_us"] = share_us
            log(f"[bench] {prec} network+blur kernel inside the frame pipeline: {us:.1f} us "
                f"(events around each launch: {ev_us:.1f} us; it adds {share_us:.1f} us to a frame of "
                f"{frame_us:.1f} us)")
        log(f"[bench] {prec} stages (us): " + ", ".join(f"{k} {v:.1f}" for k, v in res[prec]["stages_us"].items()))
        del wbuf, fws, bl

        frame(fr.field_seed, prec)
        torch.cuda.synchronize()
        outs[prec] = out.cpu().numpy().astype(np.float64)

    flops = blur_flops(C, H, W, K, P)
    nflops = mlp_flops(H, W, wl.mlp_dims)
    fused_s = res["bf16"]["mlp_blur_loop_us"] * 1e-6
    achieved = (flops + nflops) / fused_s / 1e12
    kernel_src = ["paper_2107_11627_amd/csrc/blur.hip", "paper_2107_11627_amd/csrc/mlp_block.hpp",
                  "paper_2107_11627_amd/csrc/internal.hpp"]
    blur_s = res["bf16"]["stages_us"]["blur"] * 1e-6
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_BF16_TFLOPS, "traffic": traffic_from_profiles(kernel_src),
                "kernel": "blur_mlp_kernel<33,7,4,bf16>: P2S network evaluated inside the fused basis blur",
                "algorithmic_flops_per_launch": flops + nflops,
                "algorithmic_flops_split": {"blur": flops, "network": nflops},
                "avg_launch_us": fused_s * 1e6, "src_digest": src_digest(*kernel_src),
                "timing": f"{args.pipeline_frames} back-to-back frames (fields, network and blur, warp) with the "
                          f"kernel launched twice and once per frame, per-frame difference, as bench.py --mode "
                          f"pipeline",
                "events_around_each_launch_us": res["bf16"]["mlp_blur_events_us"],
                "frame_share_us": res["bf16"]["mlp_blur_frame_share_us"],
                "blur_only": {"kernel": "blur_bf16_kernel<33,7,8> (w read from memory)", "avg_launch_us": blur_s * 1e6,
                              "achieved": flops / blur_s / 1e12, "frac": flops / blur_s / 1e12 / PEAK_BF16_TFLOPS}}
    fp32_blur_s = res["fp32"]["stages_us"]["blur"] * 1e-6
    fp32_roof = {"bound": "mfma", "achieved": flops / fp32_blur_s / 1e12, "peak": PEAK_FP32_TFLOPS,
                 "frac": flops / fp32_blur_s / 1e12 / PEAK_FP32_TFLOPS}
    fp8_s = res["fp8"]["mlp_blur_loop_us"] * 1e-6
    fp8_roof = {"bound": "mfma", "kernel": "blur_mlp_kernel<33,7,4,fp8> (FP8 blur, BF16 network)",
                "achieved": (flops + nflops) / fp8_s / 1e12,
                "peak": PEAK_FP8_TFLOPS, "frac": (flops + nflops) / fp8_s / 1e12 / PEAK_FP8_TFLOPS,
                "note": "the network's share runs on BF16 MFMA (peak 2500)"}

    anchor, anchor_out = (None, None) if args.no_anchors else anchor_section(args, torch, p2s, sim, img, fr, NZ, H,
                                                                              W, C, stream)
    spec, spec_out = (None, None) if args.no_spectral else spectral_section(args, torch, p2s, S, ptrain)
    batches, batch_samples = (None, {}) if args.no_batches else batch_section(args, torch, p2s, S, pbasis, ptrain)
    serving, serving_samples = (None, None) if args.no_serving else serving_section(args, torch, p2s, S, pbasis, ptrain)

    cpu = None
    errs = None
    if not args.no_cpu_baseline:
        from oracle.simulate import simulate as osimulate
        try:
            from threadpoolctl import threadpool_info
            threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
        except Exception:
            threads = os.cpu_count()
        log(f"[bench] oracle: {args.cpu_frames} full frames in FP64 on the host ({threads} BLAS threads)")
        t0 = time.perf_counter()
        ref = None
        for i in range(args.cpu_frames):
            r = osimulate(img_h, fr.d_over_r0, basis, Ws, bs, seed=fr.field_seed + i)["out"]
            if i == 0:
                ref = r
        dt = time.perf_counter() - t0
        cpu = {"value": args.cpu_frames / dt, "unit": "frames/s", "cores": int(threads), "kind": "oracle",
               "sample": f"{args.cpu_frames} whole single512 frames (fields, network, blur, warp) in FP64 NumPy",
               "host_cpus": os.cpu_count()}
        errs = {p: float(np.linalg.norm(outs[p] - ref) / np.linalg.norm(ref)) for p in outs}
        # the kept frames of each batch workload and served requests, every
        # precision they ran in, against the oracle (parity checks; untimed)
        t1 = time.perf_counter()
        for name in ("batch256", "ragged"):
            if name not in batch_samples:
                continue
            ob, oW, ob_ = batch_samples[name + "_basis"]
            for k, smp in enumerate(batch_samples[name]):
                e, how = oracle_error(smp, ob, oW, ob_, 4000, k)
                batches[name]["oracle_frames"][k].update({"rel_l2": e, "compared_on": how})
            worst = {p: max(f["rel_l2"][p] for f in batches[name]["oracle_frames"]) for p in ("fp32", "bf16", "fp8")}
            batches[name]["oracle_worst_rel_l2"] = worst
            log(f"[bench] {name}: worst rel-L2 vs oracle over {len(batch_samples[name])} frames: " +
                ", ".join(f"{p} {v:.2e}" for p, v in worst.items()))
        if serving_samples:
            checked = []
            for k, smp in enumerate(serving_samples["requests"]):
                e, how = oracle_error(smp, serving_samples["basis"], serving_samples["Ws"], serving_samples["bs"],
                                      4000, 100 + k)
                checked.append({"request": smp["rid"], "shape": list(smp["image"].shape), "rel_l2_bf16": e["bf16"],
                                "compared_on": how})
            serving["oracle_requests"] = checked
            serving["oracle_worst_rel_l2_bf16"] = max(c["rel_l2_bf16"] for c in checked)
            log(f"[bench] serving: worst BF16 rel-L2 vs oracle over {len(checked)} requests: "
                f"{serving['oracle_worst_rel_l2_bf16']:.2e}")
        if anchor_out is not None:
            from oracle.simulate import simulate_pixels as osimulate_pixels
            rng = np.random.default_rng(7)
            pix = [(0, y, x) for y in (0, H // 2, H - 1) for x in (0, W // 2, W - 1)]
            pix += [(0, int(y), int(x)) for y, x in zip(rng.integers(0, H, 247), rng.integers(0, W, 247))]
            ref = osimulate_pixels(img_h, fr.d_over_r0, basis, Ws, bs, fr.field_seed, pix, n_zernike=NZ,
                                   field_model="anchor", G=ANCHOR_GRID, anchor_corr=ANCHOR_CORR)
            idx = tuple(np.array(pix).T)
            anchor["rel_l2_bf16_vs_oracle"] = float(np.linalg.norm(anchor_out[idx] - ref) / np.linalg.norm(ref))
            anchor["oracle_compared_on"] = f"{len(pix)} sampled pixels"
            log(f"[bench] anchor frame: BF16 rel-L2 vs oracle {anchor['rel_l2_bf16_vs_oracle']:.2e}")
        if spec_out is not None:
            from oracle import spectral as ospec
            rng = np.random.default_rng(8)
            pix = [(c, y, x) for c in range(3) for y in (0, 255, 511) for x in (0, 256, 511)]
            pix += [(int(c), int(y), int(x)) for c, y, x in zip(rng.integers(0, 3, 223), rng.integers(0, 512, 223),
                                                                 rng.integers(0, 512, 223))]
            ref = ospec.simulate_spectral_pixels(spec_out["image"], spec_out["d"], spec_out["bases"], spec_out["Ws"],
                                                 spec_out["bs"], spec_out["seed"], pix)
            idx = tuple(np.array(pix).T)
            spec["rel_l2_bf16_vs_oracle"] = float(np.linalg.norm(spec_out["out"][idx] - ref) / np.linalg.norm(ref))
            spec["oracle_compared_on"] = f"{len(pix)} sampled pixels"
            log(f"[bench] spectral frame: BF16 rel-L2 vs oracle {spec['rel_l2_bf16_vs_oracle']:.2e}")
        log(f"[bench] oracle parity checks of batches, serving, anchor and spectral frames took "
            f"{time.perf_counter() - t1:.1f} s")
        log(f"[bench] oracle {cpu['value']:.3f} frames/s; rel-L2 vs oracle: " +
            ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))

    line = {
        "metric": "frames/s at 512^2 K=100 (FP32 vs BF16-MFMA) + p50/p99 frame latency",
        "value": res["bf16"]["frames_per_s"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_s": args.settle_s,
        "ms_per_step": res["bf16"]["ms_per_frame"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "single512: 512x512 C=1 blob image, D/r0=3, 35 Zernike planes, K=100 basis of "
                               "33x33, network 33-100-100-100 (trained), new field seed per frame",
                   "network": net_meta["file"],
                   "H": H, "W": W, "C": C, "K": K, "P": P, "n_zernike": NZ, "global_batch": 1},
        "latency_ms": {p: res[p]["latency_ms"] for p in res},
        "fp32": {"frames_per_s": res["fp32"]["frames_per_s"], "ms_per_frame": res["fp32"]["ms_per_frame"],
                 "blur_roofline": fp32_roof},
        "fp8": {"frames_per_s": res["fp8"]["frames_per_s"], "ms_per_frame": res["fp8"]["ms_per_frame"],
                "blur_roofline": fp8_roof,
                "note": "blur on FP8 E4M3 MFMA with per-basis power-of-two scales; network in BF16"},
        "stages_us": {p: res[p]["stages_us"] for p in res},
        "roofline": roofline,
        "anchor_fields": anchor,
        "spectral": spec,
        "batches": batches,
        "serving": serving,
        "cpu_baseline": cpu,
        "rel_l2_vs_oracle": errs,
        "paper_context": "0.026 s/frame on a Tesla V100 for a 256x256 frame (Table 2); different hardware and frame",
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
