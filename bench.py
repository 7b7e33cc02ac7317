"""Benchmark: 4K frames/s at N_max = 200 on one MI355X.

Workload: batches of 3840 x 2160 FP32 frames (inscribed disk of diameter
2160 px), every Zernike moment up to n_max = 200 (10201 complex moments per
frame) on a 1080-ring x 4096-angle polar grid.  One step = the whole hot path
over one batch: fused resample + angular FFT (zm_spectra), then the radial
projection on the matrix cores (zm_project).  Frames are device resident
before the timed region starts.  The timed steps carry events only around the
whole run; the kernels' own durations come from the same number of steps run
right after with an event around each kernel (HIP events on the launch stream).

Prints ONE JSON line (rank 0).  Extra keys beside the standard ones (metric,
value, unit, ms_per_step, config, ...):
  roofline       resample+FFT kernel: algorithmic bytes per launch / average
                 launch duration (HIP events on the launch stream, in the
                 instrumented steps) vs 8 TB/s;
                 traffic = HBM bytes per launch from the committed rocprofv3
                 counter summary (null once the kernel source has changed)
  projection     the projection kernel's useful FLOP rate vs the MFMA peak
  split_bf16, split_f16
                 the same step with the hi/lo split-BF16 / split-FP16
                 projection: the spectra kernel's HBM rate, the projection's
                 useful and issued MFMA fractions and its operand HBM rate
  cpu_baseline   the FP64 CPU oracle on a bounded sample, scaled to images/s,
                 on all host threads and (single_thread) on one
  batch_sweep    the FP32 step at batch 1, 8 and 128 (kernel times by HIP
                 events; the spectra kernel's HBM fraction)
  resample_alone the same FP32 step as two launches: the resampler alone
                 (zm_resample_polar, polar image written to HBM) and moments
                 from that image; times and bit-identity with the fused step
  batch_form     64 mixed square frames (sides 256..2048, N_max 30/50/100) in
                 one persistent launch replayed from a HIP graph, with its HBM
                 rate (algorithmic bytes of the whole batch), tuned and
                 untuned shape; beside it the same frames as per-plan
                 zm_moments launches, and 64 4K frames of one plan
  latency        the serving form: Poisson arrivals at a fixed rate of
                 640x480 / 1080p / 4K frames (N_max 30/100/200) from pinned host
                 memory, continuous batching under an HBM budget; p50 / p99 /
                 p99.9 latency (arrival -> moments in host memory) with the
                 per-request split (queue, copies, compute, other), FP32 and
                 split-BF16 projection; saturation throughput from a burst,
                 then streams at the fixed rate and at 50 % / 80 % of it; and
                 (persistent) each admission round as one persistent launch
  reconstruction eq. (9) of one 4K frame at N_max 200 at the pixel centres
                 (FP64 rate vs the FP64 vector peak) and at the polar nodes
  cartesian_single_moment
                 one moment of 4000 x 4000 frames by the Cartesian pixel sum
                 (eq. (6), 8-point symmetry) at orders 10 / 200 / 500; HBM
                 rate of the disk pixels
  dedup          moments as image hashes (eq. (16)/(17)) over a synthetic set
                 with planted duplicate groups
  stability      orthogonality of the radial table to order 500 on
                 Gauss-Legendre rings (Sec. 3.1), FP64 and the operand forms
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

H, W = 2160, 3840
NMAX, RINGS, ANGLES = 200, 1080, 4096
DISTINCT = 4          # distinct seeded frames (seeds 3..6), tiled to fill the batch
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "bf16x2": 2500.0, "f16x2": 2500.0}
FP64_VECTOR_PEAK_TFLOPS = 78.6
# pixel-centre reconstruction, per (disk pixel, moment): the recurrence step
# (alpha x + beta) q1 + gamma q2 (5 flops) and the complex accumulation (4)
RECON_FLOPS_PER_PIXEL_MOMENT = 9
METRIC = "4K images/s at N_max=200 (FP32 vs split-BF16) + p50/p99 latency at fixed QPS"


# HBM bytes of the resample+FFT kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters (scaled by a copy of known size), as committed with the counter
# summary; used only while the kernel sources are the ones it was taken on.
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "polar_fft_kernel_4k_n200_b64.md")
COUNTER_BATCH = 64
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2304_14492_amd", "csrc", f)
                  for f in ("fft_body.h", "fft_pair_body.inc", "polar_fft.hip")]


def measured_traffic(batch):
    try:
        txt = open(COUNTER_SUMMARY).read()
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(f, "rb").read())
    except OSError:
        return None
    t = re.search(r"traffic-bytes-per-launch: (\d+)", txt)
    k = re.search(r"kernel-source-sha256: ([0-9a-f]{64})", txt)
    if not (t and k) or k.group(1) != h.hexdigest() or batch != COUNTER_BATCH:
        return None
    return int(t.group(1))


def disk_pixels(h, w):
    d = min(h, w)
    X = 2 * np.arange(w, dtype=np.int64) - (w - 1)
    Y = (h - 1) - 2 * np.arange(h, dtype=np.int64)
    return int(np.count_nonzero(X[None, :] ** 2 + Y[:, None] ** 2 <= d * d))


def spectra_bytes_per_frame():
    # algorithmic traffic of the fused resample+FFT: every pixel of the disk
    # footprint read once (FP32) + the ring spectra written once (FP32 complex,
    # n_max + 1 bins per ring)
    return 4 * disk_pixels(H, W) + (NMAX + 1) * 2 * RINGS * 4


def projection_flops_per_frame():
    # useful work: 2 (re, im) x 2 flops per multiply-add, over rings, per moment
    return 4 * RINGS * ((NMAX // 2 + 1) ** 2)


def operand_bytes(plan):
    """Bytes of a plan's projection operand (rows padded to 16 per m block,
    rings to rings_padded; FP32, or two 16-bit parts for the splits)."""
    rows = sum((plan.n_max - m) // 2 // 16 * 16 + 16 for m in range(plan.n_max + 1))
    return rows * plan.rings_padded * 4


def projection_entry(dtype, proj_ms, batch):
    """Projection figures for one dtype: useful and issued MFMA rates (the
    split forms issue three products per useful one) against the dtype's
    dense peak, and the HBM rate of its operands (operand table once, spectra
    read, moments written) against 8 TB/s."""
    import paper_2304_14492_amd as zm
    plan = zm.Plan.__new__(zm.Plan)
    plan.n_max, plan.rings_padded = NMAX, (RINGS + 31) // 32 * 32
    flops = projection_flops_per_frame() * batch
    issued = flops * (1 if dtype == "f32" else 3)
    tf = flops / (proj_ms / 1e3) / 1e12
    nbytes = operand_bytes(plan) + batch * ((NMAX + 1) * 2 * RINGS * 4 + (NMAX // 2 + 1) ** 2 * 2 * 4)
    gbs = nbytes / (proj_ms / 1e3) / 1e9
    return {"kernel": "project_kernel", "avg_launch_ms": round(proj_ms, 4), "useful_tflops": round(tf, 2),
            "peak_tflops": MFMA_PEAK_TFLOPS[dtype], "frac": round(tf / MFMA_PEAK_TFLOPS[dtype], 4),
            "issued_frac": round(issued / (proj_ms / 1e3) / 1e12 / MFMA_PEAK_TFLOPS[dtype], 4),
            "hbm": {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": nbytes}}


def stability_sweep():
    """Sec. 3.1 / Fig. 1: orthogonality error of the radial table to order 500
    on Gauss-Legendre rings (502), FP64 as built on the GPU by eq. (7) and in
    the projection operand's FP32 / hi+lo BF16 / hi+lo FP16 forms; maximum per
    band of 50 orders."""
    import paper_2304_14492_amd as zm
    from paper_2304_14492_amd import stability
    plan = zm.Plan(500, 2048, 2048, dtype="f32", rings=502, angles=1024, rule="gauss_legendre")
    res = stability.sweep(plan)
    res.pop("curves")
    res["measure"] = "max over m, n' of |2(n+1) sum_r w_r R_nm R_n'm - delta_nn'|"
    return res


def make_frames(batch):
    import synth
    from synth.frames import FrameSpec
    spec = FrameSpec(H, W, blobs=32, polygons=16, noise=False, zero_outside=False)
    base = [synth.make_frame(spec, 3 + i) for i in range(min(DISTINCT, batch))]
    return base


def run_gpu(batch, steps, warmup, dtype):
    import torch
    import paper_2304_14492_amd as zm
    plan = zm.Plan(NMAX, H, W, dtype=dtype, rings=RINGS, angles=ANGLES)
    base = make_frames(batch)
    frames = torch.empty(batch, H, W, dtype=torch.float32, device="cuda")
    for i in range(batch):
        frames[i].copy_(torch.from_numpy(base[i % len(base)]))
    ws = plan.workspace(batch)
    Z = torch.empty(batch, plan.num_moments, 2, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan.spectra(frames, ws, stream)
        if ev is not None:
            ev[1].record(stream)
        plan.project(batch, Z, ws, stream)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # the timed steps: events only around the whole run (an event recorded
    # between the two kernels costs the step 1-5 %)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    for k in range(steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    # then the same number of steps with events around each kernel, for the
    # kernels' own durations (the rooflines)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    spec_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    proj_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    out = dict(total_ms=total_ms, wall_s=wall, spec_ms=spec_ms, proj_ms=proj_ms, Z=Z, plan=plan)
    return out


def resample_alone(batch, steps, warmup):
    """The same step split in two: the resampler alone (zm_resample_polar, tiles
    of 32 rings x 64 angles, polar image written to HBM) then moments from the
    polar image (from-polar transform + projection).  Same moments, bit for bit."""
    import torch
    import paper_2304_14492_amd as zm
    plan = zm.Plan(NMAX, H, W, dtype="f32", rings=RINGS, angles=ANGLES)
    base = make_frames(batch)
    frames = torch.empty(batch, H, W, dtype=torch.float32, device="cuda")
    for i in range(batch):
        frames[i].copy_(torch.from_numpy(base[i % len(base)]))
    ws = plan.workspace(batch)
    P = torch.empty(batch, RINGS, ANGLES, dtype=torch.float32, device="cuda")
    Z1 = torch.empty(batch, plan.num_moments, 2, dtype=torch.float32, device="cuda")
    Z2 = torch.empty_like(Z1)
    stream = torch.cuda.current_stream()
    plan.moments(frames, out=Z1, workspace=ws, stream=stream)
    for _ in range(warmup):
        plan.resample_polar(frames, out=P, stream=stream)
        plan.moments_polar(P, out=Z2, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    same = bool(torch.equal(Z1, Z2))
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record(stream)
        plan.resample_polar(frames, out=P, stream=stream)
        ev[k][1].record(stream)
        plan.moments_polar(P, out=Z2, workspace=ws, stream=stream)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    res_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    pol_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    polar_bytes = batch * RINGS * ANGLES * 4
    return {"resample_ms": round(res_ms, 4), "moments_from_polar_ms": round(pol_ms, 4),
            "step_ms": round(res_ms + pol_ms, 4), "polar_image_bytes": polar_bytes,
            "resample_write_tbs": round(polar_bytes / (res_ms / 1e3) / 1e12, 3), "bit_identical_to_fused": same}


def cpu_baseline(budget_s):
    """FP64 oracle (resample + angular DFT + radial sum per frame; the exact
    radial table is plan-time work and is built once, untimed) on 4K frames."""
    import oracle
    import synth
    from synth.frames import FrameSpec
    spec = FrameSpec(H, W, blobs=32, polygons=16, noise=False, zero_outside=False)
    f = synth.make_frame(spec, 3).astype(np.float64)
    grid = oracle.ring_grid(RINGS)
    pl = oracle.pairs(NMAX)
    table = oracle.zrp(pl, grid)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.moments(f, NMAX, RINGS, ANGLES, plist=pl, table=table)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 200:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=n / el, unit="images/s", cores=min(cores, os.cpu_count() or cores), kind="oracle",
                sample=f"{n} full 3840x2160 frame(s) at N_max=200 (all 10201 moments), {el:.1f} s; "
                       "exact radial table built once beforehand (plan-time, untimed)")


def cpu_baseline_single_thread(budget_s):
    """The same oracle timing on one host thread, in a child process started
    with OMP_NUM_THREADS=1 (the oracle's OpenMP team is fixed at load)."""
    import subprocess
    code = ("import json, bench; r = bench.cpu_baseline(%r); print('CPU1 ' + json.dumps(r))" % budget_s)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=600)
    for line in out.stdout.splitlines():
        if line.startswith("CPU1 "):
            r = json.loads(line[5:])
            r["cores"] = 1
            return r
    raise RuntimeError("single-thread oracle run failed: " + out.stderr[-2000:])


def batch_form(steps):
    import torch
    import paper_2304_14492_amd as zm
    import synth
    from synth.frames import FrameSpec
    specs = synth.batch_sides(64, seed=4)
    frames, plans, cache = [], [], {}
    for side, nmax, seed in specs:
        frames.append(torch.from_numpy(synth.make_frame(FrameSpec(side, side, blobs=8), seed)).cuda())
        if (side, nmax) not in cache:
            cache[(side, nmax)] = zm.Plan(nmax, side, side, dtype="f32")
        plans.append(cache[(side, nmax)])
    ms, cfg = _time_batch(zm.Batch(plans, frames, autotune=True, graph=True), steps)
    ms_default, _ = _time_batch(zm.Batch(plans, frames, autotune=False, graph=True), steps)
    # reference: the same frames as one zm_moments launch pair per plan (frames of
    # a plan stacked), back to back on one stream
    groups = {}
    for (side, nmax, _), f in zip(specs, frames):
        groups.setdefault((side, nmax), []).append(f)
    stacks = [(cache[k], torch.stack(v)) for k, v in groups.items()]
    outs = [(pl, st, pl.workspace(st.shape[0]), torch.empty(st.shape[0], pl.num_moments, 2, device="cuda"))
            for pl, st in stacks]
    for pl, st, ws, z in outs:
        pl.moments(st, out=z, workspace=ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        for pl, st, ws, z in outs:
            pl.moments(st, out=z, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    ms_plan = e0.elapsed_time(e1) / steps
    # algorithmic HBM bytes of one batch: every frame's disk footprint read
    # once, its ring spectra written and read back once, its moments written,
    # and each plan's projection operand read once
    nbytes = 0
    for (side, nmax, _), pl in zip(specs, plans):
        spec_b = (nmax + 1) * 2 * pl.rings * 4
        nbytes += 4 * disk_pixels(side, side) + 2 * spec_b + pl.num_moments * 2 * 4
    for pl in cache.values():
        nbytes += operand_bytes(pl)
    gbs = nbytes / (ms / 1e3) / 1e9
    return {"images_per_s": round(len(frames) / (ms / 1e3), 1), "ms_per_batch": round(ms, 4), "frames": len(frames),
            "plans": len(cache), "route": cfg["route"], "grid": cfg["grid"], "item_order": cfg["order"],
            "queue_items": cfg["n_items"], "untuned_ms_per_batch": round(ms_default, 4),
            "per_plan_launches_ms": round(ms_plan, 4),
            "roofline": {"bound": "hbm", "kernel": "batch_kernel (persistent: resample + FFT + projection)",
                         "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": nbytes},
            "homogeneous_4k": batch_homogeneous(steps)}


def _time_batch(b, steps):
    """Average time of one graph replay of batch object b (then closed) and its tuned shape."""
    import torch
    b.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        b.run()
    e1.record()
    torch.cuda.synchronize()
    b.check()
    cfg = b.config()
    b.close()
    return e0.elapsed_time(e1) / steps, cfg


def batch_homogeneous(steps):
    """The batched form on 64 benchmark 4K frames of one plan (N_max 200, 1080 x
    4096 grid): tuned shape and time against the untuned default."""
    import torch
    import paper_2304_14492_amd as zm
    n = 64
    plan = zm.Plan(NMAX, H, W, dtype="f32", rings=RINGS, angles=ANGLES)
    base = [torch.from_numpy(f).cuda() for f in make_frames(DISTINCT)]
    stack = torch.empty(n, H, W, dtype=torch.float32, device="cuda")  # the frames as slices of one array
    for i in range(n):
        stack[i].copy_(base[i % DISTINCT])
    frames = [stack[i] for i in range(n)]
    ms, cfg = _time_batch(zm.Batch([plan] * n, frames, autotune=True, graph=True), steps)
    ms_default, cfg_default = _time_batch(zm.Batch([plan] * n, frames, autotune=False, graph=True), steps)
    return {"frames": n, "ms_per_batch": round(ms, 4), "images_per_s": round(n / (ms / 1e3), 1),
            "route": cfg["route"], "grid": cfg["grid"], "item_order": cfg["order"],
            "untuned_ms_per_batch": round(ms_default, 4),
            "untuned": {"route": cfg_default["route"], "grid": cfg_default["grid"],
                        "item_order": cfg_default["order"]}}


def reconstruction(reps=3):
    """eq. (9) reconstruction of one benchmark 4K frame from its N_max = 200
    moments: at the pixel centres (FP64 recurrence per pixel) and at the
    plan's polar nodes (FP64 table of eq. (7))."""
    import torch
    import paper_2304_14492_amd as zm
    f = torch.from_numpy(make_frames(1)[0]).cuda()[None]
    plan = zm.Plan(NMAX, H, W, dtype="f32", rings=RINGS, angles=ANGLES)
    Z = plan.moments(f)
    out = {"frame": [H, W], "n_max": NMAX}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for kind in ("cartesian", "polar"):
        zm.reconstruct(plan, Z, kind=kind)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            zm.reconstruct(plan, Z, kind=kind)
        e1.record()
        torch.cuda.synchronize()
        out[f"{kind}_ms"] = round(e0.elapsed_time(e1) / reps, 3)
    n_disk = int(disk_pixels(H, W))
    flops = RECON_FLOPS_PER_PIXEL_MOMENT * n_disk * plan.num_moments
    tf = flops / (out["cartesian_ms"] / 1e3) / 1e12
    out["cartesian_roofline"] = {"bound": "alu", "kernel": "recon_cart_kernel", "achieved": round(tf, 2),
                                 "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4), "flops": flops}
    return out


def cartesian_single_moment(side=4000, reps=20):
    """Fig. 5's workload: one moment of any order of side x side frames (the
    figure's largest side) by the Cartesian pixel sum of eq. (6) with 8-point
    symmetry; seeded uniform frames.  Algorithmic HBM bytes = the pixels of
    the disk (4 B each), the only pixels eq. (6) reads."""
    import torch
    import paper_2304_14492_amd as zm
    g = torch.Generator(device="cuda").manual_seed(4000)
    runs = []
    disk_bytes = 4 * disk_pixels(side, side)
    for B in (1, 16):
        f = torch.rand(B, side, side, device="cuda", generator=g)
        for n, m in ((10, 2), (200, 100), (500, 250)):
            zm.moment_cartesian(f, n, m)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                zm.moment_cartesian(f, n, m)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = B * disk_bytes / (ms / 1e3) / 1e9
            runs.append({"batch": B, "n": n, "m": m, "ms_per_call": round(ms, 4),
                         "us_per_frame": round(ms * 1e3 / B, 2), "GB_per_s": round(gbs, 1)})
        del f
    head = [r for r in runs if r["batch"] == 16 and r["n"] == 200][0]
    return {"side": side, "runs": runs,
            "roofline": {"bound": "hbm", "kernel": "cart_moment_kernel (batch 16, n 200, m 100)",
                         "achieved": head["GB_per_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(head["GB_per_s"] / HBM_PEAK_GBS, 4),
                         "bytes_per_launch": 16 * disk_bytes}}


def dedup_throughput(side=256, n_distinct=700, reps=3):
    """Sec. 2.7: duplicate groups of a synthetic set of side x side frames
    (the paper's image side): n_distinct originals, about half of them with
    copies, quarter / half turns and mirror images.  Moments to order 20 on
    the GPU (256 frames per launch), hashes at orders 16 and 20."""
    import torch
    import synth
    from paper_2304_14492_amd import Plan, dedup
    frames, truth = synth.dedup_set(side, n_distinct=n_distinct, seed=900)
    dev = torch.from_numpy(np.stack(frames)).cuda()
    plan = Plan(20, side, side, dtype="f32")
    groups, _ = dedup.find_duplicates(dev, orders=(16, 20), plan=plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        groups, _ = dedup.find_duplicates(dev, orders=(16, 20), plan=plan)
    dt = (time.perf_counter() - t0) / reps
    return {"frames": len(frames), "side": side, "orders": [16, 20], "seconds": round(dt, 4),
            "frames_per_s": round(len(frames) / dt, 1), "groups_found": len(groups),
            "groups_planted": len(truth), "all_found": groups == truth}


def serving(dtype, count, qps, warmup_s):
    """Serving form for one projection dtype: saturation throughput (every
    request queued at t = 0), then Poisson streams at the fixed rate `qps` and
    at 50 % / 80 % of the measured saturation, one zm_moments launch per plan
    group; then (`persistent`) saturation and the fixed rate with all admitted
    requests of a round in one persistent launch."""
    from paper_2304_14492_amd import serve
    dev = serve.GpuDevice(dtype=dtype, n_streams=4)

    def one(rate, n, burst=False):
        reqs = serve.make_requests(n, rate, seed=5, pool_per_size=3)
        if burst:
            for r in reqs:
                r.t_arrival = 0.0
        dev.warm({(r.H, r.W, r.nmax) for r in reqs})
        sch = serve.Scheduler(dev, budget_bytes=4 << 30, max_inflight=8, max_batch=8)
        gc.collect()
        gc.disable()  # no collector pauses inside the timed stream
        try:
            # poll while work is queued or in flight; sleep through idle gaps
            done = serve.run_stream(reqs, sch, idle_sleep=time.sleep)
        finally:
            gc.enable()
        st = serve.latency_stats(done, warmup_s=0.0 if burst else warmup_s, by_size=not burst)
        st.update(qps=None if burst else rate, requests=n, peak_budget_bytes=sch.peak_used)
        return st

    sat = one(qps, max(count // 4, 200), burst=True)["images_per_s"]
    out = {"dtype": dtype, "warmup_s": warmup_s, "saturation_images_per_s": sat, "runs": []}
    for rate in (qps, 0.5 * sat, 0.8 * sat):
        n = int(min(count, max(200, rate * (warmup_s + 8.0))))  # about 8 s after the warm-up
        out["runs"].append(one(rate, n))
    dev = serve.GpuDevice(dtype=dtype, n_streams=4, mode="persistent")
    sat_p = one(qps, max(count // 4, 200), burst=True)["images_per_s"]
    out["persistent"] = {"saturation_images_per_s": sat_p,
                         "runs": [one(qps, int(min(count, max(200, qps * (warmup_s + 8.0)))))]}

    def rnd(v):
        if isinstance(v, float):
            return round(v, 4)
        if isinstance(v, dict):
            return {k: rnd(x) for k, x in v.items()}
        if isinstance(v, list):
            return [rnd(x) for x in v]
        return v
    return rnd(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16x2", "f16x2"])
    ap.add_argument("--no-split", action="store_true", help="skip the split-BF16 comparison run")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="0 skips the CPU baseline")
    ap.add_argument("--qps", type=float, default=1000.0, help="serving arrival rate")
    ap.add_argument("--requests", type=int, default=10000,
                    help="at most this many requests per serving run (0 skips serving)")
    ap.add_argument("--no-batch-form", action="store_true")
    ap.add_argument("--no-batch-sweep", action="store_true", help="skip the FP32 step at batch 1, 8 and 128")
    ap.add_argument("--no-two-pass", action="store_true", help="skip the resampler-alone + from-polar timing")
    ap.add_argument("--no-recon", action="store_true", help="skip the reconstruction timing")
    ap.add_argument("--no-cartesian", action="store_true", help="skip the Cartesian single-moment timing")
    ap.add_argument("--no-dedup", action="store_true", help="skip the de-duplication timing")
    ap.add_argument("--no-stability", action="store_true", help="skip the order-500 orthogonality sweep")
    ap.add_argument("--cartesian-only", action="store_true",
                    help="only the Cartesian single-moment timing (prints its JSON object)")
    ap.add_argument("--batch-form-only", action="store_true",
                    help="only the batched persistent form's timing (prints its JSON object)")
    ap.add_argument("--recon-only", action="store_true",
                    help="only the reconstruction timing (prints its JSON object)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times): the reference for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters into bytes")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: every frame is independent, so frames shard across GPUs "
              "with no communication and the figure per GPU is the one to measure; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_mib": args.calibrate_copy, "bytes_read_per_copy": 4 * n,
                          "bytes_written_per_copy": 4 * n}))
        return
    if args.cartesian_only:
        print(json.dumps({"cartesian_single_moment": cartesian_single_moment()}), flush=True)
        return
    if args.batch_form_only:
        print(json.dumps({"batch_form": batch_form(args.steps)}), flush=True)
        return
    if args.recon_only:
        print(json.dumps({"reconstruction": reconstruction()}), flush=True)
        return
    print(f"[bench] batch={args.batch} steps={args.steps} warmup={args.warmup} dtype={args.dtype}",
          file=sys.stderr, flush=True)
    r = run_gpu(args.batch, args.steps, args.warmup, args.dtype)
    ms = r["total_ms"] / args.steps
    value = args.batch / (ms / 1e3)
    bytes_launch = spectra_bytes_per_frame() * args.batch
    achieved = bytes_launch / (r["spec_ms"] / 1e3) / 1e9
    flops_launch = projection_flops_per_frame() * args.batch
    proj_tflops = flops_launch / (r["proj_ms"] / 1e3) / 1e12
    print(f"[bench] {args.dtype}: {ms:.3f} ms/step, spectra {r['spec_ms']:.3f} ms, projection "
          f"{r['proj_ms']:.3f} ms", file=sys.stderr, flush=True)
    res = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "f32" else args.dtype,
        "data": "synthetic",
        "config": {"workload": f"{W}x{H} FP32 frames (32 blobs + 16 polygons), N_max={NMAX} (10201 moments), "
                               f"{RINGS} rings x {ANGLES} angles, batch {args.batch}",
                   "batch": args.batch, "frame": [H, W], "n_max": NMAX, "rings": RINGS, "angles": ANGLES,
                   "projection": args.dtype},
        "roofline": {"bound": "hbm", "kernel": "polar_fft_kernel (fused resample + angular FFT)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(args.batch),
                     "bytes_per_launch": bytes_launch, "avg_launch_ms": round(r["spec_ms"], 4)},
        "projection": projection_entry(args.dtype, r["proj_ms"], args.batch),
    }
    assert abs(res["projection"]["useful_tflops"] - proj_tflops) < 0.01 * proj_tflops + 0.01
    if not args.no_split and args.dtype == "f32":
        del r
        for dt, key in (("bf16x2", "split_bf16"), ("f16x2", "split_f16")):
            torch.cuda.empty_cache()
            r2 = run_gpu(args.batch, args.steps, args.warmup, dt)
            ms2 = r2["total_ms"] / args.steps
            sb = bytes_launch / (r2["spec_ms"] / 1e3) / 1e9
            res[key] = {"value": round(args.batch / (ms2 / 1e3), 2), "unit": "images/s",
                        "ms_per_step": round(ms2, 4),
                        "spectra_roofline": {"bound": "hbm", "kernel": "polar_fft_kernel",
                                             "achieved": round(sb, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                             "frac": round(sb / HBM_PEAK_GBS, 4),
                                             "avg_launch_ms": round(r2["spec_ms"], 4)},
                        "projection": projection_entry(dt, r2["proj_ms"], args.batch)}
            print(f"[bench] {dt}: {ms2:.3f} ms/step, projection {r2['proj_ms']:.3f} ms", file=sys.stderr,
                  flush=True)
            del r2
    if not args.no_batch_sweep and args.dtype == "f32":
        # the same FP32 step at other batch sizes (kernel times by HIP events, as above)
        res["batch_sweep"] = []
        for b in (1, 8, 128):
            torch.cuda.empty_cache()
            rb = run_gpu(b, args.steps, args.warmup, "f32")
            msb = rb["total_ms"] / args.steps
            res["batch_sweep"].append({"batch": b, "images_per_s": round(b / (msb / 1e3), 1),
                                       "ms_per_step": round(msb, 4), "spectra_ms": round(rb["spec_ms"], 4),
                                       "spectra_hbm_frac": round(spectra_bytes_per_frame() * b /
                                                                 (rb["spec_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                       "projection_ms": round(rb["proj_ms"], 4)})
            del rb
        print(f"[bench] batch sweep: {res['batch_sweep']}", file=sys.stderr, flush=True)
    if not args.no_two_pass and args.dtype == "f32":
        torch.cuda.empty_cache()
        res["resample_alone"] = resample_alone(args.batch, args.steps, args.warmup)
        print(f"[bench] resampler alone: {res['resample_alone']}", file=sys.stderr, flush=True)
    if not args.no_batch_form:
        torch.cuda.empty_cache()
        res["batch_form"] = batch_form(args.steps)
        print(f"[bench] batch form: {res['batch_form']}", file=sys.stderr, flush=True)
    if not args.no_recon:
        torch.cuda.empty_cache()
        res["reconstruction"] = reconstruction()
        print(f"[bench] reconstruction: {res['reconstruction']}", file=sys.stderr, flush=True)
    if not args.no_cartesian:
        torch.cuda.empty_cache()
        res["cartesian_single_moment"] = cartesian_single_moment()
        print(f"[bench] cartesian: {res['cartesian_single_moment']['roofline']}", file=sys.stderr, flush=True)
    if not args.no_stability:
        res["stability"] = stability_sweep()
        print(f"[bench] stability: {res['stability']['max']}", file=sys.stderr, flush=True)
    if not args.no_dedup:
        torch.cuda.empty_cache()
        res["dedup"] = dedup_throughput()
        print(f"[bench] dedup: {res['dedup']}", file=sys.stderr, flush=True)
    if args.requests > 0:
        torch.cuda.empty_cache()
        res["latency"] = {}
        for dt in ("f32", "bf16x2"):
            res["latency"][dt] = serving(dt, args.requests, args.qps, warmup_s=2.0)
            print(f"[bench] serving {dt}: {res['latency'][dt]}", file=sys.stderr, flush=True)
    if args.cpu_seconds > 0:
        print("[bench] timing the CPU oracle ...", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        res["cpu_baseline"]["single_thread"] = cpu_baseline_single_thread(args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
