"""Batched persistent form: mixed frame sizes and orders in one launch.
Each frame's moments must equal the standalone path bit for bit (same kernel
code per item) and match the FP64 oracle within the FP32 gate."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_14492_amd as m
    return m


def _frames(specs):
    out = []
    for side, nmax, seed in specs:
        f = synth.make_frame(synth.FrameSpec(side, side, blobs=8, polygons=0, noise=True), seed=seed)
        out.append(torch.from_numpy(f).cuda())
    return out


def _plans(zm, specs, dtype="f32"):
    cache = {}
    plans = []
    for side, nmax, _ in specs:
        key = (side, nmax)
        if key not in cache:
            cache[key] = zm.Plan(nmax, side, side, dtype=dtype)
        plans.append(cache[key])
    return plans


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dtype", ["f32", "bf16x2", "f16x2"])
def test_small_mixed_batch_bit_exact(zm, dtype):
    specs = [(256, 30, 1), (384, 50, 2), (256, 30, 3), (512, 100, 4), (768, 50, 5), (384, 50, 6), (256, 100, 7)]
    frames = _frames(specs)
    plans = _plans(zm, specs, dtype)
    outs = zm.moments_batch(plans, frames)
    torch.cuda.synchronize()
    for p, f, z in zip(plans, frames, outs):
        ref = p.moments(f)
        torch.cuda.synchronize()
        assert torch.equal(z.cpu(), ref.cpu())


def test_config4_batch_graph_autotune(zm):
    specs = synth.batch_sides(64, seed=4)
    frames = _frames(specs)
    plans = _plans(zm, specs)
    b = zm.Batch(plans, frames, autotune=True, graph=True)
    cfg = b.config()
    assert cfg["n_items"] > 0 and (cfg["grid"] > 0) == (cfg["route"] == "persistent")
    b.run()
    b.check()
    ref = [p.moments(f) for p, f in zip(plans, frames)]
    torch.cuda.synchronize()
    first = [z.clone() for z in b.outs]
    for z, r in zip(first, ref):
        assert torch.equal(z, r)
    # graph replays with eager work in between give the same result every time
    for rep in range(3):
        for z in b.outs:
            z.fill_(float("nan"))
        _ = torch.randn(1 << 20, device="cuda").sum()
        b.run()
        torch.cuda.synchronize()
        for z, r in zip(b.outs, first):
            assert torch.equal(z, r), rep
    b.check()
    # oracle spot checks on the largest and a small frame
    order = sorted(range(len(specs)), key=lambda i: -specs[i][0])
    for i in [order[0], order[-1]]:
        side, nmax, _ = specs[i]
        Zo = oracle.moments(frames[i].cpu().numpy().astype(np.float64), nmax, plans[i].rings, plans[i].angles)
        Z = zm.as_complex(first[i]).cpu().numpy()
        assert _rel(Z, Zo) <= 1e-5, (side, nmax)
    # new frames through the same batch
    new = [torch.flip(f, dims=[0]).contiguous() for f in frames]
    b.update(new)
    b.run()
    torch.cuda.synchronize()
    for k in range(0, len(new), 9):
        r = plans[k].moments(new[k])
        torch.cuda.synchronize()
        assert torch.equal(b.outs[k], r)
    b.close()


@pytest.mark.parametrize("graph", [True, False])
def test_per_plan_route_bit_exact(zm, graph):
    """ZM_BATCH_PER_PLAN: each plan's frames (slices of one tensor per plan, jobs
    interleaved across plans) run as the standalone launches; the moments equal
    zm_moments bit for bit, after an update to other strided frames too, and a
    batch whose new frames are not at one stride returns to the persistent
    kernel with the same results."""
    kinds = [(256, 30, "f32"), (384, 50, "f16x2"), (320, 40, "bf16x2")]
    counts = [3, 2, 1]
    plans, stacks = [], []
    for (side, nmax, dt), n in zip(kinds, counts):
        plans.append(zm.Plan(nmax, side, side, dtype=dt))
        st = torch.stack([torch.from_numpy(synth.make_frame(synth.FrameSpec(side, side, blobs=6, noise=True),
                                                            seed=31 * side + k)) for k in range(n)]).cuda()
        stacks.append(st)
    order = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
    jplans = [plans[g] for g, _ in order]
    jframes = [stacks[g][k] for g, k in order]
    b = zm.Batch(jplans, jframes, graph=graph, per_plan=True)
    assert b.config()["route"] == "per_plan"
    b.run()
    b.check()
    torch.cuda.synchronize()
    for p, f, z in zip(jplans, jframes, b.outs):
        assert torch.equal(z, p.moments(f))
    # other strided frames: still per-plan launches
    flipped = [torch.flip(st, dims=[1]).contiguous() for st in stacks]
    b.update([flipped[g][k] for g, k in order])
    assert b.config()["route"] == "per_plan"
    for z in b.outs:
        z.fill_(float("nan"))
    b.run()
    torch.cuda.synchronize()
    for (g, k), z in zip(order, b.outs):
        assert torch.equal(z, plans[g].moments(flipped[g][k]))
    # frames no longer at one stride (the first plan's at frame offsets 0, 1
    # and 3 of one buffer): the persistent kernel, same bits
    side0 = kinds[0][0]
    buf = torch.empty(4, side0, side0, device="cuda")
    slots = [0, 1, 3]
    for k in range(3):
        buf[slots[k]].copy_(stacks[0][k])
    loose = [buf[slots[k]] if g == 0 else stacks[g][k] for g, k in order]
    b.update(loose)
    assert b.config()["route"] == "persistent"
    for z in b.outs:
        z.fill_(float("nan"))
    b.run()
    b.check()
    torch.cuda.synchronize()
    for p, f, z in zip(jplans, loose, b.outs):
        assert torch.equal(z, p.moments(f))
    b.close()


def test_tuner_times_per_plan_route(zm):
    """On a homogeneous batch of strided frames the tuner also times the
    per-plan launches; whichever it keeps, the moments equal zm_moments."""
    plan = zm.Plan(60, 512, 512, dtype="f32")
    st = torch.stack([torch.from_numpy(synth.make_frame(synth.FrameSpec(512, 512, blobs=6), seed=k))
                      for k in range(8)]).cuda()
    b = zm.Batch([plan] * 8, [st[k] for k in range(8)], autotune=True)
    cfg = b.config()
    assert cfg["route"] in ("persistent", "per_plan")
    b.run()
    b.check()
    ref = plan.moments(st)
    torch.cuda.synchronize()
    for k in range(8):
        assert torch.equal(b.outs[k], ref[k])
    b.close()


_TUNE_SCRIPT = r"""
import json, sys, torch
import paper_2304_14492_amd as zm
import synth
plan = zm.Plan(40, 320, 320, dtype="f32")
st = torch.stack([torch.from_numpy(synth.make_frame(synth.FrameSpec(320, 320, blobs=4), seed=k))
                  for k in range(4)]).cuda()
b = zm.Batch([plan] * 4, [st[k] for k in range(4)], autotune=True)
b.run()
b.check()
ok = all(torch.equal(b.outs[k], plan.moments(st[k])) for k in range(4))
print(json.dumps(dict(b.config(), ok=ok)))
"""


def _tune_run(tmp_path, cache):
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, ZM_TUNE_CACHE=str(cache), PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", _TUNE_SCRIPT], cwd=root, env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_tune_cache_file_routes(zm, tmp_path):
    """ZM_TUNE_CACHE: a tuned batch appends '<grid> <order> <route> <signature>';
    a later process takes its shape from the file, in that form or in the
    older two-field form (persistent kernel), and the moments stay exact."""
    cache = tmp_path / "tune.txt"
    first = _tune_run(tmp_path, cache)
    assert first["ok"]
    lines = [ln for ln in cache.read_text().splitlines() if ln.strip()]
    assert len(lines) == 1
    grid, order, route, sig = lines[0].split(" ", 3)
    assert int(grid) > 0 and order in ("0", "1") and route in ("0", "1") and sig.startswith("gfx")
    # the file's choice is taken as written: per-plan launches, item order 1
    cache.write_text(f"{grid} 1 1 {sig}\n")
    forced = _tune_run(tmp_path, cache)
    assert forced["ok"] and forced["route"] == "per_plan" and forced["grid"] == 0 and forced["order"] == 1
    # the two-field form names a persistent-kernel shape
    cache.write_text(f"384 1 {sig}\n")
    old = _tune_run(tmp_path, cache)
    assert old["ok"] and old["route"] == "persistent" and old["grid"] == 384 and old["order"] == 1


@pytest.mark.parametrize("specs", [
    [(192, 20, 11)],                    # one small frame: fewer tiles than the 8 queue ranges
    [(192, 20, 12), (320, 40, 13)],     # two plans, a few tiles each
])
def test_batch_fewer_tiles_than_ranges(zm, specs):
    # Most stage-1 ranges are empty: workgroups take tiles from other ranges
    # or go straight to the projection items, whose wait must still end with
    # every group's tiles released; replays reset the queue counters.
    frames = _frames(specs)
    plans = _plans(zm, specs)
    b = zm.Batch(plans, frames, graph=True)
    assert b.config()["n_items"] < 64
    ref = [p.moments(f) for p, f in zip(plans, frames)]
    torch.cuda.synchronize()
    for rep in range(4):
        for z in b.outs:
            z.fill_(float("nan"))
        b.run()
        torch.cuda.synchronize()
        for z, r in zip(b.outs, ref):
            assert torch.equal(z, r), rep
    b.check()
    b.close()


def test_batch_wait_bound_reports_error(zm, monkeypatch):
    # Failure handling forced from the host: with a bound of 0 polls, the
    # first projection item that finds its group's tiles still running stops
    # waiting and raises the error flag (the kernel finishes normally).  One
    # 4K frame has 540 tiles over 512 workgroups, so projection items start
    # while the last tiles run.
    monkeypatch.setenv("ZM_BATCH_SPIN_LIMIT", "0")
    plan = zm.Plan(200, 2160, 3840, dtype="f32", rings=1080, angles=4096)
    f = torch.rand(2160, 3840, device="cuda")
    b = zm.Batch([plan], [f], graph=False)
    b.run()
    with pytest.raises(zm.ZmError) as e:
        b.check()
    assert e.value.status == zm.ZM_EDEVICE
    b.close()
    # with the default bound the same batch is fine
    monkeypatch.delenv("ZM_BATCH_SPIN_LIMIT")
    b = zm.Batch([plan], [f], graph=False)
    b.run()
    b.check()
    ref = plan.moments(f)
    torch.cuda.synchronize()
    assert torch.equal(b.outs[0], ref)
    b.close()


def test_batch_rejects_unsupported(zm):
    f = torch.zeros(64, 64, device="cuda", dtype=torch.float64)
    p = zm.Plan(10, 64, 64, dtype="f64")
    with pytest.raises(zm.ZmError) as e:
        zm.moments_batch([p], [f])
    assert e.value.status == zm.ZM_EUNSUPPORTED
    p2 = zm.Plan(10, 64, 64, dtype="f32")  # angles 256 < 512
    with pytest.raises(zm.ZmError):
        zm.moments_batch([p2], [torch.zeros(64, 64, device="cuda")])


@pytest.mark.parametrize("dtype", ["f32", "f16x2"])
def test_caller_workspace_batch_bit_exact(zm, dtype):
    # zm_moments_batch_ws: the same batch in caller-owned device memory, twice
    # in a row in one workspace (the second with fewer jobs), on a side stream
    specs = [(256, 30, 11), (512, 100, 12), (256, 30, 13), (384, 50, 14), (1024, 50, 15)]
    frames = _frames(specs)
    plans = _plans(zm, specs, dtype)
    outs = [torch.empty(p.num_moments, 2, device="cuda") for p in plans]
    need = zm.batch_workspace_size(plans, frames, outs)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        zm.moments_batch(plans, frames, outs, workspace=ws[:need - 1])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        zm.moments_batch(plans, frames, outs, workspace=ws, stream=s)
        k = 3
        outs2 = [torch.full((p.num_moments, 2), float("nan"), device="cuda") for p in plans[:k]]
        zm.moments_batch(plans[:k], frames[:k], outs2, workspace=ws, stream=s)
    torch.cuda.synchronize()
    ref = [p.moments(f) for p, f in zip(plans, frames)]
    torch.cuda.synchronize()
    for z, r in zip(outs, ref):
        assert torch.equal(z, r)
    for z, r in zip(outs2, ref[:k]):
        assert torch.equal(z, r)


@pytest.mark.parametrize("dtype", ["f32", "bf16x2"])
def test_async_launches_bit_exact(zm, dtype):
    # zm_moments_batch_async: three mixed launches in flight on two streams
    # (the second and third reuse nothing of the first), each checked through
    # its staging buffer once its stream has passed it
    specs = [(256, 30, 31), (512, 100, 32), (384, 50, 33), (1024, 50, 34), (256, 30, 35), (768, 100, 36)]
    frames = _frames(specs)
    plans = _plans(zm, specs, dtype)
    ref = [p.moments(f) for p, f in zip(plans, frames)]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for s in (s1, s2):
        s.wait_stream(torch.cuda.current_stream())
    runs = []
    for s, sel in ((s1, [0, 1, 2]), (s2, [3, 4, 5]), (s1, [5, 0, 3, 1])):
        with torch.cuda.stream(s):
            bl = zm.BatchLaunch([plans[i] for i in sel], [frames[i] for i in sel], stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        runs.append((bl, ev, sel))
    for bl, ev, sel in runs:
        ev.synchronize()
        bl.check()
        for z, i in zip(bl.outs, sel):
            assert torch.equal(z, ref[i]), (dtype, i)


def test_async_launch_arguments(zm):
    specs = [(256, 30, 41), (512, 50, 42)]
    frames = _frames(specs)
    plans = _plans(zm, specs)
    with pytest.raises(ValueError):  # staging buffer not pinned
        zm.BatchLaunch(plans, frames, stage=torch.empty(1 << 20, dtype=torch.uint8))
    outs = [torch.empty(p.num_moments, 2, device="cuda") for p in plans]
    jobs = zm._jobs(plans, frames, outs)
    n = zm._sz()
    assert zm._lib.zm_batch_stage_size(jobs, 2, zm.ctypes.byref(n)) == zm.ZM_OK
    stage = torch.zeros(n.value, dtype=torch.uint8, pin_memory=True)
    ws = torch.empty(zm.batch_workspace_size(plans, frames, outs), dtype=torch.uint8, device="cuda")
    # too small a staging buffer is refused before anything is enqueued
    assert zm._lib.zm_moments_batch_async(jobs, 2, ws.data_ptr(), ws.numel(), stage.data_ptr(), n.value - 1,
                                          None) == zm.ZM_EINVAL
    # a buffer that no launch has written is not a staging buffer
    assert zm._lib.zm_batch_stage_status(stage.data_ptr()) == zm.ZM_EINVAL


def test_async_launch_reports_wait_bound(zm, monkeypatch):
    # the error flag of a run comes back through the staging buffer: with a
    # bound of 0 polls a projection item that finds a 4K frame's tiles still
    # running gives up (the kernel finishes normally)
    monkeypatch.setenv("ZM_BATCH_SPIN_LIMIT", "0")
    plan = zm.Plan(200, 2160, 3840, dtype="f32", rings=1080, angles=4096)
    f = torch.rand(2160, 3840, device="cuda")
    bl = zm.BatchLaunch([plan], [f])
    torch.cuda.synchronize()
    with pytest.raises(zm.ZmError) as e:
        bl.check()
    assert e.value.status == zm.ZM_EDEVICE
    monkeypatch.delenv("ZM_BATCH_SPIN_LIMIT")
    bl = zm.BatchLaunch([plan], [f])
    torch.cuda.synchronize()
    bl.check()
    ref = plan.moments(f)
    torch.cuda.synchronize()
    assert torch.equal(bl.outs[0], ref)


def test_destroy_reports_busy(zm):
    # a plan with work in flight, or with a batch built on it, is not freed
    plan = zm.Plan(100, 1024, 1024, dtype="f32")
    x = torch.rand(4, 1024, 1024, device="cuda")
    out = torch.empty(4, plan.num_moments, 2, device="cuda")
    ws = plan.workspace(4)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        torch.cuda._sleep(200_000_000)  # keeps the stream busy for tens of milliseconds
        plan.moments(x, out=out, workspace=ws, stream=s)
    assert zm._lib.zm_destroy(plan.handle) == zm.ZM_EBUSY
    s.synchronize()
    b = zm.Batch([plan], [x[0]], graph=False)
    assert zm._lib.zm_destroy(plan.handle) == zm.ZM_EBUSY
    b.run()
    b.check()
    b.close()
    ref = plan.moments(x[:1])
    torch.cuda.synchronize()
    assert torch.equal(b.outs[0], ref[0])
    plan.close()
    assert plan.handle is None
