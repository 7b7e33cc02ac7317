"""zm_moments_static (the entry point that allocates nothing: its spectra
workspace is the library's static device scratch) against zm_moments on the
same frames, through the C ABI: bit-identical moments on two calls in a row
in one process, the second with a smaller input (so the scratch holds the
first call's data when the second starts), for the FP32 projection and for
the split-FP16 one (whose per-frame scale slots sit at a batch-dependent
offset in the scratch and must be cleared by each call); a batch beyond the
scratch is refused with ZM_EINVAL and leaves the output untouched."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_14492_amd as m
    return m


def _frames(H, W, n, seed):
    fs = [synth.make_frame(synth.FrameSpec(H, W, blobs=8, polygons=4, zero_outside=False), seed + i)
          for i in range(n)]
    return torch.from_numpy(np.stack(fs)).cuda()


def _static(zm, plan, frames, out):
    B = frames.shape[0]
    return zm._lib.zm_moments_static(plan.handle, zm._vp(frames.data_ptr()), B, plan.H * plan.W,
                                     zm._vp(out.data_ptr()), None)


def _reference(zm, plan, frames):
    B = frames.shape[0]
    out = torch.empty(B, plan.num_moments, 2, device="cuda")
    ws = plan.workspace(B)
    st = zm._lib.zm_moments(plan.handle, zm._vp(frames.data_ptr()), B, plan.H * plan.W, zm._vp(out.data_ptr()),
                            zm._vp(ws.data_ptr()), ws.numel(), None)
    assert st == zm.ZM_OK
    return out


@pytest.mark.parametrize("dtype", ["f32", "f16x2"])
@pytest.mark.parametrize("H,W,nmax,b1,b2", [(2160, 3840, 200, 19, 5), (1024, 1024, 100, 40, 3)])
def test_static_scratch_matches_workspace_entry_point(zm, dtype, H, W, nmax, b1, b2):
    plan = zm.Plan(nmax, H, W, dtype=dtype)
    assert zm._lib.zm_static_scratch_bytes() == 32 << 20
    assert plan.workspace_size(b1) <= 32 << 20 < plan.workspace_size(b1 + 1) or H == 1024
    big = _frames(H, W, b1, seed=300)
    small = _frames(H, W, b2, seed=400)
    for frames in (big, small):  # second call smaller: the scratch holds the first call's spectra
        B = frames.shape[0]
        print(f"static scratch: {dtype} {H}x{W} n_max {nmax} batch {B}", flush=True)
        out = torch.full((B, plan.num_moments, 2), float("nan"), device="cuda")
        assert _static(zm, plan, frames, out) == zm.ZM_OK
        ref = _reference(zm, plan, frames)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (dtype, B)


def test_static_scratch_refuses_oversized_batch(zm):
    plan = zm.Plan(200, 2160, 3840, dtype="f32")
    fit = 1
    while plan.workspace_size(fit + 1) <= zm._lib.zm_static_scratch_bytes():
        fit += 1
    frames = torch.zeros(fit + 1, 2160, 3840, device="cuda")
    out = torch.full((fit + 1, plan.num_moments, 2), 7.0, device="cuda")
    st = _static(zm, plan, frames, out)
    assert st == zm.ZM_EINVAL
    assert f"at most {fit} frames" in zm._lib.zm_last_error().decode()
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
    # the largest batch that fits still runs
    assert _static(zm, plan, frames[:fit], out[:fit]) == zm.ZM_OK
    torch.cuda.synchronize()
    assert bool(torch.all(torch.isfinite(out[:fit])))
