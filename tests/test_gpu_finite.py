"""GPU: zm_count_nonfinite, the non-finite screen of the moments.

  * planted values: NaN / +Inf / -Inf written into a moment array at chosen
    positions (first, last, inside the ragged last scan block), FP32 and
    FP64: the per-frame counts equal the host's count of non-finite values;
  * frames: a NaN or Inf pixel inside the disk makes that frame's moments
    non-finite and is counted (equal to the host count of the returned
    moments); a NaN pixel beyond D/2 + 1.5 px of the centre, which the
    resampler never reads, leaves the frame's moments finite.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_14492_amd as m
    return m


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_planted_values_counted(zm, dtype):
    plan = zm.Plan(60, 96, 112, dtype=dtype)
    K = plan.num_moments
    real = torch.float64 if dtype == "f64" else torch.float32
    B = 5
    Z = torch.randn(B, K, 2, dtype=real, device="cuda")
    flat = Z.view(B, -1)
    n = flat.shape[1]
    plants = {1: [(0, float("nan"))], 2: [(n - 1, float("inf")), (n - 2, float("-inf"))],
              3: [(i, float("nan")) for i in range(0, n, 7)], 4: [(n - 3, float("nan")), (1024, float("inf"))]}
    for b, items in plants.items():
        for i, v in items:
            flat[b, i] = v
    counts = plan.count_nonfinite(Z)
    torch.cuda.synchronize()
    expect = (~torch.isfinite(Z.view(B, -1))).sum(dim=1).to(torch.int32)
    assert torch.equal(counts.cpu(), expect.cpu()), (counts.cpu(), expect.cpu())
    assert counts[0].item() == 0 and counts[3].item() == len(range(0, n, 7))
    # a second call overwrites the counts (no accumulation across calls)
    flat[1, 0] = 0.0
    plan.count_nonfinite(Z, counts=counts)
    torch.cuda.synchronize()
    assert counts[1].item() == 0


@pytest.mark.parametrize("dtype", ["f32", "bf16x2", "f64"])
def test_nonfinite_pixels_inside_disk_only(zm, dtype):
    H, W = 70, 90
    plan = zm.Plan(30, H, W, dtype=dtype)
    real = torch.float64 if dtype == "f64" else torch.float32
    rng = np.random.default_rng(5)
    frames = torch.from_numpy(rng.random((4, H, W))).to(real).cuda()
    cy, cx = (H - 1) / 2, (W - 1) / 2
    frames[1, int(cy), int(cx)] = float("nan")         # the centre pixel
    frames[2, int(cy) + 10, int(cx) - 12] = float("inf")
    frames[3, 0, 0] = float("nan")                     # corner: beyond D/2 + 1.5 px
    assert np.hypot(cx, cy) > min(H, W) / 2 + 1.5
    Z = plan.moments(frames)
    counts = plan.count_nonfinite(Z)
    torch.cuda.synchronize()
    host = (~torch.isfinite(Z.view(4, -1))).sum(dim=1).cpu().numpy()
    c = counts.cpu().numpy()
    assert np.array_equal(c, host.astype(np.int32)), (c, host)
    assert c[0] == 0 and c[3] == 0, c
    assert c[1] > 0 and c[2] > 0, c
