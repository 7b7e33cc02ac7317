"""Serving form on the GPU: requests that arrive while others run are admitted
under the HBM budget, their launches overlap on several streams, and every
result is bit-identical to computing that frame alone."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_14492_amd as m
    return m


@pytest.mark.parametrize("dtype,mode", [("f32", "per_plan"), ("bf16x2", "per_plan"), ("f32", "persistent"),
                                        ("bf16x2", "persistent")])
def test_mixed_stream_equals_alone(zm, dtype, mode):
    # per_plan: a launch per plan group; persistent: the admitted requests of
    # all sizes and orders in one persistent launch (zm_moments_batch_async)
    from paper_2304_14492_amd import serve
    reqs = serve.make_requests(48, qps=4000.0, seed=5, pool_per_size=2)
    dev = serve.GpuDevice(dtype=dtype, n_streams=4, mode=mode)
    dev.warm({(r.H, r.W, r.nmax) for r in reqs})
    budget = 1 << 30
    sch = serve.Scheduler(dev, budget, max_inflight=6, max_batch=4)
    done = serve.run_stream(reqs, sch)
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    assert sch.peak_used <= budget
    for r in done:
        p = dev.plan(r.H, r.W, r.nmax)
        alone = p.moments(r.frame.cuda()).cpu()
        assert torch.equal(alone, r.result), r.rid
    st = serve.latency_stats(done)
    assert st["count"] == len(reqs) and st["p99_ms"] >= st["p50_ms"] > 0
    # one spot check against the oracle (a 640x480 request)
    r = next(r for r in done if r.H == 480)
    p = dev.plan(r.H, r.W, r.nmax)
    Zo = oracle.moments(r.frame.numpy().astype(np.float64), r.nmax, p.rings, p.angles)
    Z = torch.view_as_complex(r.result.contiguous()).numpy()
    tol = 1e-5 if dtype == "f32" else 1e-4
    assert np.linalg.norm(Z - Zo) / np.linalg.norm(Zo) <= tol


def test_budget_limits_inflight(zm):
    from paper_2304_14492_amd import serve
    reqs = serve.make_requests(12, qps=1e6, seed=6, pool_per_size=1)
    dev = serve.GpuDevice(dtype="f32", n_streams=2)
    dev.warm({(r.H, r.W, r.nmax) for r in reqs})
    biggest = max(dev.request_bytes(r) for r in reqs)
    sch = serve.Scheduler(dev, biggest, max_inflight=4, max_batch=4)
    done = serve.run_stream(reqs, sch)
    assert len(done) == 12 and sch.peak_used <= biggest
