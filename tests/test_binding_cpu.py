"""The binding rejects buffers that do not match the plan before any pointer
crosses the ABI (no GPU needed): wrong shape, element type, layout, device
or size would otherwise become out-of-bounds device accesses."""
import pytest

torch = pytest.importorskip("torch")

import paper_2304_14492_amd as zm  # noqa: E402


def _stub_plan(dtype="f32", H=64, W=80, nmax=10):
    """A Plan object with the geometry of a real one and no library handle:
    every check below must fire before the library is called."""
    p = zm.Plan.__new__(zm.Plan)
    p._h = None
    p.dtype = dtype
    p.n_max, p.H, p.W = nmax, H, W
    p.rings, p.angles, p.num_moments = 32, 64, zm.num_moments(nmax)
    p.rings_padded, p.neumann, p.device = 32, False, 0
    p.workspace_size = lambda batch: 1000 * max(batch, 1)
    return p


def test_moments_rejects_frame_mismatches():
    p = _stub_plan()
    with pytest.raises(ValueError, match="shape"):
        p.moments(torch.zeros(2, 64, 81))
    with pytest.raises(ValueError, match="float32"):
        p.moments(torch.zeros(2, 64, 80, dtype=torch.float64))
    with pytest.raises(ValueError, match="contiguous"):
        p.moments(torch.zeros(2, 64, 160)[:, :, ::2])
    with pytest.raises(ValueError, match="CUDA"):
        p.moments(torch.zeros(2, 64, 80))
    with pytest.raises(ValueError, match="overlap"):
        p.moments(torch.zeros(64 * 80 + 5).as_strided((2, 64, 80), (5, 80, 1)))


def test_output_and_workspace_mismatches():
    p = _stub_plan()
    M = p.num_moments
    with pytest.raises(ValueError, match="dtype"):
        p._check_out(torch.zeros(3, M, 2, dtype=torch.float64), 3)
    with pytest.raises(ValueError, match="shape"):
        p._check_out(torch.zeros(2, M, 2), 3)
    with pytest.raises(ValueError, match="CUDA"):
        p._check_out(torch.zeros(3, M, 2), 3)
    with pytest.raises(ValueError, match="at least"):
        p._check_workspace(torch.zeros(2999, dtype=torch.uint8), 3)
    with pytest.raises(ValueError, match="dtype"):
        p._check_workspace(torch.zeros(3000, dtype=torch.float32), 3)
    p64 = _stub_plan("f64")
    with pytest.raises(ValueError, match="float64"):
        p64._check_out(torch.zeros(1, M, 2, dtype=torch.float32), 1)


def test_reconstruction_and_error_mismatches():
    p = _stub_plan()
    M = p.num_moments
    with pytest.raises(ValueError, match="dtype"):
        zm.reconstruct(p, torch.zeros(2, M, 2, dtype=torch.float64))
    with pytest.raises(ValueError, match="shape"):
        zm.reconstruct(p, torch.zeros(2, M + 1, 2))
    with pytest.raises(ValueError, match="kind"):
        zm.reconstruct(p, torch.zeros(2, M, 2), kind="spiral")
    with pytest.raises(ValueError, match="shape"):
        zm.recon_error(p, torch.zeros(2, 64, 80), torch.zeros(2, 64, 79))
    with pytest.raises(ValueError, match="dtype"):
        zm.recon_error(p, torch.zeros(2, 64, 80, dtype=torch.float64), torch.zeros(2, 64, 80))


def test_batch_job_mismatches():
    p = _stub_plan()
    M = p.num_moments
    with pytest.raises(ValueError, match="float32"):
        zm._jobs([p], [torch.zeros(64, 80, dtype=torch.float64)], [torch.zeros(M, 2)])
    with pytest.raises(ValueError, match="shape"):
        zm._jobs([p], [torch.zeros(64, 80)], [torch.zeros(M - 1, 2)])
    with pytest.raises(ValueError, match="float64"):
        zm._jobs([_stub_plan("f64")], [torch.zeros(64, 80)], [torch.zeros(M, 2)])
    with pytest.raises(ValueError, match="same length"):
        zm._jobs([p, p], [torch.zeros(64, 80)], [torch.zeros(M, 2)])


def test_embed_dtype():
    with pytest.raises(ValueError, match="float32 or float64"):
        zm.embed(torch.zeros(1, 8, 8, dtype=torch.int32))
