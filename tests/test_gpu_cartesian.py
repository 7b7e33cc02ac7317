"""Single moments by the Cartesian pixel sum (eq. (6), eq. (14)) on the GPU
against the FP64 oracle (exact R_nm at every pixel centre, no symmetry).

Gate: |Z_gpu - Z_oracle| <= 1e-10 * (n + 1)/pi * Delta^2 * sum |f| over the
disk, a bound on |Z| itself (|R_nm| <= 1); the kernel accumulates in FP64
and evaluates R_nm by a recurrence, so the differences are rounding only.
Sides cover odd grids (axis orbits and the centre), even grids, one and
several 32 x 32 orbit tiles with partial edges.
"""
import math

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


def _frame(N, seed):
    return np.random.default_rng(seed).random((N, N)).astype(np.float32)


def _bound(f, n):
    N = f.shape[0]
    X = 2 * np.arange(N) - (N - 1)
    Y = (N - 1) - 2 * np.arange(N)
    inside = X[None, :] ** 2 + Y[:, None] ** 2 <= N * N
    return (n + 1) / math.pi * (2.0 / N) ** 2 * float(np.abs(f[inside].astype(np.float64)).sum())


MOMENTS = [(0, 0), (1, 1), (2, 0), (7, 3), (20, 4), (60, 60), (100, 50), (200, 0), (200, 200), (201, 1)]


@pytest.mark.parametrize("N", [1, 2, 7, 64, 65, 130, 257])
def test_cartesian_moment_matches_oracle(zm, N):
    f = _frame(N, N)
    dev = torch.from_numpy(f).cuda()
    for n, m in MOMENTS:
        z = complex(zm.moment_cartesian(dev, n, m).item())
        zo = oracle.cartesian_moment(f.astype(np.float64), n, m)
        assert abs(z - zo) <= 1e-10 * _bound(f, n) + 1e-300, (N, n, m, z, zo)


def test_cartesian_negative_m_neumann_and_batch(zm):
    N = 96
    frames = [_frame(N, 100 + i) for i in range(3)]
    dev = torch.from_numpy(np.stack(frames)).cuda()
    for n, m, neu in [(10, -4, False), (12, 0, True), (33, -33, False)]:
        z = zm.moment_cartesian(dev, n, m, neumann=neu).cpu().numpy()
        for i, f in enumerate(frames):
            zo = oracle.cartesian_moment(f.astype(np.float64), n, m, neumann=neu)
            assert abs(z[i] - zo) <= 1e-10 * _bound(f, n), (n, m, neu, i)


@pytest.mark.parametrize("N", [1000, 4000])
def test_cartesian_quarter_turn_at_size(zm, N):
    # at full size, against a property that holds at any size: a quarter turn
    # counter-clockwise multiplies Z_nm by (-j)^m; plus the oracle at low order
    f = torch.rand(N, N, device="cuda", generator=torch.Generator(device="cuda").manual_seed(N))
    fr = torch.rot90(f, 1, dims=(0, 1)).contiguous()
    fh = f.cpu().numpy()
    scale = _bound(fh, 200)
    for n, m in [(3, 1), (40, 2), (200, 0), (201, 101)]:
        z = complex(zm.moment_cartesian(f, n, m).item())
        zr = complex(zm.moment_cartesian(fr, n, m).item())
        assert abs(zr - z * (-1j) ** m) <= 1e-11 * scale, (N, n, m)
    if N == 1000:
        z = complex(zm.moment_cartesian(f, 4, 2).item())
        zo = oracle.cartesian_moment(fh.astype(np.float64), 4, 2)
        assert abs(z - zo) <= 1e-10 * _bound(fh, 4)


def test_cartesian_rejects_bad_arguments(zm):
    f = torch.zeros(8, 8, device="cuda")
    for n, m in [(3, 2), (-1, 0), (501, 1), (2, 4)]:
        with pytest.raises(zm.ZmError) as e:
            zm.moment_cartesian(f, n, m)
        assert e.value.status == zm.ZM_EINVAL
