"""GPU parity for eq. (9) reconstruction, eq. (13) error, min-max renormalisation
and the Sec. 3 embedding, against the FP64 oracle.  The same moments are fed
to both sides (they come from the oracle or from a seeded generator)."""
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


def _z_tensor(Z, dtype):
    return torch.from_numpy(np.stack([Z.real, Z.imag], -1).astype(dtype)).cuda()


def _rand_moments(nmax, seed):
    pl = oracle.pairs(nmax)
    rng = np.random.default_rng(seed)
    Z = (rng.standard_normal(len(pl)) + 1j * rng.standard_normal(len(pl))) / (1 + np.arange(len(pl))) ** 0.5
    for i, (n, m) in enumerate(pl):
        if m == 0:
            Z[i] = Z[i].real
    return Z


@pytest.mark.parametrize("neumann", [False, True])
def test_polar_reconstruction_matches_oracle(zm, neumann):
    nmax, R, A = 24, 40, 64
    Z = _rand_moments(nmax, 1)
    plan = zm.Plan(nmax, 80, 80, dtype="f64", rings=R, angles=A, neumann=neumann)
    g = zm.reconstruct(plan, _z_tensor(Z, np.float64), kind="polar").cpu().numpy()
    o = oracle.reconstruct_polar(Z, nmax, R, A, neumann=neumann)
    assert np.max(np.abs(g - o)) <= 1e-12 * np.max(np.abs(o))
    g1 = zm.reconstruct(plan, _z_tensor(Z, np.float64), kind="polar", one_sided=True).cpu().numpy()
    o1 = oracle.reconstruct_polar(Z, nmax, R, A, one_sided=True)
    assert np.max(np.abs(g1 - o1)) <= 1e-12 * np.max(np.abs(o1))


def test_cartesian_reconstruction_matches_oracle(zm):
    nmax, H, W = 40, 70, 90
    Z = _rand_moments(nmax, 2)
    plan = zm.Plan(nmax, H, W, dtype="f64")
    g = zm.reconstruct(plan, _z_tensor(Z, np.float64), kind="cartesian").cpu().numpy()
    o = oracle.reconstruct_cartesian(Z, H, W, nmax)
    assert np.max(np.abs(g - o)) <= 1e-11 * np.max(np.abs(o))
    mask, *_ = oracle.disk_pixels(H, W)
    assert np.all(g[~mask] == 0)
    # FP32 plan: FP32 moments in, FP64 accumulation, FP32 out
    p32 = zm.Plan(nmax, H, W, dtype="f32")
    g32 = zm.reconstruct(p32, _z_tensor(Z, np.float32), kind="cartesian").cpu().numpy()
    o32 = oracle.reconstruct_cartesian(Z.astype(np.complex64).astype(np.complex128), H, W, nmax)
    assert np.max(np.abs(g32 - o32)) <= 1e-6 * np.max(np.abs(o32))


def test_cartesian_reconstruction_full_size_sampled(zm):
    # 3840 x 2160 FP32 plan at N_max 200, the size and launch the benchmark
    # times: sampled pixels (centre, disk edge, random) against eq. (9) with
    # the exact R_nm; pixels outside the disk are exactly 0
    H, W, nmax = 2160, 3840, 200
    D = min(H, W)
    Z = _rand_moments(nmax, 9)
    plan = zm.Plan(nmax, H, W, dtype="f32")
    g = zm.reconstruct(plan, _z_tensor(Z, np.float32), kind="cartesian").cpu().numpy()
    rng = np.random.default_rng(9)
    ii = np.concatenate([rng.integers(0, H, 96), [H // 2, H // 2 - 1, 0, H - 1, H // 2, H // 2, 0, H - 1]])
    jj = np.concatenate([rng.integers(0, W, 96),
                         [W // 2, W // 2 - 1, W // 2, W // 2 - 1, W // 2 + D // 2 - 1, W // 2 - D // 2, 0, W - 1]])
    X = 2 * jj - (W - 1)
    Y = (H - 1) - 2 * ii
    P = X * X + Y * Y
    inside = P <= D * D
    assert 40 <= inside.sum() < len(ii)
    assert np.all(g[ii[~inside], jj[~inside]] == 0)
    Rv = oracle.zrp_rational(oracle.pairs(nmax), P[inside].astype(np.int64), D * D)
    o = oracle.reconstruct(Z.astype(np.complex64).astype(np.complex128), nmax, Rv,
                           np.arctan2(Y[inside], X[inside]).astype(np.float64))
    assert np.max(np.abs(g[ii[inside], jj[inside]] - o)) <= 1e-6 * np.max(np.abs(o))


@pytest.mark.parametrize("n,m", [(200, 0), (200, 2), (199, 1), (200, 100), (255, 3), (180, 180)])
def test_cartesian_high_order_basis_function(zm, n, m):
    # a single moment Z_nm = 1 reconstructs c_m R_nm(rho) cos(m theta): checks the
    # Jacobi recurrence against the exact eq. (2) at high order
    nmax = max(n, 1)
    H = W = 96
    pl = oracle.pairs(nmax)
    Z = np.zeros(len(pl), dtype=complex)
    Z[pl.index((n, m))] = 1.0
    plan = zm.Plan(nmax, H, W, dtype="f64")
    g = zm.reconstruct(plan, _z_tensor(Z, np.float64), kind="cartesian").cpu().numpy()
    mask, P, b, th = oracle.disk_pixels(H, W)
    sel = np.arange(0, P.size, 37)
    Rv = oracle.zrp_rational([(n, m)], P[sel], b)[0]
    expect = (1.0 if m == 0 else 2.0) * Rv * np.cos(m * th[sel])
    assert np.max(np.abs(g[mask][sel] - expect)) <= 1e-9


def test_round_trip_error_and_minmax(zm):
    H = W = 128
    f = synth.make_frame(synth.FrameSpec(H, W, blobs=6, polygons=0, noise=False), seed=8)
    nmax = 40
    plan = zm.Plan(nmax, H, W, dtype="f32", rings=nmax + 2, angles=128, rule="gauss_legendre")
    ft = torch.from_numpy(f)[None].cuda()
    Z = plan.moments(ft)
    rec = zm.reconstruct(plan, Z, kind="cartesian")
    err = zm.recon_error(plan, ft, rec)[0]
    Zo = zm.as_complex(Z)[0].cpu().numpy().astype(np.complex128)
    reco = oracle.reconstruct_cartesian(Zo, H, W, nmax)
    mask, *_ = oracle.disk_pixels(H, W)
    ref = oracle.recon_error(f.astype(np.float64), reco, mask)
    assert abs(err["eps13"] - ref["eps13"]) <= 1e-6 * ref["eps13"] + 1e-12
    assert abs(err["eps10"] - ref["eps10"]) <= 1e-6 * ref["eps10"] + 1e-12
    assert err["count"] == int(mask.sum())
    assert abs(err["eps12"] - ref["eps12"]) <= 1e-6 * ref["eps12"] + 1e-12
    assert err["zeros"] == ref["zeros"]
    assert err["eps13"] < 0.01  # smooth content is well captured at order 40
    mm = zm.reconstruct(plan, Z, kind="cartesian", minmax_ref=ft).cpu().numpy()[0]
    mmo = oracle.minmax(reco, f.astype(np.float64), mask)
    assert np.max(np.abs(mm - mmo)) <= 1e-5 * np.max(np.abs(mmo))
    assert abs(mm[mask].min() - f[mask].min()) < 1e-5 and abs(mm[mask].max() - f[mask].max()) < 1e-5


def test_error_measures_with_zero_pixels(zm):
    # eq. (12) leaves out the disk pixels where f = 0; eq. (10)/(13) keep them
    H, W = 96, 80
    plan = zm.Plan(10, H, W, dtype="f32")
    rng = np.random.default_rng(21)
    f = rng.uniform(0.5, 2.0, size=(H, W)).astype(np.float32)
    f[30:50, 20:45] = 0.0                       # a zero block inside the disk
    g = (f + rng.normal(0.0, 0.05, size=(H, W))).astype(np.float32)
    err = zm.recon_error(plan, torch.from_numpy(f).cuda(), torch.from_numpy(g).cuda())[0]
    mask, *_ = oracle.disk_pixels(H, W)
    ref = oracle.recon_error(f.astype(np.float64), g.astype(np.float64), mask)
    assert ref["zeros"] == 500 and err["zeros"] == ref["zeros"]
    for k in ("eps12", "eps13", "eps10"):
        assert abs(err[k] - ref[k]) <= 1e-12 * abs(ref[k]), k


def test_neumann_moments_reconstruct_same_image(zm):
    H = W = 64
    f = synth.make_frame(synth.FrameSpec(H, W, blobs=5), seed=3)
    t = torch.from_numpy(f)[None].cuda()
    outs = []
    for neu in (False, True):
        plan = zm.Plan(20, H, W, dtype="f32", neumann=neu)
        outs.append(zm.reconstruct(plan, plan.moments(t), kind="cartesian").cpu().numpy())
    assert np.max(np.abs(outs[0] - outs[1])) <= 1e-6 * np.max(np.abs(outs[0]))


def test_embed(zm):
    x = torch.rand(2, 256, 256, device="cuda")
    y = zm.embed(x)
    assert y.shape == (2, 382, 382)
    assert torch.equal(y[:, 63:63 + 256, 63:63 + 256], x)
    y2 = y.clone()
    y2[:, 63:63 + 256, 63:63 + 256] = 0
    assert float(y2.abs().max()) == 0.0
