"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Gates (relative L2 over the whole complex moment vector, m >= 0):
  FP32 projection          <= 1e-5
  split BF16 / FP16        <= 1e-4
  FP64 (small frames)      <= 1e-11
and, for the precision forms, per n-band (bands of 20 orders): the band's
error norm within errmodel.GATE_SIGMAS standard deviations of the rounding
error that tests/errmodel.py derives for that dtype.
Radial table (eq. (7), FP64 on the GPU) vs exact eq. (2): <= 1e-11 absolute.
Index/layout is checked bit-exactly through these comparisons: every moment
is compared at its canonical position.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import errmodel  # noqa: E402
import oracle  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2304_14492_amd as m
    return m


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_moments(zm, plan, frames_np):
    t = torch.from_numpy(np.ascontiguousarray(frames_np)).cuda()
    Z = plan.moments(t)
    torch.cuda.synchronize()
    return zm.as_complex(Z.double() if Z.dtype == torch.float64 else Z).cpu().numpy().astype(np.complex128)


# ---------------------------------------------------------------- tables ----
@pytest.mark.parametrize("nmax,R", [(20, 32), (100, 512), (200, 1080)])
def test_radial_table_matches_exact_series(zm, nmax, R):
    H = W = 2 * R
    plan = zm.Plan(nmax, H, W, dtype="f32")
    assert plan.rings == R
    T = plan.radial_table()
    To = oracle.zrp_table(nmax, oracle.ring_grid(R))
    err = float(np.max(np.abs(T - To)))
    print(f"table N{nmax} R{R}: max abs err {err:.3e}")
    assert err <= 1e-11


def test_ring_nodes_midpoint_bit_exact(zm):
    plan = zm.Plan(10, 64, 80, dtype="f32", rings=37)
    rho, w = plan.ring_nodes()
    g = oracle.ring_grid(37)
    assert np.array_equal(rho, g["rho"]) and np.array_equal(w, g["w"])


def test_gauss_legendre_table_orthogonality(zm):
    nmax = 60
    plan = zm.Plan(nmax, 256, 256, dtype="f32", rings=nmax + 2, rule="gauss_legendre")
    T = plan.radial_table()
    rho, w = plan.ring_nodes()
    g = oracle.ring_grid(nmax + 2, "gauss_legendre")
    np.testing.assert_allclose(rho, g["rho"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, g["w"], rtol=0, atol=1e-15)
    pl = oracle.pairs(nmax)
    worst = 0.0
    for m in range(nmax + 1):
        idx = [i for i, (n, mm) in enumerate(pl) if mm == m]
        ns = np.array([pl[i][0] for i in idx])
        G = (T[idx] * w[None, :]) @ T[idx].T * 2.0 * (ns[:, None] + 1)
        worst = max(worst, float(np.max(np.abs(G - np.eye(len(idx))))))
    assert worst < 1e-11
    To = oracle.zrp_table(nmax, g)
    assert float(np.max(np.abs(T - To))) < 1e-11


def test_high_order_table_only_plan(zm):
    # n_max = 500 on Gauss-Legendre rings: the FP64 eq. (7) table stays
    # orthonormal for every m (the paper's high-order stability claim,
    # Sec. 3.1), and sampled rows equal the exact eq. (2) values of the
    # oracle; moments beyond order 255 are reported as unsupported.
    nmax = 500
    R = nmax + 2
    plan = zm.Plan(nmax, 2048, 2048, dtype="f32", rings=R, rule="gauss_legendre")
    T = plan.radial_table()
    rho, w = plan.ring_nodes()
    pl = oracle.pairs(nmax)
    ns = np.array([n for n, _ in pl])
    ms = np.array([m for _, m in pl])
    worst = np.zeros(nmax + 1)
    for m in range(nmax + 1):
        idx = np.nonzero(ms == m)[0]
        G = (T[idx] * w[None, :]) @ T[idx].T * 2.0 * (ns[idx][:, None] + 1)
        worst[ns[idx]] = np.maximum(worst[ns[idx]], np.max(np.abs(G - np.eye(len(idx))), axis=1))
    for b in range(0, nmax + 1, 50):
        print(f"n {b:3d}-{min(nmax, b + 49):3d}: orthogonality error {worst[b:b + 50].max():.3e}")
    assert worst.max() < 1e-10
    sample = [(500, 0), (500, 2), (500, 250), (500, 500), (499, 1), (499, 263), (499, 499), (480, 96),
              (450, 200), (401, 3), (400, 398), (350, 120), (300, 100), (256, 0), (255, 255), (201, 77),
              (150, 150), (101, 51), (50, 10), (7, 3)]
    # exact eq. (2) at the plan's own nodes (an ulp of node difference moves
    # R_nm by up to n^2 ulp at order 500)
    To = oracle.zrp(sample, oracle.node_grid(rho, w))
    Tg = T[[pl.index(p) for p in sample]]
    err = float(np.max(np.abs(Tg - To)))
    print(f"sampled rows vs exact eq. (2): max abs err {err:.3e}")
    assert err <= 1e-11
    x = torch.zeros(1, 2048, 2048, device="cuda")
    with pytest.raises(zm.ZmError) as e:
        plan.moments(x)
    assert e.value.status == zm.ZM_EUNSUPPORTED


# --------------------------------------------------------------- moments ----
def test_config1_f64_and_f32(zm):
    f = synth.config_frame(1)  # 64x64 FP64, N20, 32 x 128
    Zo = oracle.moments(f, 20, 32, 128)
    p64 = zm.Plan(20, 64, 64, dtype="f64", rings=32, angles=128)
    Z = gpu_moments(zm, p64, f[None])[0]
    e64 = rel_l2(Z, Zo)
    print(f"config1 f64 rel {e64:.3e}")
    assert e64 <= 1e-11
    f32 = f.astype(np.float32)
    Zo32 = oracle.moments(f32.astype(np.float64), 20, 32, 128)
    p32 = zm.Plan(20, 64, 64, dtype="f32", rings=32, angles=128)
    Z32 = gpu_moments(zm, p32, f32[None])[0]
    e32 = rel_l2(Z32, Zo32)
    print(f"config1 f32 rel {e32:.3e}")
    assert e32 <= 1e-5


@pytest.mark.parametrize("neumann", [False, True])
@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("bf16x2", 1e-4), ("f16x2", 1e-4)])
def test_config2(zm, neumann, dtype, tol):
    f = synth.config_frame(2)  # 1024^2 FP32, N100, 512 x 1024
    ref = errmodel.reference(f.astype(np.float64), 100, 512, 1024, neumann=neumann)
    Zo = ref["Z"]
    plan = zm.Plan(100, 1024, 1024, dtype=dtype, neumann=neumann, rings=512, angles=1024)
    Z = gpu_moments(zm, plan, f[None])[0]
    e = rel_l2(Z, Zo)
    rows = errmodel.band_table(Z, ref, dtype)
    print(f"config2 {dtype} neumann={neumann} rel {e:.3e}")
    print(errmodel.format_table(rows))
    assert e <= tol
    assert max(r[4] for r in rows) <= errmodel.GATE_SIGMAS, rows


def test_neumann_halves_m0_on_gpu(zm):
    f = synth.config_frame(2)
    t = torch.from_numpy(f)[None].cuda()
    a = zm.Plan(100, 1024, 1024, dtype="f32", neumann=False).moments(t)
    b = zm.Plan(100, 1024, 1024, dtype="f32", neumann=True).moments(t)
    torch.cuda.synchronize()
    a, b = a[0].cpu().numpy(), b[0].cpu().numpy()
    pl = oracle.pairs(100)
    m0 = np.array([m == 0 for _, m in pl])
    # the folded operand differs by exactly 2 for m = 0 (power of two), so
    # the products and sums are bit-exact halves
    assert np.array_equal(b[m0], a[m0] / 2)
    assert np.array_equal(b[~m0], a[~m0])


@pytest.mark.parametrize("H,W,nmax,R,A", [
    (50, 70, 12, 25, 64),      # odd ring count, non-square, ragged ring tile
    (37, 37, 9, 18, 32),       # odd frame size, smallest A
    (200, 120, 30, 60, 256),   # ring count not a multiple of 16
    (130, 130, 63, 33, 128),   # A2 = 64, A1 = 2
    (300, 300, 7, 150, 512),   # A2 = 16, many sub-transforms
    (1024, 1024, 20, 512, 128),  # arc step up to 25x the ring step: V lane map in every angle band
])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_ragged_geometries(zm, H, W, nmax, R, A, dtype):
    f = synth.make_frame(synth.FrameSpec(H, W, blobs=5, polygons=3, zero_outside=False, dtype="float64"), seed=H * W)
    fin = f if dtype == "f64" else f.astype(np.float32)
    Zo = oracle.moments(fin.astype(np.float64), nmax, R, A)
    plan = zm.Plan(nmax, H, W, dtype=dtype, rings=R, angles=A)
    Z = gpu_moments(zm, plan, fin[None])[0]
    e = rel_l2(Z, Zo)
    assert e <= (1e-11 if dtype == "f64" else 1e-5), e


@pytest.mark.parametrize("H,W,nmax,R,A,dtype", [
    (64, 64, 0, 32, 32, "f32"),      # n_max = 0: the single moment Z_00
    (64, 64, 5, 1, 32, "f32"),       # one ring
    (2, 2, 0, 1, 32, "f64"),         # smallest frame (disk radius one pixel)
    (2, 3, 3, 1, 32, "f32"),         # smallest non-square frame
    (260, 260, 255, 130, 512, "f32"),  # the largest order the moment kernels serve
])
def test_degenerate_plans(zm, H, W, nmax, R, A, dtype):
    f = synth.make_frame(synth.FrameSpec(H, W, blobs=3, polygons=1, zero_outside=False, dtype="float64"),
                         seed=7 * H + W)
    fin = f if dtype == "f64" else f.astype(np.float32)
    Zo = oracle.moments(fin.astype(np.float64), nmax, R, A)
    plan = zm.Plan(nmax, H, W, dtype=dtype, rings=R, angles=A)
    Z = gpu_moments(zm, plan, fin[None])[0]
    assert Z.shape == Zo.shape == (zm.num_moments(nmax),)
    e = rel_l2(Z, Zo)
    assert e <= (1e-11 if dtype == "f64" else 1e-5), e


def test_gauss_legendre_moments(zm):
    f = synth.config_frame(2)
    Zo = oracle.moments(f.astype(np.float64), 60, 62, 256, rule="gauss_legendre")
    plan = zm.Plan(60, 1024, 1024, dtype="f32", rings=62, angles=256, rule="gauss_legendre")
    assert rel_l2(gpu_moments(zm, plan, f[None])[0], Zo) <= 1e-5


def test_polar_entry_point_isolates_projection(zm):
    nmax, R, A = 40, 100, 128
    rng = np.random.default_rng(4)
    fhat = rng.random((R, A))
    g = oracle.ring_grid(R)
    Zo = oracle.moments_polar(fhat, oracle.pairs(nmax), g)
    plan = zm.Plan(nmax, 256, 256, dtype="f32", rings=R, angles=A)
    Z = zm.as_complex(plan.moments_polar(torch.from_numpy(fhat.astype(np.float32)).cuda())).cpu().numpy()
    assert rel_l2(Z, oracle.moments_polar(fhat.astype(np.float32).astype(np.float64), oracle.pairs(nmax), g)) <= 1e-5
    assert rel_l2(Z, Zo) <= 1e-5


@pytest.mark.parametrize("H,W,nmax,R,A,dtype", [
    (96, 128, 20, 40, 256, "f32"),     # smallest angle count the resampler serves; ragged band
    (540, 960, 40, 270, 1024, "f32"),
    (540, 960, 40, 270, 1024, "f64"),
    (301, 257, 60, 150, 512, "bf16x2"),  # odd sizes, rings touching the frame edge
    (257, 301, 30, 77, 512, "f16x2"),
])
def test_resampler_alone(zm, H, W, nmax, R, A, dtype):
    """zm_resample_polar (Sec. 2.5) against the oracle's bilinear resample, and
    fed to zm_moments_polar it gives zm_moments' moments bit for bit."""
    B = 3
    real = np.float64 if dtype == "f64" else np.float32
    frames = np.stack([synth.make_frame(synth.FrameSpec(H, W, blobs=4, polygons=2, zero_outside=False,
                                                        dtype="float64"), seed=11 * H + W + b).astype(real)
                       for b in range(B)])
    plan = zm.Plan(nmax, H, W, dtype=dtype, rings=R, angles=A)
    dev = torch.from_numpy(frames).cuda()
    P = plan.resample_polar(dev)
    Z1 = plan.moments(dev)
    Z2 = plan.moments_polar(P)
    torch.cuda.synchronize()
    assert torch.equal(Z1, Z2), dtype
    rho = oracle.ring_grid(R)["rho"]
    Pn = P.cpu().numpy()
    for b in range(B):
        ref = oracle.resample(frames[b].astype(np.float64), R, A, rho)
        err = np.abs(Pn[b] - ref).max()
        # FP32: the fractions and the three lerps rounded in FP32
        scale = max(1.0, float(np.abs(frames[b]).max()))
        assert err <= (1e-12 if dtype == "f64" else 1e-6) * scale, (dtype, b, err)
    # frames at a stride larger than H * W (every other slice of a larger array)
    spaced = torch.zeros(2 * B, H, W, dtype=dev.dtype, device="cuda")
    spaced[::2].copy_(dev)
    Ps = plan.resample_polar(spaced[::2])
    torch.cuda.synchronize()
    assert torch.equal(Ps, P)
    with pytest.raises(RuntimeError):
        zm.Plan(10, 64, 64, dtype="f32", rings=16, angles=128).resample_polar(torch.zeros(1, 64, 64, device="cuda"))


def test_only_disk_footprint_is_read(zm):
    # NaN beyond D/2 + 1.5 px from the centre must not reach any moment.
    H, W = 540, 960
    f = synth.make_frame(synth.FrameSpec(H, W, blobs=8, polygons=4, zero_outside=False), seed=21)
    X = np.arange(W) - (W - 1) / 2
    Y = (H - 1) / 2 - np.arange(H)
    far = np.hypot(X[None, :], Y[:, None]) > min(H, W) / 2 + 1.5
    g = f.copy()
    g[far] = np.nan
    plan = zm.Plan(60, H, W, dtype="f32")
    Za = gpu_moments(zm, plan, f[None])[0]
    Zb = gpu_moments(zm, plan, g[None])[0]
    assert np.all(np.isfinite(Zb))
    assert np.array_equal(Za, Zb)


def test_batch_equals_single_bit_exact(zm):
    frames = np.stack([synth.make_frame(synth.FrameSpec(256, 256, blobs=6), seed=100 + i) for i in range(5)])
    for dtype in ["f32", "bf16x2"]:
        plan = zm.Plan(50, 256, 256, dtype=dtype)
        Zb = gpu_moments(zm, plan, frames)
        for i in range(5):
            Zi = gpu_moments(zm, plan, frames[i:i + 1])[0]
            assert np.array_equal(Zi, Zb[i]), (dtype, i)


@pytest.mark.parametrize("dtype", ["f32", "bf16x2", "f16x2", "f64"])
def test_projection_splits_bit_identical(zm, dtype):
    # N_max 100 has 138 projection items: batch 1 runs four waves per output
    # block (138 blocks), batch 128 one wave per block (8 column blocks: 1,104
    # blocks), batch 300 two waves per block (19 column blocks: 2,622 blocks);
    # the ring chunks are summed in the same order every way
    real = np.float64 if dtype == "f64" else np.float32
    base = np.stack([synth.make_frame(synth.FrameSpec(96, 96, blobs=5), seed=300 + i) for i in range(6)])
    plan = zm.Plan(100, 96, 96, dtype=dtype)
    frames = base[np.arange(300) % 6].astype(real)
    Z300 = gpu_moments(zm, plan, frames)
    Z128 = gpu_moments(zm, plan, frames[:128])
    for i in range(6):
        Z1 = gpu_moments(zm, plan, frames[i:i + 1])[0]
        assert np.array_equal(Z1, Z128[i]) and np.array_equal(Z1, Z300[i]), (dtype, i)
    for i in (127, 299):
        assert np.array_equal(Z300[i], Z300[i % 6]), (dtype, i)


def test_strided_batch_and_zero_batch(zm):
    big = np.zeros((3, 80, 100), dtype=np.float32)
    big[:, :, :90] = np.stack([synth.make_frame(synth.FrameSpec(80, 90, blobs=4), seed=s) for s in (1, 2, 3)])
    t = torch.from_numpy(big).cuda()[:, :, :90]  # row stride 100 != W: rejected
    plan = zm.Plan(16, 80, 90, dtype="f32")
    with pytest.raises(ValueError):
        plan.moments(t)
    # frames spaced by a larger image stride are fine
    buf = torch.zeros(3 * 80 * 90 + 2 * 17, device="cuda")
    ref = []
    for i in range(3):
        off = i * (80 * 90 + 17)
        buf[off:off + 80 * 90] = torch.from_numpy(big[i, :, :90].copy()).cuda().reshape(-1)
        ref.append(oracle.moments(big[i, :, :90].astype(np.float64), 16, 40, plan.angles))
    frames = torch.as_strided(buf, (3, 80, 90), (80 * 90 + 17, 90, 1))
    Z = zm.as_complex(plan.moments(frames)).cpu().numpy()
    for i in range(3):
        assert rel_l2(Z[i], ref[i]) <= 1e-5
    # batch 0 is a no-op
    out = plan.moments(torch.zeros(0, 80, 90, device="cuda"))
    assert out.shape == (0, plan.num_moments, 2)


def test_argument_errors(zm):
    with pytest.raises(zm.ZmError) as e:
        zm.Plan(20, 64, 64, angles=40)  # not a power of two
    assert e.value.status == zm.ZM_EINVAL
    with pytest.raises(zm.ZmError):
        zm.Plan(100, 64, 64, angles=128)  # A < 2 n_max + 2
    with pytest.raises(zm.ZmError):
        zm.Plan(-1, 64, 64)
    with pytest.raises(zm.ZmError):
        zm.Plan(10, 1, 64)
    plan = zm.Plan(10, 64, 64)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    x = torch.zeros(1, 64, 64, device="cuda")
    with pytest.raises(ValueError):  # the binding checks the size first
        plan.moments(x, workspace=ws)
    out = torch.empty(1, plan.num_moments, 2, device="cuda")
    st = zm._lib.zm_moments(plan.handle, zm._vp(x.data_ptr()), 1, 64 * 64, zm._vp(out.data_ptr()),
                            zm._vp(ws.data_ptr()), 16, None)
    assert st == zm.ZM_EINVAL  # and so does the library


@pytest.mark.parametrize("dtype", ["f32", "f16x2"])
def test_staged_gather_bit_identical(zm, dtype, monkeypatch):
    # the staged resample + FFT (frame pixels through LDS, plan-time windows;
    # ZM_STAGED=1 at plan creation) forms the same samples and the same
    # transform as the direct gather: bit-identical spectra and moments at 4K
    H, W = 2160, 3840
    frames = np.stack([synth.make_frame(synth.FrameSpec(H, W, blobs=8, polygons=4, zero_outside=False), 30 + i)
                       for i in range(3)])
    x = torch.from_numpy(frames).cuda()
    monkeypatch.setenv("ZM_STAGED", "1")
    ps = zm.Plan(200, H, W, dtype=dtype, rings=1080, angles=4096)
    monkeypatch.setenv("ZM_STAGED", "0")
    pd = zm.Plan(200, H, W, dtype=dtype, rings=1080, angles=4096)
    assert ps.info.resident_bytes > pd.info.resident_bytes  # the windows are resident
    wss, wsd = ps.workspace(3).zero_(), pd.workspace(3).zero_()  # unused slot bytes compare equal too
    ps.spectra(x, wss)
    pd.spectra(x, wsd)
    Zs, Zd = ps.moments(x), pd.moments(x)
    torch.cuda.synchronize()
    assert torch.equal(wss, wsd)
    assert torch.equal(Zs, Zd)
    Zo = oracle.moments(frames[0].astype(np.float64), 200, 1080, 4096)
    assert rel_l2(zm.as_complex(Zs[0]).cpu().numpy().astype(np.complex128), Zo) <= (1e-5 if dtype == "f32" else 1e-4)
