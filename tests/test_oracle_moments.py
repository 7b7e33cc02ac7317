"""Pins for the oracle's moments (eq. (1), eq. (14)), the Cartesian pixel sum
(eq. (6)), resampler, reconstruction (eq. (9)) and error measures (eq. (12),
(13)).

The checks use closed forms (constant and linear frames), exact symmetry laws
of eq. (1) (rotation / flip phase laws, conjugate symmetry of Sec. 2),
orthogonality on Gauss-Legendre rings, linearity, and the Neumann factor of
eq. (15) as an exact halving of m = 0.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_constant_frame():
    # f = c over the whole frame: f^ = c on every polar node, so by eq. (1)
    # Z_00 = (1/pi)(2 pi / A) sum_r w_r A c = 2 c sum_r w_r = c (sum w = 1/2),
    # Z_{n, m>0} = 0, and Z_{n,0} = c 2 (n+1) sum_r w_r R_n0(rho_r).
    c = 0.625
    f = np.full((40, 56), c)
    nmax, R, A = 12, 20, 64
    Z = oracle.moments(f, nmax, R, A)
    pl = oracle.pairs(nmax)
    assert abs(Z[0] - c) < 1e-15
    g = oracle.ring_grid(R)
    for z, (n, m) in zip(Z, pl):
        if m > 0:
            assert abs(z) < 1e-14
        elif n > 0:
            resid = c * 2 * (n + 1) * float(np.sum(g["w"] * oracle.zrp([(n, 0)], g)[0]))
            assert abs(z - resid) < 1e-14
    # on Gauss-Legendre rings the radial residual vanishes for n > 0.  The
    # outermost GL node sits at rho ~ 0.997, so the frame must be large enough
    # (rho_max * D/2 <= D/2 - 1/2) for all its bilinear taps to be in-frame.
    f = np.full((1000, 1000), c)
    Zgl = oracle.moments(f, nmax, nmax + 2, A, rule="gauss_legendre")
    assert abs(Zgl[0] - c) < 1e-14
    assert np.max(np.abs(Zgl[1:])) < 1e-13


def test_linear_frame_pins_resampler_geometry():
    # f = gamma + alpha x + beta y in unit-disk coordinates (x right, y up,
    # radius D/2 px around ((W-1)/2, (H-1)/2)).  Bilinear interpolation is
    # exact for it, so f^(rho, theta) = gamma + rho (alpha cos + beta sin), and
    #   Z_00 = gamma,  Z_11 = 2 (alpha - j beta) sum_r w_r rho_r^2,
    #   Z_{n,m} = 0 for m >= 2.
    H, W = 30, 44
    D = min(H, W)
    alpha, beta, gamma = 0.75, -1.25, 0.5
    jj, ii = np.meshgrid(np.arange(W), np.arange(H))
    x = (jj - (W - 1) / 2) / (D / 2)
    y = ((H - 1) / 2 - ii) / (D / 2)
    f = gamma + alpha * x + beta * y
    nmax, R, A = 9, 15, 32
    Z = oracle.moments(f, nmax, R, A)
    pl = oracle.pairs(nmax)
    s3 = sum(Fraction(2 * r + 1, 2 * R) ** 3 / R for r in range(R))  # sum_r w_r rho_r^2, exactly
    assert abs(Z[pl.index((0, 0))] - gamma) < 1e-14
    z11 = 2 * (alpha - 1j * beta) * float(s3)
    assert abs(Z[pl.index((1, 1))] - z11) < 1e-14
    for z, (n, m) in zip(Z, pl):
        if m >= 2:
            assert abs(z) < 1e-13


def test_polar_basis_functions_on_gl_rings():
    # f^ = R_n'm'(rho) cos(m' theta)  ->  Z_n'm' = 1 (m' = 0) or 1/2 (m' > 0);
    # f^ = R_n'm'(rho) sin(m' theta)  ->  Z_n'm' = -j/2 (sign of exp(-j m theta));
    # every other moment is 0 (orthogonality on GL rings, A > 2 nmax).
    nmax, A = 14, 64
    g = oracle.ring_grid(nmax + 2, "gauss_legendre")
    pl = oracle.pairs(nmax)
    T = oracle.zrp(pl, g)
    th = 2 * np.pi * np.arange(A) / A
    for (n1, m1) in [(0, 0), (4, 0), (5, 3), (14, 14), (13, 1)]:
        i1 = pl.index((n1, m1))
        for kind in ("cos", "sin"):
            if kind == "sin" and m1 == 0:
                continue
            ang = np.cos(m1 * th) if kind == "cos" else np.sin(m1 * th)
            fhat = T[i1][:, None] * ang[None, :]
            Z = oracle.moments_polar(fhat, pl, g)
            expect = np.zeros(len(pl), dtype=complex)
            if kind == "cos":
                expect[i1] = 1.0 if m1 == 0 else 0.5
            else:
                expect[i1] = -0.5j
            assert np.max(np.abs(Z - expect)) < 1e-12, (n1, m1, kind)
            # Neumann (eq. (14)-(15)): only m = 0 changes, halved
            Zn = oracle.moments_polar(fhat, pl, g, neumann=True)
            e2 = expect.copy()
            e2[[i for i, (n, m) in enumerate(pl) if m == 0]] /= 2
            assert np.max(np.abs(Zn - e2)) < 1e-12


@pytest.mark.parametrize("square", [48, 33])
def test_rotation_and_flip_phase_laws(square):
    # Rotating the image by +90 deg (np.rot90, counter-clockwise) maps
    # f(rho, theta) -> f(rho, theta - pi/2), hence Z_nm -> (-j)^m Z_nm.
    # Up-down flip: theta -> -theta, Z -> conj(Z).  Left-right flip:
    # theta -> pi - theta, Z -> (-1)^m conj(Z).  Exact on a square frame with
    # A divisible by 4 (the polar grid maps onto itself).
    f = synth.make_frame(synth.FrameSpec(square, square, blobs=5, polygons=2, dtype="float64"), seed=11)
    nmax, R, A = 16, 24, 64
    pl = oracle.pairs(nmax)
    ms = np.array([m for _, m in pl])
    Z = oracle.moments(f, nmax, R, A)
    Zr = oracle.moments(np.rot90(f), nmax, R, A)
    np.testing.assert_allclose(Zr, (-1j) ** ms * Z, rtol=0, atol=1e-13)
    Zud = oracle.moments(np.flipud(f), nmax, R, A)
    np.testing.assert_allclose(Zud, np.conj(Z), rtol=0, atol=1e-13)
    Zlr = oracle.moments(np.fliplr(f), nmax, R, A)
    np.testing.assert_allclose(Zlr, (-1.0) ** ms * np.conj(Z), rtol=0, atol=1e-13)
    # |Z_nm| is invariant under the exact 90-degree rotations
    np.testing.assert_allclose(np.abs(Zr), np.abs(Z), rtol=0, atol=1e-13)


def test_neumann_halves_m0_exactly_and_linearity():
    f = synth.config_frame(1)
    g2 = synth.make_frame(synth.FrameSpec(64, 64, blobs=3, dtype="float64"), seed=99)
    pl = oracle.pairs(20)
    Z = oracle.moments(f, 20, 32, 128)
    Zn = oracle.moments(f, 20, 32, 128, neumann=True)
    for z, zn, (n, m) in zip(Z, Zn, pl):
        if m == 0:
            assert zn == z / 2
        else:
            assert zn == z
    Zg = oracle.moments(g2, 20, 32, 128)
    Zc = oracle.moments(0.5 * f - 1.5 * g2, 20, 32, 128)
    assert _rel(Zc, 0.5 * Z - 1.5 * Zg) < 1e-14


def test_only_the_disk_footprint_is_read():
    # Samples lie at radius <= D/2 - 1/2 px (outermost midpoint ring), and a
    # bilinear tap is at most sqrt(2) px from its sample, so pixels whose
    # centre is farther than D/2 + 1.5 px from the disk centre are never read:
    # filling them with NaN must leave every moment finite and unchanged.
    for H, W in [(16, 16), (20, 31)]:
        f = synth.make_frame(synth.FrameSpec(H, W, blobs=3, polygons=1, zero_outside=False,
                                             dtype="float64"), seed=5)
        D = min(H, W)
        X = np.arange(W) - (W - 1) / 2
        Y = (H - 1) / 2 - np.arange(H)
        far = np.hypot(X[None, :], Y[:, None]) > D / 2 + 1.5
        assert far.any()
        g = f.copy()
        g[far] = np.nan
        Z = oracle.moments(f, 8, D // 2, 32)
        Zg = oracle.moments(g, 8, D // 2, 32)
        assert np.all(np.isfinite(Zg))
        assert np.array_equal(Z, Zg)


def test_reconstruction_inverts_moments_on_gl_rings():
    # Build f^ from eq. (9) with chosen moments (n <= 10) and recover them
    # with eq. (1): the pair is exact up to rounding on GL rings, A > 2 nmax.
    nmax, A = 10, 32
    R = nmax + 2
    pl = oracle.pairs(nmax)
    rng = np.random.default_rng(3)
    Z0 = rng.standard_normal(len(pl)) + 1j * rng.standard_normal(len(pl))
    for i, (n, m) in enumerate(pl):
        if m == 0:
            Z0[i] = Z0[i].real  # real image -> Z_n0 real
    g = oracle.ring_grid(R, "gauss_legendre")
    tab = oracle.zrp(pl, g)
    th = 2 * np.pi * np.arange(A) / A
    fhat = oracle.reconstruct(Z0, nmax, np.repeat(tab, A, axis=1), np.tile(th, R)).reshape(R, A)
    Z1 = oracle.moments_polar(fhat, pl, g)
    assert np.max(np.abs(Z1 - Z0)) < 1e-12
    # Neumann-normalised moments reconstruct the same image (eps_m multiplied back)
    eps = np.array([2.0 if m == 0 else 1.0 for _, m in pl])
    fhat_n = oracle.reconstruct(Z0 / eps, nmax, np.repeat(tab, A, axis=1), np.tile(th, R),
                                neumann=True).reshape(R, A)
    assert np.max(np.abs(fhat_n - fhat)) < 1e-12


def test_cartesian_sum_is_close_at_low_order():
    # eq. (3)+(5) is a different discretisation: agreement is approximate.
    f = synth.config_frame(1)
    Zp = oracle.moments(f, 8, 32, 128)
    Zc = oracle.cartesian(f, 8)
    assert _rel(Zc, Zp) < 5e-2
    assert abs(Zc[0] - Zp[0]) / abs(Zp[0]) < 2e-2


def test_recon_error_eq13():
    f = np.array([[0.0, 2.0], [1.0, 4.0]])
    mask = np.array([[True, True], [True, False]])
    r = oracle.recon_error(f, f, mask)
    assert r["eps13"] == 0.0
    r = oracle.recon_error(f, np.zeros_like(f), mask)
    # sum over disk of f^2 = 0 + 4 + 1 = 5; f_max = 2; count = 3
    assert abs(r["eps13"] - 5.0 / (4.0 * 3)) < 1e-15
    assert abs(r["eps10"] - 1.0) < 1e-15
    # eq. (12) over the disk pixels with f != 0: (2 - 0)^2 / 4 + (1 - 0)^2 / 1 = 2;
    # the disk pixel with f = 0 is left out (the one outside the disk never counts)
    assert abs(r["eps12"] - 2.0) < 1e-15 and r["zeros"] == 1
    r = oracle.recon_error(f, 0.5 * f, mask)
    # every non-zero pixel is off by half of itself: 2 pixels x 1/4
    assert abs(r["eps12"] - 0.5) < 1e-15 and r["zeros"] == 1


def _disk_sums(N):
    # integer pixel-centre coordinates X = 2j - (N-1), Y = (N-1) - 2i (units of half a pixel)
    X = 2 * np.arange(N, dtype=np.int64) - (N - 1)
    Y = (N - 1) - 2 * np.arange(N, dtype=np.int64)
    XX, YY = np.meshgrid(X, Y)
    inside = XX * XX + YY * YY <= N * N
    return XX, YY, inside


@pytest.mark.parametrize("N", [16, 17])
def test_cartesian_moment_closed_forms(N):
    # eq. (6) with Delta = 2/N on the unit disk: closed forms from integer pixel sums
    XX, YY, inside = _disk_sums(N)
    d2 = (2.0 / N) ** 2
    cnt = int(inside.sum())
    one = inside.astype(np.float64)
    z00 = oracle.cartesian_moment(one, 0, 0)
    assert abs(z00 - d2 * cnt / math.pi) <= 1e-14 * abs(z00)
    assert abs(oracle.cartesian_moment(one, 0, 0, neumann=True) - z00 / 2) <= 1e-15
    # R_20 = 2 rho^2 - 1, rho^2 = P / N^2
    sP = int((XX * XX + YY * YY)[inside].sum())
    z20 = oracle.cartesian_moment(one, 2, 0)
    assert abs(z20 - 3.0 / math.pi * d2 * (2.0 * sP / N ** 2 - cnt)) <= 1e-13
    # rho e^{-j theta} = (X - jY) / N: the x and y coordinate images give
    # Z_11 = (2/pi) Delta^2 sum X^2 / N^2 and -j (2/pi) Delta^2 sum Y^2 / N^2
    sX2 = int((XX * XX)[inside].sum())
    zx = oracle.cartesian_moment(np.where(inside, XX / N, 0.0), 1, 1)
    zy = oracle.cartesian_moment(np.where(inside, YY / N, 0.0), 1, 1)
    ref = 2.0 / math.pi * d2 * sX2 / N ** 2
    assert abs(zx - ref) <= 1e-13 * ref and abs(zy + 1j * ref) <= 1e-13 * ref


@pytest.mark.parametrize("N", [12, 13])
def test_cartesian_moment_quarter_turn(N):
    # rotating the content a quarter turn counter-clockwise multiplies Z_nm by (-j)^m
    f = np.random.default_rng(N).normal(size=(N, N))
    for n, m in [(1, 1), (2, 2), (3, 1), (5, 3), (8, 4), (6, 0)]:
        z = oracle.cartesian_moment(f, n, m)
        zr = oracle.cartesian_moment(np.rot90(f), n, m)
        assert abs(zr - z * (-1j) ** m) <= 1e-12 * (1 + abs(z)), (n, m)
