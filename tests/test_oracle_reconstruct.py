"""Pins for the oracle's reconstruction checkers (eq. (9) at pixel centres and
at polar nodes, Sec. 2.2) and for its disk-pixel geometry.

These functions are the reference of every GPU reconstruction test, so they
are tied here to things other than themselves:
  * the pixel geometry against the frame convention written out by hand
    (x right, y up, radius D/2 px around ((W-1)/2, (H-1)/2), rho <= 1);
  * single moments whose basis function is a plain polynomial in x and y:
    V_11 = rho e^{j theta} = x + j y, V_00 = 1, and rho^3 e^{3 j theta} =
    (x + j y)^3 with the textbook R_7^3 = 21 rho^7 - 30 rho^5 + 10 rho^3, so a
    flipped theta, a transposed frame or a shifted pixel centre changes the
    values;
  * the moments of f = gamma + alpha x + beta y (Z_00 = gamma, Z_11 =
    (alpha - j beta) / 2), which eq. (9) must return exactly at every disk
    pixel centre;
  * the quarter-turn law: moments multiplied by (-j)^m reconstruct the image
    turned counter-clockwise (np.rot90);
  * the Neumann factor (eq. (14)-(15)) multiplied back, and the one-sided
    sum over stored m >= 0.
"""
import math

import numpy as np
import pytest

import oracle


def _xy(H, W):
    """Unit-disk coordinates of every pixel centre, written out directly."""
    D = min(H, W)
    x = np.array([[(j - (W - 1) / 2) / (D / 2) for j in range(W)] for _ in range(H)])
    y = np.array([[((H - 1) / 2 - i) / (D / 2) for _ in range(W)] for i in range(H)])
    return x, y


def _single(nmax, n, m, value):
    pl = oracle.pairs(nmax)
    Z = np.zeros(len(pl), dtype=complex)
    Z[pl.index((n, m))] = value
    return Z


@pytest.mark.parametrize("H,W", [(5, 5), (6, 9), (9, 6)])
def test_disk_pixels_geometry(H, W):
    mask, P, b, th = oracle.disk_pixels(H, W)
    D = min(H, W)
    assert b == D * D
    x, y = _xy(H, W)
    inside = x * x + y * y <= 1.0 + 1e-12
    assert np.array_equal(mask, inside)
    # P / b is rho^2 exactly: P = X^2 + Y^2 in half-pixel units
    np.testing.assert_allclose(P / b, (x * x + y * y)[mask], rtol=0, atol=1e-15)
    np.testing.assert_allclose(np.cos(th), (x / np.maximum(np.hypot(x, y), 1e-300))[mask] * (P > 0)
                               + (P == 0), rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.sin(th), (y / np.maximum(np.hypot(x, y), 1e-300))[mask] * (P > 0),
                               rtol=0, atol=1e-12)


def test_disk_pixels_named_points():
    # 5 x 5 frame: centre pixel (2, 2); top-middle (0, 2) is straight up (theta = pi/2);
    # right-middle (2, 4) has theta = 0; left-middle (2, 0) theta = pi; the corner
    # (0, 4) lies at rho^2 = 32/25 > 1, outside the disk.
    mask, P, b, th = oracle.disk_pixels(5, 5)
    idx = -np.ones((5, 5), dtype=np.int64)
    idx[mask] = np.arange(int(mask.sum()))
    assert not mask[0, 4] and not mask[4, 0]
    assert P[idx[2, 2]] == 0
    assert P[idx[0, 2]] == 16 and abs(th[idx[0, 2]] - math.pi / 2) < 1e-15
    assert P[idx[2, 4]] == 16 and abs(th[idx[2, 4]]) < 1e-15
    assert P[idx[2, 0]] == 16 and abs(abs(th[idx[2, 0]]) - math.pi) < 1e-15
    assert P[idx[4, 2]] == 16 and abs(th[idx[4, 2]] + math.pi / 2) < 1e-15


@pytest.mark.parametrize("H,W", [(17, 17), (12, 20), (21, 14)])
def test_cartesian_reconstruction_of_low_order_basis(H, W):
    nmax = 3
    x, y = _xy(H, W)
    mask, *_ = oracle.disk_pixels(H, W)
    # Z_00 = c -> f~ = c (the m = 0 term appears once)
    f = oracle.reconstruct_cartesian(_single(nmax, 0, 0, 0.75), H, W, nmax)
    np.testing.assert_allclose(f[mask], 0.75, rtol=0, atol=1e-15)
    assert np.all(f[~mask] == 0.0)
    # Z_11 = 1 -> 2 Re(x + j y) = 2 x ; Z_11 = j -> 2 Re(j (x + j y)) = -2 y
    f = oracle.reconstruct_cartesian(_single(nmax, 1, 1, 1.0), H, W, nmax)
    np.testing.assert_allclose(f[mask], 2 * x[mask], rtol=0, atol=1e-14)
    f = oracle.reconstruct_cartesian(_single(nmax, 1, 1, 1j), H, W, nmax)
    np.testing.assert_allclose(f[mask], -2 * y[mask], rtol=0, atol=1e-14)
    # one-sided sum: Re(Z_11 (x + j y)) once, no conj term
    f = oracle.reconstruct_cartesian(_single(nmax, 1, 1, 1j), H, W, nmax, one_sided=True)
    np.testing.assert_allclose(f[mask], -y[mask], rtol=0, atol=1e-14)


@pytest.mark.parametrize("H,W", [(23, 23), (16, 26)])
def test_cartesian_reconstruction_of_r73(H, W):
    # V_73 = R_7^3(rho) e^{3 j theta} = (21 rho^4 - 30 rho^2 + 10) (x + j y)^3
    nmax = 9
    x, y = _xy(H, W)
    mask, *_ = oracle.disk_pixels(H, W)
    r2 = x * x + y * y
    V = (21 * r2 * r2 - 30 * r2 + 10) * (x + 1j * y) ** 3
    for z in (1.0, 1j, 0.3 - 0.7j):
        f = oracle.reconstruct_cartesian(_single(nmax, 7, 3, z), H, W, nmax)
        np.testing.assert_allclose(f[mask], (2 * z * V).real[mask], rtol=0, atol=1e-12)


@pytest.mark.parametrize("H,W", [(19, 19), (14, 22)])
def test_cartesian_reconstruction_of_linear_frame(H, W):
    # f = gamma + alpha x + beta y has Z_00 = gamma, Z_11 = (alpha - j beta)/2 and no
    # other moment; eq. (9) returns f at every disk pixel centre.
    alpha, beta, gamma = 0.75, -1.25, 0.5
    nmax = 4
    pl = oracle.pairs(nmax)
    Z = np.zeros(len(pl), dtype=complex)
    Z[pl.index((0, 0))] = gamma
    Z[pl.index((1, 1))] = (alpha - 1j * beta) / 2
    x, y = _xy(H, W)
    mask, *_ = oracle.disk_pixels(H, W)
    f = oracle.reconstruct_cartesian(Z, H, W, nmax)
    np.testing.assert_allclose(f[mask], (gamma + alpha * x + beta * y)[mask], rtol=0, atol=1e-12)
    # Neumann-normalised moments (Z_00 / 2) reconstruct the same image
    Zn = Z.copy()
    Zn[pl.index((0, 0))] /= 2
    fn = oracle.reconstruct_cartesian(Zn, H, W, nmax, neumann=True)
    np.testing.assert_allclose(fn, f, rtol=0, atol=1e-14)


@pytest.mark.parametrize("N", [15, 16])
def test_cartesian_reconstruction_quarter_turn(N):
    # turning the image a quarter turn counter-clockwise multiplies Z_nm by (-j)^m
    nmax = 12
    pl = oracle.pairs(nmax)
    rng = np.random.default_rng(N)
    Z = rng.standard_normal(len(pl)) + 1j * rng.standard_normal(len(pl))
    ms = np.array([m for _, m in pl])
    Z[ms == 0] = Z[ms == 0].real
    f = oracle.reconstruct_cartesian(Z, N, N, nmax)
    fr = oracle.reconstruct_cartesian((-1j) ** ms * Z, N, N, nmax)
    np.testing.assert_allclose(fr, np.rot90(f), rtol=0, atol=1e-11)
    # up-down flip: theta -> -theta, Z -> conj(Z)
    fu = oracle.reconstruct_cartesian(np.conj(Z), N, N, nmax)
    np.testing.assert_allclose(fu, np.flipud(f), rtol=0, atol=1e-11)


def test_polar_reconstruction_closed_forms():
    # at the polar nodes (rho_r, theta_a) = ((2r+1)/(2R), 2 pi a / A):
    #   Z_11 = j -> -2 rho sin(theta);  Z_73 = 1 -> 2 R_7^3(rho) cos(3 theta)
    nmax, R, A = 8, 10, 32
    rho = (2 * np.arange(R) + 1) / (2 * R)
    th = 2 * np.pi * np.arange(A) / A
    f = oracle.reconstruct_polar(_single(nmax, 1, 1, 1j), nmax, R, A)
    np.testing.assert_allclose(f, -2 * rho[:, None] * np.sin(th)[None, :], rtol=0, atol=1e-14)
    r73 = 21 * rho ** 7 - 30 * rho ** 5 + 10 * rho ** 3
    f = oracle.reconstruct_polar(_single(nmax, 7, 3, 1.0), nmax, R, A)
    np.testing.assert_allclose(f, 2 * r73[:, None] * np.cos(3 * th)[None, :], rtol=0, atol=1e-13)
    f = oracle.reconstruct_polar(_single(nmax, 7, 3, 1.0), nmax, R, A, one_sided=True)
    np.testing.assert_allclose(f, r73[:, None] * np.cos(3 * th)[None, :], rtol=0, atol=1e-13)
    # Neumann: Z_40 / 2 with eps_0 multiplied back gives R_40 = 6 rho^4 - 6 rho^2 + 1
    r40 = 6 * rho ** 4 - 6 * rho ** 2 + 1
    f = oracle.reconstruct_polar(_single(nmax, 4, 0, 0.5), nmax, R, A, neumann=True)
    np.testing.assert_allclose(f, np.repeat(r40[:, None], A, axis=1), rtol=0, atol=1e-14)
