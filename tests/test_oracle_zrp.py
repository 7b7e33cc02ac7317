"""Pins for the oracle's radial polynomials (eq. (2)) and its moment enumeration.

Each check ties the exact big-integer evaluation of eq. (2) to something
other than eq. (2) itself: closed forms, classical special cases evaluated by
independent library routines (scipy / mpmath Jacobi and Legendre), and the
orthogonality relation implied by the (n+1)/pi factor of eq. (1) together
with the reconstruction eq. (9).
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as sp

import oracle


def test_enumeration_counts_and_order():
    # Sec. 2: n >= 0, 0 <= m <= n, n - m even.  (nmax/2 + 1)^2 for even nmax.
    for nmax, expect in [(0, 1), (1, 2), (2, 4), (20, 121), (100, 2601), (200, 10201)]:
        assert oracle.num_moments(nmax) == expect
    # brute enumeration by a different route: all (n, m) in a square, filtered
    for nmax in range(0, 30):
        brute = sorted(((n, m) for n in range(nmax + 1) for m in range(nmax + 1)
                        if m <= n and (n - m) % 2 == 0))
        assert oracle.pairs(nmax) == brute
        assert oracle._lib().zmo_num_moments(nmax) == len(brute)


def test_Rnn_is_rho_power():
    g = oracle.ring_grid(64)
    plist = [(n, n) for n in range(0, 80)]
    T = oracle.zrp(plist, g)
    for row, (n, _) in zip(T, plist):
        ref = np.array([float(mpmath.mpf(r) ** n) for r in g["rho"]])
        np.testing.assert_allclose(row, ref, rtol=4e-16, atol=0)


def test_value_at_rho_one_and_zero():
    plist = oracle.pairs(200)
    at1 = oracle.zrp_rational(plist, [1, 7], 1)  # rho^2 = 1/1 and 7/1 (unused)
    assert np.all(at1[:, 0] == 1.0)  # R_nm(1) = 1
    at0 = oracle.zrp_rational(plist, [0], 5)[:, 0]
    for v, (n, m) in zip(at0, plist):
        if m > 0:
            assert v == 0.0
        else:
            assert v == (-1.0) ** (n // 2)  # R_{2k}^0(0) = (-1)^k


def test_m0_is_shifted_legendre():
    # R_{2k}^0(rho) = P_k(2 rho^2 - 1): a classical special case, checked with
    # scipy's Legendre routine.  Its argument 2 rho^2 - 1 is itself rounded,
    # and |P_k'| <= k^2, so the reference carries up to ~k^2 * 1e-16 of error.
    g = oracle.ring_grid(1080)
    ks = [0, 1, 2, 5, 17, 40, 73, 100]
    T = oracle.zrp([(2 * k, 0) for k in ks], g)
    for row, k in zip(T, ks):
        ref = sp.eval_legendre(k, 2.0 * g["rho"] ** 2 - 1.0)
        np.testing.assert_allclose(row, ref, rtol=0, atol=max(3e-14, 2.5e-16 * k * k))


def test_matches_jacobi_form_low_orders():
    # R_n^m(rho) = (-1)^k rho^m P_k^(m,0)(1 - 2 rho^2), k = (n-m)/2 (scipy).
    g = oracle.ring_grid(512)
    plist = oracle.pairs(60)
    T = oracle.zrp(plist, g)
    rho = g["rho"]
    worst = 0.0
    for row, (n, m) in zip(T, plist):
        k = (n - m) // 2
        ref = (-1) ** k * rho ** m * sp.eval_jacobi(k, m, 0, 1.0 - 2.0 * rho * rho)
        worst = max(worst, float(np.max(np.abs(row - ref))))
    assert worst < 1e-13


def test_matches_mpmath_jacobi_high_orders():
    # Independent arbitrary-precision evaluation (mpmath hypergeometric Jacobi)
    # at high order, where the factorial series is catastrophically unstable
    # in floating point (terms ~2^250 at n = 200).
    mpmath.mp.dps = 60
    g = oracle.ring_grid(1080)
    rings = [0, 1, 3, 100, 539, 540, 900, 1078, 1079]
    sub = dict(rho=g["rho"][rings], w=g["w"][rings], ax=g["ax"][rings], ay=g["ay"][rings],
               ash=g["ash"][rings], bx=g["bx"], by=g["by"], bsh=g["bsh"])
    plist = [(200, 0), (200, 2), (199, 1), (200, 100), (151, 37), (200, 198), (120, 0), (97, 3)]
    T = oracle.zrp(plist, sub)
    for row, (n, m) in zip(T, plist):
        k = (n - m) // 2
        for v, r in zip(row, rings):
            rho = mpmath.mpf(2 * r + 1) / (2 * 1080)
            ref = (-1) ** k * rho ** m * mpmath.jacobi(k, m, 0, 1 - 2 * rho * rho)
            assert abs(v - float(ref)) <= 1.2e-16 * max(1.0, abs(float(ref))), (n, m, r, v, float(ref))


def test_gauss_legendre_orthogonality():
    # int_0^1 R_nm R_n'm rho drho = delta_nn' / (2(n+1)): GL rings with
    # nmax+2 nodes integrate the degree <= 2 nmax + 1 integrand exactly.
    for nmax in (20, 100):
        g = oracle.ring_grid(nmax + 2, "gauss_legendre")
        plist = oracle.pairs(nmax)
        T = oracle.zrp(plist, g)
        worst = 0.0
        for m in range(0, nmax + 1):
            idx = [i for i, (n, mm) in enumerate(plist) if mm == m]
            ns = np.array([plist[i][0] for i in idx])
            Tm = T[idx]
            Gm = (Tm * g["w"][None, :]) @ Tm.T
            Gm = Gm * 2.0 * (ns[:, None] + 1)
            worst = max(worst, float(np.max(np.abs(Gm - np.eye(len(idx))))))
        assert worst < 1e-11, (nmax, worst)


def test_midpoint_weights_sum_to_half():
    for R in (1, 2, 32, 512, 1080):
        g = oracle.ring_grid(R)
        assert abs(math.fsum(g["w"]) - 0.5) < 1e-15


def test_bad_pair_rejected():
    with pytest.raises(ValueError):
        oracle.zrp([(3, 2)], oracle.ring_grid(4))
