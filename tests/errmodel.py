"""Rounding-error model of the moment path, for per-n-band parity gates.

Test infrastructure: built from the FP64 oracle's intermediate quantities
(the polar image f^ of Sec. 2.5, the ring spectra F_r[m] and the radial
table of eq. (2)), never from the GPU path.

A moment is Z_nm = sum_r T_r F_r[m] with the folded operand
T_r = 2 (n+1) / (A eps_m) w_r R_nm(rho_r) (eq. (1) / (14), the 2 pi / A of
the angular sum and the 1/pi folded in) and the unnormalised ring spectrum
F_r[m] = sum_a f^(rho_r, theta_a) exp(-2 pi i m a / A).  The GPU forms it
with these roundings, each modelled as an independent error of zero mean:

  * spectrum: bilinear resampling in FP32 (fraction and three blends) and a
    length-A FP32 FFT over two real rings packed as one complex sequence.
    Each bin of ring r then carries an error of variance
    k_fft u^2 ||x_pair(r)||^2, where x_pair is the ring pair's samples,
    u = 2^-24 and k_fft = 2 log2(A) (about 2/3 u^2 per level of additions,
    4 u^2 for each of the three twiddle stages, plus the resampling);
  * operands: every product T_r F_r carries a relative error of RMS
    u_p = 2^-24 (FP32: T rounded from FP64, product rounding),
    2^-16 (hi + lo bfloat16 parts of both operands and the dropped lo*lo
    term: each part keeps 8 significant bits, so |x - hi - lo| <= 2^-16 |x|
    and |lo_T lo_F| <= 2^-16 |T F|) or 2^-22 (hi + lo half parts, 11 bits
    each);
  * accumulation: s sequential FP32 additions into one accumulator (one per
    MFMA: K = 4 rings for FP32, 32 rings times three products for the split
    forms), each rounding the running sum: variance u^2/3 per step times the
    running sum's square, bounded by s (P^2 + |Z|^2) / 3 in total.

So for each moment
  sigma^2 = u_p^2 P^2 + k_fft u^2 S^2 + u^2 s (P^2 + |Z|^2) / 3,
  P^2 = sum_r |T_r F_r[m]|^2,  S^2 = sum_r T_r^2 ||x_pair(r)||^2,
and for a band of moments sigma_band^2 = sum of sigma^2 over the band.  The
errors are sums of many independent roundings, so the band's error norm sits
near sigma_band; the gates allow GATE_SIGMAS times it.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

GATE_SIGMAS = 5.0
U32 = 2.0 ** -24
U_PRODUCT = {"f32": 2.0 ** -24, "bf16x2": 2.0 ** -16, "f16x2": 2.0 ** -22}


def reference(frame, nmax, R, A, neumann=False, rule="midpoint", table=None):
    """FP64 oracle moments of eq. (1) plus the per-moment scales of the model.
    Returns dict(Z=[M] complex, P2, S2 [M], ns, ms, A, R)."""
    grid = oracle.ring_grid(R, rule)
    pl = oracle.pairs(nmax)
    if table is None:
        table = oracle.zrp(pl, grid)
    fhat = oracle.resample(np.asarray(frame, dtype=np.float64), R, A, grid["rho"])
    mlist = list(range(nmax + 1))
    G = oracle.angular_dft(fhat, mlist)  # [R][M]
    Z = oracle.radial_sum(G, mlist, pl, A, table, grid["w"], neumann)
    ns = np.array([n for n, _ in pl])
    ms = np.array([m for _, m in pl])
    eps = np.where((ms == 0) & bool(neumann), 2.0, 1.0)
    T = (2.0 * (ns + 1) / (A * eps))[:, None] * grid["w"][None, :] * table  # [M][R]
    ring_e = np.sum(fhat * fhat, axis=1)
    pair_e = ring_e.copy()
    for r in range(0, R - 1, 2):  # rings (2k, 2k+1) share one complex transform
        pair_e[r] = pair_e[r + 1] = ring_e[r] + ring_e[r + 1]
    F = G.T[ms]  # [M][R] complex
    P2 = np.sum(np.abs(T * F) ** 2, axis=1)
    S2 = (T * T) @ pair_e
    return dict(Z=Z, P2=P2, S2=S2, ns=ns, ms=ms, A=A, R=R)


def sigma(ref, dtype):
    """Per-moment standard deviation of the GPU's rounding error."""
    A, R = ref["A"], ref["R"]
    Rp = -(-R // 32) * 32
    steps = Rp // 4 if dtype == "f32" else 3 * (Rp // 32)
    kfft = 2.0 * math.log2(A)
    up = U_PRODUCT[dtype]
    z2 = np.abs(ref["Z"]) ** 2
    var = up * up * ref["P2"] + kfft * U32 * U32 * ref["S2"] + U32 * U32 * steps * (ref["P2"] + z2) / 3.0
    return np.sqrt(var)


def band_table(Z, ref, dtype, width=20):
    """Per n-band rows: (n_lo, n_hi, error / band norm, error / total norm,
    error / sigma_band).  The last column is what the gate bounds."""
    Zo = ref["Z"]
    ns = ref["ns"]
    sg = sigma(ref, dtype)
    tot = float(np.linalg.norm(Zo))
    nmax = int(ns.max())
    rows = []
    for b in range(nmax // width + 1):
        sel = (ns // width) == b
        d = float(np.linalg.norm(Z[sel] - Zo[sel]))
        bn = float(np.linalg.norm(Zo[sel]))
        sb = float(np.sqrt(np.sum(sg[sel] ** 2)))
        rows.append((b * width, min(nmax, b * width + width - 1), d / max(bn, 1e-300), d / tot,
                     d / max(sb, 1e-300)))
    return rows


def format_table(rows):
    return "\n".join(f"   n {lo:3d}-{hi:3d}: band-rel {eb:.2e}  total-rel {et:.2e}  err/sigma {es:.3f}"
                     for lo, hi, eb, et, es in rows)
