"""The per-band rounding-error model (tests/errmodel.py) against a CPU
simulation of the same arithmetic.

The simulation rounds exactly where the GPU path rounds: FP32 samples, an
FP32 FFT of two rings packed as one complex sequence (numpy's single-precision
transform), operands rounded to FP32 or split into hi + lo bfloat16 / half
parts (half parts scaled per row and per frame by powers of two), three
products for the split forms, and sequential FP32 accumulation in steps of 4
rings (FP32) or 32 rings (split forms).  The model must bound the simulated
error of every n-band within its gate, and must not be loose by more than a
factor of 50 either (so the per-band gates stay meaningful).
"""
import numpy as np
import pytest

import errmodel
import oracle
import synth


def _bf16(x):
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _split(x, kind):
    x = np.asarray(x, dtype=np.float32)
    if kind == "bf16x2":
        h = _bf16(x)
        lo = _bf16(x - h)
    else:
        h = x.astype(np.float16).astype(np.float32)
        lo = (x - h).astype(np.float16).astype(np.float32)
    return h.astype(np.float64), lo.astype(np.float64)


def _acc32(P, K):
    acc = np.zeros(P.shape[0], dtype=np.float32)
    for k in range(0, P.shape[1], K):
        acc = (acc + P[:, k:k + K].sum(axis=1).astype(np.float32)).astype(np.float32)
    return acc.astype(np.float64)


def _simulate(frame, nmax, R, A, kind):
    grid = oracle.ring_grid(R)
    pl = oracle.pairs(nmax)
    table = oracle.zrp(pl, grid)
    fhat = oracle.resample(frame, R, A, grid["rho"]).astype(np.float32)
    X = np.fft.fft((fhat[0::2] + 1j * fhat[1::2]).astype(np.complex64), axis=1)
    assert X.dtype == np.complex64
    k = np.arange(nmax + 1)
    Xm, Xn = X[:, k], np.conj(X[:, (-k) % A])
    F = np.empty((R, nmax + 1), dtype=np.complex64)
    F[0::2], F[1::2] = 0.5 * (Xm + Xn), (Xm - Xn) / 2j
    ns = np.array([n for n, _ in pl])
    ms = np.array([m for _, m in pl])
    T = (2.0 * (ns + 1) / A)[:, None] * grid["w"][None, :] * table
    Fm = F.T[ms]
    if kind == "f32":
        T32 = T.astype(np.float32)
        pr = (T32 * Fm.real).astype(np.float32).astype(np.float64)
        pi = (T32 * Fm.imag).astype(np.float32).astype(np.float64)
        return _acc32(pr, 4) + 1j * _acc32(pi, 4)
    rs, fs = np.ones(len(pl)), 1.0
    if kind == "f16x2":
        mx = np.abs(T).max(axis=1)
        rs = 2.0 ** (14 - np.floor(np.log2(np.where(mx > 0, mx, 1.0))))
        fs = 2.0 ** (13 - np.floor(np.log2(max(np.abs(Fm.real).max(), np.abs(Fm.imag).max()))))
    th, tl = _split(T * rs[:, None], kind)
    out = []
    for part in (Fm.real, Fm.imag):
        fh, fl = _split(part * fs, kind)
        out.append(_acc32(np.concatenate([th * fh, th * fl, tl * fh], axis=1), 32))
    return (out[0] + 1j * out[1]) / rs / fs


@pytest.mark.parametrize("kind", ["f32", "bf16x2", "f16x2"])
def test_error_model_bounds_simulated_rounding(kind):
    frame = synth.make_frame(synth.FrameSpec(256, 256, blobs=8, polygons=4), seed=21).astype(np.float64)
    nmax, R, A = 60, 128, 256
    ref = errmodel.reference(frame, nmax, R, A)
    Z = _simulate(frame, nmax, R, A, kind)
    rows = errmodel.band_table(Z, ref, kind)
    print(kind)
    print(errmodel.format_table(rows))
    ratios = [r[4] for r in rows]
    assert max(ratios) <= errmodel.GATE_SIGMAS, rows
    assert min(ratios) >= errmodel.GATE_SIGMAS / 400, rows
