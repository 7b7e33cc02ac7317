"""Pins from values the paper prints.

Table I (Sec. 3) lists a 5x5 segment of a reconstruction before and after
the per-band min-max renormalisation.  The reading taken for that step (an
affine map per band, positive slope) must reproduce the printed normalised
values from the printed raw ones up to the integer rounding of both.
"""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_minmax.txt")


def _load():
    d = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        d[k] = np.array(v, dtype=float)
    return d


def test_table1_minmax_is_affine_per_band():
    d = _load()
    for band in ("red", "green", "blue"):
        raw, nrm = d["raw_" + band], d["norm_" + band]
        assert raw.size == 25 and nrm.size == 25
        ok = raw > 0  # printed zeros are clipped negatives
        A = np.vstack([raw[ok], np.ones(ok.sum())]).T
        (slope, icpt), *_ = np.linalg.lstsq(A, nrm[ok], rcond=None)
        assert slope > 0
        assert np.max(np.abs(A @ [slope, icpt] - nrm[ok])) < 0.75, band


def test_oracle_minmax_matches_affine_reading():
    rng = np.random.default_rng(0)
    f = rng.uniform(10, 250, size=(9, 9))
    ft = 40.0 * f - 3000.0 + rng.normal(0, 1e-9, size=f.shape)
    mask = np.ones_like(f, dtype=bool)
    out = oracle.minmax(ft, f, mask)
    assert abs(out.min() - f.min()) < 1e-9 and abs(out.max() - f.max()) < 1e-9
    np.testing.assert_allclose(out, f, atol=1e-6)
