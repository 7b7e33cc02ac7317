"""De-duplication by moment hashes (Sec. 2.7, eq. (16)-(17)) on the CPU: the
oracle's grouping recovers the planted duplicate groups of a synthetic set
(copies, quarter / half turns, mirror images; a one-pixel-shifted decoy must
stay apart), and the library's host-side grouping (sort and sweep) gives the
same groups as the oracle's all-pairs comparison on the oracle's moments."""
import numpy as np
import pytest

import oracle
import synth

NMAX, ORDERS = 12, (8, 12)


@pytest.fixture(scope="module")
def planted():
    frames, truth = synth.dedup_set(48)
    Z = np.array([oracle.moments(f.astype(np.float64), NMAX, 24, 128) for f in frames])
    return frames, truth, Z


def test_oracle_recovers_planted_groups(planted):
    frames, truth, Z = planted
    assert oracle.dedup_groups(Z, NMAX, ORDERS, 1e-9) == truth
    # one order alone is already enough here; a vanishing tolerance keeps only exact copies
    assert oracle.dedup_groups(Z, NMAX, (12,), 1e-9) == truth
    exact = [[g[0], g[1]] for g in truth]  # original and its plain copy
    assert oracle.dedup_groups(Z, NMAX, ORDERS, 0.0) == exact


def test_host_grouping_matches_oracle(planted):
    pytest.importorskip("torch")
    from paper_2304_14492_amd import dedup
    frames, truth, Z = planted
    for rtol in (0.0, 1e-9, 1e-3):
        assert dedup.groups_from_moments(Z, ORDERS, rtol) == oracle.dedup_groups(Z, NMAX, ORDERS, rtol)
    assert dedup.groups_from_moments(Z[:1], ORDERS) == []
    assert dedup.groups_from_moments(Z[[0, 5, 7]], ORDERS, 1e-9) == []  # three distinct originals
