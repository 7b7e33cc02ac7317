"""The Sec. 3 embedding size, a host-side function of the library (no GPU)."""
import math
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sec3_padding.txt")


@pytest.fixture(scope="module")
def zm():
    import paper_2304_14492_amd as m
    return m


def _floor_n_sqrt2_minus_1(n):
    # floor(n (sqrt 2 - 1)) by exact integer comparison: the largest q with (q + n)^2 <= 2 n^2
    q = 0
    while (q + 1 + n) ** 2 <= 2 * n * n:
        q += 1
    return q


def test_paper_example(zm):
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        n, size, off, printed = map(int, line.split())
        assert zm.pad_size(n) == (size, off)
        assert printed == size + 1  # the paper's printed grid size is one larger than its formula


def test_formula_many_sizes(zm):
    for n in list(range(1, 300)) + [1000, 2160, 4096, 65535]:
        q = _floor_n_sqrt2_minus_1(n)
        assert zm.pad_size(n) == (n + q + 20, q // 2 + 10)
        # the whole image fits in the inscribed disk of the padded grid
        size, off = zm.pad_size(n)
        assert math.hypot(n, n) <= size
