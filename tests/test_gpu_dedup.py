"""De-duplication by moment hashes (Sec. 2.7) through the GPU path: the
planted groups of synthetic sets are recovered exactly."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_14492_amd import dedup
    return dedup


def test_planted_groups_small(dd):
    frames, truth = synth.dedup_set(96)
    dev = torch.from_numpy(np.stack(frames)).cuda()
    groups, Z = dd.find_duplicates(dev, orders=(12, 16), rtol=1e-5)
    assert groups == truth


def test_planted_groups_mixed_set(dd):
    # 40 originals with their variants, shuffled, in chunks of 64 frames
    frames, truth = synth.dedup_set(128, n_distinct=40, seed=500)
    perm = np.random.default_rng(7).permutation(len(frames))
    inv = np.argsort(perm)
    dev = torch.from_numpy(np.stack([frames[p] for p in perm])).cuda()
    groups, _ = dd.find_duplicates(dev, orders=(16, 20), rtol=1e-5, chunk=64)
    expected = sorted(sorted(int(inv[i]) for i in g) for g in truth)
    assert groups == expected
