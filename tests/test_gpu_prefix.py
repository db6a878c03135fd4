"""GPU prefix depths (pfac_prefix_histogram) against the oracle's histogram computed from
the prefix set: random pattern sets over several alphabets, texts across many
workgroups, bytes outside the alphabet, both table forms, every cap, and edge cases."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_02272_amd.pfac as pfac  # noqa: E402
from oracle import prefix  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _gpu_hist(a, text, cap):
    h = pfac.pfac_prefix_histogram(a, torch.from_numpy(np.ascontiguousarray(text)).to(DEV), cap)
    torch.cuda.synchronize()
    return h.cpu().tolist()


@pytest.mark.parametrize("alphabet", [2, 4, 20, 52, 256])
@pytest.mark.parametrize("levels", [0, 3])
def test_random_sets(alphabet, levels):
    rng = np.random.default_rng(alphabet * 10 + levels)
    pats = [bytes(rng.integers(0, alphabet, size=int(rng.integers(1, 14))).astype(np.uint8)) for _ in range(80)]
    n = 200_000 + int(rng.integers(0, 1000))  # many workgroups, ragged end
    text = rng.integers(0, min(256, alphabet + 2), size=n).astype(np.uint8)
    for k in range(300):  # plants, so deep bins are populated
        p = pats[int(rng.integers(0, len(pats)))]
        o = int(rng.integers(0, n - len(p)))
        text[o:o + len(p)] = np.frombuffer(p, np.uint8)
    a = pfac.pfac_build(pats, alphabet, merge_levels=levels)
    sample = text[:20_000]
    for cap in (1, 5, 13, 63):
        assert _gpu_hist(a, sample, cap) == prefix.depth_histogram(pats, sample, cap)
    # the whole text: bins sum to n, and the first bins agree with the sample-free
    # definition computed on the CPU in numpy-free Python for a shorter cap
    full = _gpu_hist(a, text, 6)
    assert sum(full) == n
    assert full == prefix.depth_histogram(pats, text, 6)


def test_equal_length_patterns_and_edges():
    rng = np.random.default_rng(5)
    pats = [bytes(rng.integers(0, 4, size=20).astype(np.uint8)) for _ in range(100)]
    a = pfac.pfac_build(pats, 4)
    text = rng.integers(0, 4, size=(1 << 18) + 3).astype(np.uint8)
    for i in range(0, len(text) - 20, 20_000):
        text[i:i + 20] = np.frombuffer(pats[i % 100], np.uint8)
    h = _gpu_hist(a, text, 20)
    assert h == prefix.depth_histogram(pats, text, 20)
    assert h[20] >= len(range(0, len(text) - 20, 20_000))  # every plant reaches full depth
    assert _gpu_hist(a, text[:0], 4) == [0, 0, 0, 0, 0]
    assert _gpu_hist(a, text[:1], 4) == prefix.depth_histogram(pats, text[:1], 4)
    with pytest.raises(pfac.PfacError):
        pfac.pfac_prefix_histogram(a, torch.zeros(4, dtype=torch.uint8, device=DEV), 64)
