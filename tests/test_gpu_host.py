"""GPU parity of the host-memory scan (chunks with a halo, two slots in flight) against
the oracle: chunk boundaries must neither lose nor duplicate a match."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_02272_amd.pfac as pfac  # noqa: E402
from oracle import native  # noqa: E402

pytestmark = pytest.mark.gpu


def _pairs(keys):
    keys = np.asarray(keys, dtype=np.uint64)
    return (keys >> np.uint64(32)).astype(np.uint64), (keys & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def _check(got, want_keys):
    s, j = _pairs(want_keys)
    assert len(got) == len(s)
    assert np.array_equal(got["start"], s) and np.array_equal(got["pattern_id"], j)
    assert not got["reserved"].any()


def test_chunk_boundaries_and_halo():
    rng = np.random.default_rng(21)
    pats = [bytes(rng.integers(32, 127, size=int(rng.integers(4, 48))).astype(np.uint8)) for _ in range(500)]
    n = 24 * (1 << 20) + 12345
    text = rng.integers(0, 256, size=n).astype(np.uint8)
    chunk = 1 << 20
    # a plant across every chunk end, and random ones
    for c in range(chunk, n, chunk):
        p = pats[int(rng.integers(0, len(pats)))]
        o = c - int(rng.integers(1, len(p)))
        text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
    for _ in range(3000):
        p = pats[int(rng.integers(0, len(pats)))]
        o = int(rng.integers(0, n - len(p)))
        text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
    want = native.AhoCorasick(pats, 256).scan(text)
    a = pfac.pfac_build(pats, 256)
    for cb in (chunk, 3 * chunk + 7, 0):
        _check(pfac.pfac_scan_host(a, text, chunk_bytes=cb), want)


def test_pinned_input_and_many_matches():
    rng = np.random.default_rng(22)
    pats = [bytes(rng.integers(0, 4, size=int(rng.integers(3, 7))).astype(np.uint8)) for _ in range(60)]
    n = 8 * (1 << 20) + 3
    pinned = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    text = pinned.numpy()
    text[:] = rng.integers(0, 4, size=n).astype(np.uint8)
    want = native.AhoCorasick(pats, 4).scan(text)
    assert len(want) > n // 8  # far more matches than a slot's first key buffer holds
    a = pfac.pfac_build(pats, 4)
    _check(pfac.pfac_scan_host(a, text, chunk_bytes=(1 << 20) + 1), want)
    _check(pfac.pfac_scan_host(a, np.array(text), chunk_bytes=1 << 22), want)


def test_tiny_and_empty_texts():
    a = pfac.pfac_build([b"ab", b"b", b"abc"], 256)
    assert len(pfac.pfac_scan_host(a, np.zeros(0, np.uint8))) == 0
    got = pfac.pfac_scan_host(a, np.frombuffer(b"xabcab", np.uint8), chunk_bytes=1)
    assert got["start"].tolist() == [1, 1, 2, 4, 5] and got["pattern_id"].tolist() == [0, 2, 1, 0, 1]


def test_host_scans_release_their_stream_scratch():
    # every host scan makes and destroys its own streams; the scratch the automaton keeps
    # per stream must go with them, so repeated calls hold no more of it than one did
    rng = np.random.default_rng(23)
    pats = [bytes(rng.integers(0, 256, size=int(rng.integers(4, 12))).astype(np.uint8)) for _ in range(50)]
    text = rng.integers(0, 256, size=(3 << 20) + 5).astype(np.uint8)
    a = pfac.pfac_build(pats, 256)
    want = native.AhoCorasick(pats, 256).scan(text)
    _check(pfac.pfac_scan_host(a, text, chunk_bytes=1 << 20), want)
    held = pfac.pfac_table_info(a)["stream_scratch"]
    assert held == 0
    for _ in range(5):
        _check(pfac.pfac_scan_host(a, text, chunk_bytes=1 << 20), want)
    assert pfac.pfac_table_info(a)["stream_scratch"] == held
