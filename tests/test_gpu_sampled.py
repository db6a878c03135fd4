"""GPU parity of the sampled prefilter form: byte patterns of four or more bytes with a
4-byte filter key, where only every second start is probed (with its 3-gram) and each
lane then checks the 4-grams of its own candidates, reading their bytes back from its
copy of the step's bytes in LDS. The edge cases of
that path, each compared element by element with the oracle: texts shorter than a step,
ragged ends, several span lengths, texts that do not start on a 16-byte boundary (the
guarded loads), matches across lane, step and span boundaries, lanes with many
candidates in one step, and spans with more matching starts than records."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_02272_amd.pfac as pfac  # noqa: E402
from oracle import native  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
STEP = 2048  # bytes a wave streams per step (64 lanes x 32 bytes)


def _sampled(a, alphabet):
    info = pfac.pfac_table_info(a)
    # the sampled form: bytes (not two-bit codes), key of four, no pattern shorter
    assert alphabet > 4 and info["filter_k"] == 4 and info["min_len"] >= 4, info


def _scan_view(a, text, off):
    """Scan `text` from a device buffer at byte offset `off` (a view that starts `off`
    bytes past a 256-byte aligned allocation)."""
    buf = torch.zeros(len(text) + 64, dtype=torch.uint8, device=DEV)
    if len(text):
        buf[off:off + len(text)] = torch.from_numpy(np.array(text, dtype=np.uint8, copy=True)).to(DEV)
    view = buf[off:off + len(text)]
    got = pfac.keys_to_numpy(pfac.pfac_scan(a, view))
    torch.cuda.synchronize()
    return got


def _patterns(rng, n, lo, hi, sigma=256):
    return [bytes(rng.integers(0, sigma, size=int(rng.integers(lo, hi + 1))).astype(np.uint8)) for _ in range(n)]


def _plant_at_boundaries(rng, text, pats):
    """Plant patterns so they start or end right at lane (32 B), step and span bounds."""
    n = len(text)
    for b in [32, 64, 2016, STEP, 2 * STEP, 4096 + 32, 1 << 14, 1 << 16, 3 << 16]:
        for d in (-5, -3, -2, -1, 0, 1, 2):
            p = pats[int(rng.integers(0, len(pats)))]
            o = b + d
            if 0 <= o and o + len(p) <= n:
                text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
            o = b + d - len(p)
            if 0 <= o and o + len(p) <= n:
                text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)


def test_sizes_offsets_and_spans():
    rng = np.random.default_rng(2101)
    pats = _patterns(rng, 80, 4, 12) + [b"abcd", b"abcde", b"bcde"]
    a = pfac.pfac_build(pats, 256)
    _sampled(a, 256)
    ac = native.AhoCorasick(pats, 256)
    sizes = [0, 1, 3, 4, 5, 31, 32, 33, 2047, 2048, 2049, 4095, 4096, 4097, 65535, 65536, 65537, 200001]
    for span in (0, 11, 12, 16):
        pfac.pfac_set_tuning(a, span_log2=span)
        for n in sizes:
            text = rng.integers(0, 256, size=n).astype(np.uint8)
            for _ in range(n // 300):
                p = pats[int(rng.integers(0, len(pats)))]
                o = int(rng.integers(0, n - len(p) + 1)) if n >= len(p) else 0
                if n >= len(p):
                    text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
            _plant_at_boundaries(rng, text, pats)
            want = ac.scan(text)
            for off in (0, 1, 3, 7, 13):
                got = _scan_view(a, text, off)
                assert np.array_equal(got, want), (span, n, off)


def test_printable_like_text_all_spans():
    """Printable bytes on both sides (many true 3-gram hits, so many candidates per step),
    a few hundred KiB, every span length the tuning allows."""
    rng = np.random.default_rng(2102)
    pats = _patterns(rng, 400, 4, 24, sigma=95)
    pats = [bytes(c + 32 for c in p) for p in pats]
    text = (rng.integers(0, 95, size=(300 << 10) + 77) + 32).astype(np.uint8)
    for _ in range(600):
        p = pats[int(rng.integers(0, len(pats)))]
        o = int(rng.integers(0, len(text) - len(p)))
        text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
    _plant_at_boundaries(rng, text, pats)
    a = pfac.pfac_build(pats, 256)
    _sampled(a, 256)
    want = native.AhoCorasick(pats, 256).scan(text)
    assert len(want) > 600
    for span in range(11, 17):
        pfac.pfac_set_tuning(a, span_log2=span)
        assert np.array_equal(_scan_view(a, text, 0), want), span
        assert np.array_equal(_scan_view(a, text, 5), want), span


def test_dense_candidates_and_record_overflow():
    """A periodic text where every start matches: every odd start of a step is a
    candidate (more than one listing window per step) and every span holds more matching
    starts than records, so placement walks the rest again."""
    pats = [b"abcd", b"bcda", b"cdab", b"dabc", b"abcdabcd", b"dabcdabcda"]
    text = np.frombuffer(b"abcd" * 100003, dtype=np.uint8).copy()
    a = pfac.pfac_build(pats, 256)
    _sampled(a, 256)
    want = native.AhoCorasick(pats, 256).scan(text)
    assert len(want) > len(text)
    for span in (11, 14, 16):
        pfac.pfac_set_tuning(a, span_log2=span)
        for off in (0, 2):
            assert np.array_equal(_scan_view(a, text, off), want), (span, off)


def test_two_terminal_starts_and_multi_id():
    """Starts that pass two terminals with one id each (two records), one terminal with
    several ids (duplicate patterns), and several terminals on one path."""
    rng = np.random.default_rng(2103)
    base = _patterns(rng, 30, 4, 6)
    pats = base + [base[0] + b"xy", base[1] + b"z", base[2], base[2] + base[3], base[4] + base[5] + b"q"]
    text = rng.integers(0, 256, size=(1 << 18) + 3).astype(np.uint8)
    for _ in range(900):
        p = pats[int(rng.integers(0, len(pats)))]
        o = int(rng.integers(0, len(text) - len(p)))
        text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
    a = pfac.pfac_build(pats, 256)
    _sampled(a, 256)
    want = native.AhoCorasick(pats, 256).scan(text)
    for span in (12, 16):
        pfac.pfac_set_tuning(a, span_log2=span)
        assert np.array_equal(_scan_view(a, text, 0), want), span
