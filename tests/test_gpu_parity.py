"""GPU parity: keys from the HIP path, through the C ABI, equal the oracle's element by
element (bit-exact: this is integer work).

Covers the hand cases, random small cases over many alphabets (several tiles and a
ragged tail), the capacity-overflow protocol, and the full-size workloads: 1 MiB
uniform (alphabet 256, 100 patterns), 256 MiB printable (5,000 patterns) and 1 GiB
DNA (alphabet 4, 10,000 patterns)."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_02272_amd.pfac as pfac  # noqa: E402
from oracle import literal, native  # noqa: E402
from paper_1704_02272_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DEV = "cuda:0"


def _keys(pairs):
    return np.array([(s << 32) | j for s, j in pairs], dtype=np.uint64)


ALGOS = ["tiled", "plain"]


def build(pats, alphabet, algo="tiled", grid=0):
    a = pfac.pfac_build(pats, alphabet)
    pfac.pfac_set_tuning(a, algo=algo, grid=grid)
    return a


def gpu_scan(a, text_np, **kw):
    t = torch.from_numpy(np.array(text_np, dtype=np.uint8, copy=True)).to(DEV)
    k = pfac.pfac_scan(a, t, **kw)
    torch.cuda.synchronize()
    return pfac.keys_to_numpy(k)


def _hand():
    with open(os.path.join(GOLDEN, "hand_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("case", _hand(), ids=lambda c: c["name"])
def test_hand_cases(case, algo):
    pats = [bytes.fromhex(p) for p in case["patterns"]]
    text = np.frombuffer(bytes.fromhex(case["text"]), dtype=np.uint8)
    a = build(pats, case["alphabet"], algo)
    got = gpu_scan(a, text)
    assert np.array_equal(got, _keys([tuple(x) for x in case["expected"]]))


@pytest.mark.parametrize("algo", ALGOS)
def test_random_small_cases(algo):
    rng = np.random.default_rng(1234)
    for trial in range(120):
        sigma = int(rng.choice([1, 2, 3, 4, 5, 16, 32, 33, 64, 100, 256]))
        npat = int(rng.integers(1, 80))
        maxl = int(rng.choice([3, 8, 20, 70]))
        pats = [bytes(rng.integers(0, sigma, size=int(rng.integers(1, maxl + 1))).astype(np.uint8))
                for _ in range(npat)]
        n = int(rng.choice([0, 1, 7, 100, 4095, 4096, 4097, 70000, 300001]))
        hi = min(256, sigma + (2 if trial % 4 == 0 else 0))
        text = rng.integers(0, hi, size=n).astype(np.uint8)
        # plant a few patterns so matches exist at any alphabet
        for _ in range(min(20, n // 8)):
            p = pats[int(rng.integers(0, npat))]
            if len(p) <= n:
                o = int(rng.integers(0, n - len(p) + 1))
                text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
        a = build(pats, sigma, algo, grid=int(rng.choice([0, 1, 3])))
        want = native.AhoCorasick(pats, sigma).scan(text, chunk=1 << 16)
        got = gpu_scan(a, text)
        assert np.array_equal(got, want), (trial, sigma, npat, n)


@pytest.mark.parametrize("algo", ALGOS)
def test_long_patterns_past_any_halo(algo):
    rng = np.random.default_rng(5)
    base = rng.integers(0, 256, size=5000).astype(np.uint8).tobytes()
    pats = [base[:3000], base[:10], base[100:2100], b"\x00\x01"]
    text = np.frombuffer(base * 3, dtype=np.uint8).copy()
    a = build(pats, 256, algo)
    assert np.array_equal(gpu_scan(a, text), native.AhoCorasick(pats, 256).scan(text))


@pytest.mark.parametrize("algo", ALGOS)
def test_capacity_overflow_protocol(algo):
    pats = [b"a", b"aa"]
    text = np.frombuffer(b"a" * 50000, dtype=np.uint8)
    a = build(pats, 256, algo)
    t = torch.from_numpy(text.copy()).to(DEV)
    small = torch.empty(10, dtype=torch.int64, device=DEV)
    got = pfac.keys_to_numpy(pfac.pfac_scan(a, t, keys=small))
    assert len(got) == 50000 + 49999
    assert np.array_equal(got, literal.keys(literal.match_set(pats, text.tobytes())))


def test_async_count_and_no_patterns():
    a = pfac.pfac_build([b"xyz"], 256)
    t = torch.from_numpy(np.frombuffer(b"..xyz..xyz", dtype=np.uint8).copy()).to(DEV)
    keys = torch.empty(16, dtype=torch.int64, device=DEV)
    cnt = torch.full((1,), -1, dtype=torch.int64, device=DEV)
    pfac.pfac_scan_async(a, t, keys, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 2
    assert list(pfac.keys_to_numpy(keys[:2])) == [(2 << 32), (7 << 32)]
    e = pfac.pfac_build([], 256)
    pfac.pfac_scan_async(e, t, keys, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0


@pytest.mark.parametrize("algo", ALGOS)
def test_uniform_1mib_full(algo):
    w = W.uniform_256()
    a = build(w.patterns, 256, algo)
    got = gpu_scan(a, w.text)
    assert np.array_equal(got, native.brute(w.patterns, w.text))


@pytest.mark.timeout(600)
def test_printable_256mib_full_and_repeatable():
    w = W.printable_256()
    a = build(w.patterns, 256, "tiled")
    want = native.AhoCorasick(w.patterns, 256).scan(w.text)
    t = torch.from_numpy(w.text).to(DEV)
    got1 = pfac.keys_to_numpy(pfac.pfac_scan(a, t))
    got2 = pfac.keys_to_numpy(pfac.pfac_scan(a, t))
    # 4 KiB spans: 65,536 spans, past the direct-prefix limit, so the placement takes
    # blocks by ticket and finds their offsets by decoupled look-back
    pfac.pfac_set_tuning(a, span_log2=12)
    got4 = pfac.keys_to_numpy(pfac.pfac_scan(a, t))
    got5 = pfac.keys_to_numpy(pfac.pfac_scan(a, t))
    pfac.pfac_set_tuning(a)  # and back to direct placement on the same workspace
    got6 = pfac.keys_to_numpy(pfac.pfac_scan(a, t))
    assert np.array_equal(got6, want)
    pfac.pfac_set_tuning(a, algo="plain")
    got3 = pfac.keys_to_numpy(pfac.pfac_scan(a, t))
    assert np.array_equal(got4, want) and np.array_equal(got5, want)
    assert np.array_equal(got3, want)
    assert np.array_equal(got1, want)
    assert np.array_equal(got2, want)
    # brute force on sampled windows (the definition, independent of the automaton)
    rng = np.random.default_rng(0)
    for _ in range(8):
        o = int(rng.integers(0, len(w.text) - (1 << 16)))
        win = w.text[o:o + (1 << 16) + w.max_len - 1]
        b = native.brute(w.patterns, win)
        b = b[(b >> np.uint64(32)) < (1 << 16)] + np.uint64(o << 32)
        lo, hi = np.uint64(o << 32), np.uint64((o + (1 << 16)) << 32)
        assert np.array_equal(got1[(got1 >= lo) & (got1 < hi)], b)


@pytest.mark.timeout(900)
def test_dna_1gib_full():
    w = W.dna_4()
    a = build(w.patterns, 4, "tiled")
    want = native.AhoCorasick(w.patterns, 4).scan(w.text)
    got = gpu_scan(a, w.text, keys=torch.empty(len(want) + 16, dtype=torch.int64, device=DEV))
    assert np.array_equal(got, want)


def test_grid_sizes_and_repeats_agree():
    """Metamorphic: the persistent grid size (1, 2, 7, auto) and repeated launches on a
    reused workspace leave the keys unchanged (look-back, ticket and epoch reuse)."""
    w = W.printable_256(text_bytes=6 << 20, n_patterns=3000, plant_block=1 << 12)
    want = native.AhoCorasick(w.patterns, 256).scan(w.text)
    t = torch.from_numpy(w.text).to(DEV)
    for grid in (1, 2, 7, 0, 0):
        a = build(w.patterns, 256, "tiled", grid)
        for _ in range(2):
            assert np.array_equal(pfac.keys_to_numpy(pfac.pfac_scan(a, t)), want), grid
        torch.cuda.synchronize()
