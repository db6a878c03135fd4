"""GPU parity of scans over the compressed trie of Section 3.2 (pfac_build_ex with
merge_levels > 0): the keys equal the oracle's element by element, at every compression
level, for single texts and packet batches, including starts that pass several
terminals inside shared blocks (their ids come from the rank of the spelled string)."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_02272_amd.pfac as pfac  # noqa: E402
from oracle import native  # noqa: E402
from paper_1704_02272_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LEVELS = [1, 3, 255]


def gpu_scan(a, text_np):
    t = torch.from_numpy(np.array(text_np, dtype=np.uint8, copy=True)).to(DEV)
    k = pfac.pfac_scan(a, t)
    torch.cuda.synchronize()
    return pfac.keys_to_numpy(k)


def _hand():
    with open(os.path.join(GOLDEN, "hand_cases.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("levels", LEVELS)
@pytest.mark.parametrize("case", _hand(), ids=lambda c: c["name"])
def test_hand_cases(case, levels):
    pats = [bytes.fromhex(p) for p in case["patterns"]]
    text = np.frombuffer(bytes.fromhex(case["text"]), dtype=np.uint8)
    a = pfac.pfac_build(pats, case["alphabet"], merge_levels=levels)
    want = np.array([(s << 32) | j for s, j in case["expected"]], dtype=np.uint64)
    assert np.array_equal(gpu_scan(a, text), want)


def _planted(rng, pats, n, sigma, k):
    text = rng.integers(0, sigma, size=n).astype(np.uint8)
    for _ in range(k):
        p = pats[int(rng.integers(0, len(pats)))]
        o = int(rng.integers(0, n - len(p)))
        text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
    return text


@pytest.mark.parametrize("levels", LEVELS)
@pytest.mark.parametrize("sigma", [4, 52])
def test_equal_length_patterns(sigma, levels):
    """The paper's compression workload: 20-symbol random patterns (Section 4.1)."""
    rng = np.random.default_rng(sigma * 7 + levels)
    pats = sorted({rng.integers(0, sigma, size=20).astype(np.uint8).tobytes() for _ in range(3000)})
    a = pfac.pfac_build(pats, sigma, merge_levels=levels)
    info = pfac.pfac_table_info(a)
    assert info["table_records"] < info["n_nodes"]
    print("sigma %d levels %d: %d nodes, %d reduced, %d records"
          % (sigma, levels, info["n_nodes"], info["reduced_nodes"], info["table_records"]), flush=True)
    text = _planted(rng, pats, (1 << 22) + 77, sigma, 4000)
    want = native.AhoCorasick(pats, sigma).scan(text)
    assert len(want) >= 3000
    assert np.array_equal(gpu_scan(a, text), want)


@pytest.mark.parametrize("levels", LEVELS)
def test_nested_terminals_in_shared_blocks(levels):
    """Patterns plus their own prefixes of the last few lengths: a start passes several
    terminals below shared_base, and duplicates share one string's rank."""
    rng = np.random.default_rng(100 + levels)
    base = sorted({rng.integers(0, 4, size=14).astype(np.uint8).tobytes() for _ in range(1500)})
    pats = base + [p[:-1] for p in base[::3]] + [p[:-2] for p in base[::5]] + base[::7]
    a = pfac.pfac_build(pats, 4, merge_levels=levels)
    text = _planted(rng, pats, (1 << 21) + 5, 4, 6000)
    want = native.AhoCorasick(pats, 4).scan(text)
    got = gpu_scan(a, text)
    assert np.array_equal(got, want), (len(got), len(want))


@pytest.mark.parametrize("levels", LEVELS)
@pytest.mark.parametrize("name", ["uniform_256", "printable_small", "dna_small"])
def test_workloads(name, levels):
    if name == "uniform_256":
        w = W.uniform_256()
    elif name == "printable_small":
        w = W.printable_256(text_bytes=(1 << 24) + 3, n_patterns=5000)
    else:
        w = W.dna_4(text_bytes=1 << 24, n_patterns=10000, plant_block=1 << 12)
    a = pfac.pfac_build(w.patterns, w.alphabet, merge_levels=levels)
    want = native.AhoCorasick(w.patterns, w.alphabet).scan(w.text)
    got = gpu_scan(a, w.text)
    assert np.array_equal(got, want), (len(got), len(want))


@pytest.mark.parametrize("levels", [3])
def test_packet_batch(levels):
    w = W.packets_256(n_packets=8192, plant_every=4)
    a = pfac.pfac_build(w.patterns, w.alphabet, merge_levels=levels)
    data = torch.from_numpy(w.data.copy()).to(DEV)
    offs = torch.from_numpy(w.offsets.view(np.int64).copy()).to(DEV)
    got = pfac.keys_to_numpy(pfac.pfac_scan_batch(a, data, offs))
    want = native.AhoCorasick(w.patterns, w.alphabet).scan_packets(w.data, w.offsets)
    assert np.array_equal(got, want), (len(got), len(want))


def test_plain_baseline_refuses_compressed_tables():
    a = pfac.pfac_build([b"abc", b"bbc"], 256, merge_levels=3)
    with pytest.raises(pfac.PfacError) as e:
        pfac.pfac_set_tuning(a, algo="plain")
    assert e.value.code == pfac.PFAC_EINVAL
