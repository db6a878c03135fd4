"""GPU parity across launch choices: span length, root depth, filter key, positions per
thread (16 or 32 starts a lane and step) and grid change only the speed, never the keys
(positions per thread are a free parameter of the method). Also the autotuner, and
captured graphs that outlive a change of tuning."""
import itertools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_02272_amd.pfac as pfac  # noqa: E402
from oracle import native  # noqa: E402
from paper_1704_02272_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(a, dtype=torch.uint8):
    return torch.from_numpy(np.array(a, copy=True)).to(DEV).to(dtype)


def _case(rng, sigma, npat, n, lo, hi):
    pats = [bytes(rng.integers(0, sigma, size=int(rng.integers(lo, hi + 1))).astype(np.uint8))
            for _ in range(npat)]
    text = rng.integers(0, sigma, size=n).astype(np.uint8)
    for _ in range(n // 512):
        p = pats[int(rng.integers(0, npat))]
        o = int(rng.integers(0, n - len(p)))
        text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
    return pats, text


def test_every_tuning_point_gives_the_same_keys_bytes():
    rng = np.random.default_rng(11)
    pats, text = _case(rng, 256, 400, (1 << 20) + 333, 3, 40)
    pats += [b"ab", b"abc"]          # shortest pattern 2: root depth up to 2
    want = native.AhoCorasick(pats, 256).scan(text)
    a = pfac.pfac_build(pats, 256)
    t = _dev(text)
    points = 0
    for span, d, k, lb in itertools.product(range(11, 17), (1, 2), (1, 2, 3, 4), (16, 32)):
        if k < d:
            continue
        pfac.pfac_set_tuning(a, span_log2=span, root_depth=d, filter_k=k, grid=[0, 7][span % 2], lane_bytes=lb)
        assert pfac.pfac_get_tuning(a)["lane_bytes"] == lb
        got = pfac.keys_to_numpy(pfac.pfac_scan(a, t))
        assert np.array_equal(got, want), (span, d, k, lb)
        points += 1
    assert points == 6 * 7 * 2
    # a text that starts off a 16-byte boundary and ends ragged (the guarded load path),
    # 16 starts a lane
    pfac.pfac_set_tuning(a, lane_bytes=16)
    assert np.array_equal(pfac.keys_to_numpy(pfac.pfac_scan(a, t[5:-3])),
                          native.AhoCorasick(pats, 256).scan(text[5:-3]))


def test_sampled_form_keeps_32_positions_per_thread():
    rng = np.random.default_rng(14)
    pats, text = _case(rng, 256, 300, (1 << 20) + 45, 4, 30)   # shortest pattern 4: sampled form
    want = native.AhoCorasick(pats, 256).scan(text)
    a = pfac.pfac_build(pats, 256)
    pfac.pfac_set_tuning(a, lane_bytes=16)
    assert pfac.pfac_get_tuning(a)["lane_bytes"] == 32   # the sampled form reads 32 bytes a lane
    assert np.array_equal(pfac.keys_to_numpy(pfac.pfac_scan(a, _dev(text))), want)


def test_tuning_points_two_bit_symbols():
    rng = np.random.default_rng(12)
    pats, text = _case(rng, 4, 2000, (1 << 20) + 77, 8, 24)
    want = native.AhoCorasick(pats, 4).scan(text)
    a = pfac.pfac_build(pats, 4)
    t = _dev(text)
    combos = [(s, d, k) for s in (11, 12, 14, 16) for d in range(1, 9) for k in range(d, 17)]
    for j, i in enumerate(rng.choice(len(combos), size=24, replace=False)):
        s, d, k = combos[int(i)]
        lb = (16, 32)[j % 2]
        pfac.pfac_set_tuning(a, span_log2=s, root_depth=d, filter_k=k, lane_bytes=lb)
        got = pfac.keys_to_numpy(pfac.pfac_scan(a, t))
        assert np.array_equal(got, want), (s, d, k, lb)


def test_autotuner_keeps_results_and_reports_its_choice():
    w = W.packets_256(n_packets=8192, n_patterns=4000, plant_every=4)
    a = pfac.pfac_build(w.patterns, w.alphabet)
    want = native.AhoCorasick(w.patterns, w.alphabet).scan_packets(w.data, w.offsets)
    d = _dev(w.data)
    o = _dev(w.offsets.view(np.int64), torch.int64)
    t = pfac.pfac_tune(a, d, o, reps=3)
    assert t["algo"] == "tiled" and (t["span_log2"] == 0 or 11 <= t["span_log2"] <= 16) and t["ms"] > 0
    assert pfac.pfac_get_tuning(a) == {k: v for k, v in t.items() if k != "ms"}
    got = pfac.keys_to_numpy(pfac.pfac_scan_batch(a, d, o))
    assert np.array_equal(got, want)
    # packet batches with either number of positions per thread
    for lb in (16, 32):
        pfac.pfac_set_tuning(a, **dict({k: v for k, v in t.items() if k != "ms"}, lane_bytes=lb))
        assert np.array_equal(pfac.keys_to_numpy(pfac.pfac_scan_batch(a, d, o)), want), lb


def test_graph_outlives_a_change_of_tuning():
    rng = np.random.default_rng(13)
    pats, text = _case(rng, 256, 300, 1 << 19, 4, 30)
    ac = native.AhoCorasick(pats, 256)
    a = pfac.pfac_build(pats, 256)
    t = _dev(text)
    keys = torch.zeros(1 << 16, dtype=torch.int64, device=DEV)
    count = torch.zeros(1, dtype=torch.int64, device=DEV)
    sizes = torch.tensor([len(text), 0], dtype=torch.int64, device=DEV)
    s = torch.cuda.Stream()
    g = pfac.pfac_graph_create(a, t, None, keys, count, sizes, s)
    want = ac.scan(text)
    for d, k, span, lb in [(1, 3, 12, 16), (2, 2, 16, 32), (2, 4, 11, 16)]:
        pfac.pfac_set_tuning(a, root_depth=d, filter_k=k, span_log2=span, lane_bytes=lb)
        g.launch(s)
        s.synchronize()
        c = int(count.item())
        assert c == len(want) and np.array_equal(pfac.keys_to_numpy(keys[:c]), want), (d, k, span, lb)
        assert np.array_equal(pfac.keys_to_numpy(pfac.pfac_scan(a, t)), want)
    g.close()
