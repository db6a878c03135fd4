"""GPU parity of packet batches and captured graphs against the oracle.

A batch is a CSR list of packets; each packet is its own text (no match crosses a
packet end) and keys carry the global byte offset. The oracle scans every packet on its
own (textbook Aho-Corasick) and shifts its starts by the packet offset."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_02272_amd.pfac as pfac  # noqa: E402
from oracle import native  # noqa: E402
from paper_1704_02272_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(a, dtype=torch.uint8):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype)


def gpu_batch(a, data, offsets):
    d = _dev(np.asarray(data, dtype=np.uint8))
    o = _dev(np.asarray(offsets, dtype=np.uint64).view(np.int64), torch.int64)
    k = pfac.pfac_scan_batch(a, d, o)
    torch.cuda.synchronize()
    return pfac.keys_to_numpy(k)


def random_batch(rng, pats, sigma, n_pkts, sizes, plants=0.5):
    lens = rng.choice(np.array(sizes), size=n_pkts)
    offsets = np.zeros(n_pkts + 1, dtype=np.uint64)
    np.cumsum(lens, out=offsets[1:])
    data = rng.integers(0, sigma, size=int(offsets[-1])).astype(np.uint8)
    for i in range(n_pkts):
        a, b = int(offsets[i]), int(offsets[i + 1])
        if b - a == 0 or rng.random() > plants:
            continue
        p = pats[int(rng.integers(0, len(pats)))]
        # plants that fit, and plants that straddle the packet end (must not match)
        o = int(rng.integers(max(a - len(p) + 1, 0), b))
        e = min(o + len(p), len(data))
        data[o:e] = np.frombuffer(p, dtype=np.uint8)[:e - o]
    return data, offsets


@pytest.mark.parametrize("sigma", [2, 4, 26, 256])
def test_random_batches(sigma):
    rng = np.random.default_rng(77 + sigma)
    for trial in range(12):
        npat = int(rng.integers(1, 60))
        pats = [bytes(rng.integers(0, sigma, size=int(rng.integers(1, 40))).astype(np.uint8))
                for _ in range(npat)]
        sizes = [[0, 1, 2, 7, 64], [64, 576, 1500], [0, 16383, 16384, 16385, 40000]][trial % 3]
        n_pkts = int(rng.choice([1, 2, 17, 300, 2000]))
        data, offsets = random_batch(rng, pats, sigma, n_pkts, sizes)
        a = pfac.pfac_build(pats, sigma)
        pfac.pfac_set_tuning(a, grid=int(rng.choice([0, 1, 5])))
        want = native.AhoCorasick(pats, sigma).scan_packets(data, offsets)
        got = gpu_batch(a, data, offsets)
        assert np.array_equal(got, want), (sigma, trial, len(got), len(want))


def test_batch_equals_per_packet_scans():
    w = W.packets_256(n_packets=256, n_patterns=2000, plant_every=2)
    a = pfac.pfac_build(w.patterns, w.alphabet)
    got = gpu_batch(a, w.data, w.offsets)
    parts = []
    for i in range(w.n_packets):
        lo = int(w.offsets[i])
        k = pfac.keys_to_numpy(pfac.pfac_scan(a, _dev(w.packet(i))))
        parts.append(k + np.uint64(lo << 32))
    assert len(got) >= len(w.plants)
    assert np.array_equal(got, np.concatenate(parts))


def test_batch_edge_cases():
    pats = [b"ab", b"abc", b"b", b"ab"]
    a = pfac.pfac_build(pats, 256)
    # no packets, only empty packets, one-byte packets, a pattern across a boundary
    assert len(gpu_batch(a, np.zeros(1, np.uint8), [0])) == 0
    assert len(gpu_batch(a, np.zeros(1, np.uint8), [0, 0, 0])) == 0
    data = np.frombuffer(b"abcab", dtype=np.uint8)
    got = gpu_batch(a, data, [0, 1, 3, 3, 5])  # "a" | "bc" | "" | "ab"
    want = native.AhoCorasick(pats, 256).scan_packets(data, np.array([0, 1, 3, 3, 5], np.uint64))
    assert np.array_equal(got, want)
    assert [(int(k >> np.uint64(32)), int(k & np.uint64(0xFFFFFFFF))) for k in got] == \
        [(1, 2), (3, 0), (3, 3), (4, 2)]
    pk, off, ids = pfac.pfac_key_to_packet(got, np.array([0, 1, 3, 3, 5], np.uint64))
    assert pk.tolist() == [1, 3, 3, 3] and off.tolist() == [0, 0, 0, 1] and ids.tolist() == [2, 0, 3, 2]


@pytest.mark.parametrize("planted", [0, 8])
def test_packets_256_full(planted):
    w = W.packets_256(plant_every=planted)
    a = pfac.pfac_build(w.patterns, w.alphabet)
    want = native.AhoCorasick(w.patterns, w.alphabet).scan_packets(w.data, w.offsets)
    got = gpu_batch(a, w.data, w.offsets)
    assert np.array_equal(got, want), (len(got), len(want))
    keyset = set(got.tolist())
    for pkt, off, j in w.plants:
        s = int(w.offsets[pkt]) + off
        if bytes(w.data[s:s + len(w.patterns[j])]) == w.patterns[j]:
            assert (s << 32) | j in keyset


def test_graph_replays_with_varying_batches():
    w = W.packets_256(n_packets=3000, n_patterns=3000, plant_every=3)
    a = pfac.pfac_build(w.patterns, w.alphabet)
    ac = native.AhoCorasick(w.patterns, w.alphabet)
    max_pkts, max_bytes = w.n_packets, int(w.offsets[-1])
    data = torch.zeros(max_bytes, dtype=torch.uint8, device=DEV)
    offs = torch.zeros(max_pkts + 1, dtype=torch.int64, device=DEV)
    keys = torch.zeros(200000, dtype=torch.int64, device=DEV)
    count = torch.zeros(1, dtype=torch.int64, device=DEV)
    sizes = torch.zeros(2, dtype=torch.int64, device=DEV)
    s = torch.cuda.Stream()
    g = pfac.pfac_graph_create(a, data, offs, keys, count, sizes, s)
    rng = np.random.default_rng(5)
    for rep, n_pk in enumerate([max_pkts, 10, 1, 1700, 0, max_pkts, 333]):
        lo = int(rng.integers(0, max_pkts - n_pk + 1))
        o = (w.offsets[lo:lo + n_pk + 1] - w.offsets[lo]).astype(np.uint64)
        if n_pk == 0:
            o = np.zeros(1, np.uint64)
        nb = int(o[-1])
        chunk = w.data[int(w.offsets[lo]):int(w.offsets[lo]) + nb]
        with torch.cuda.stream(s):
            if nb:
                data[:nb].copy_(_dev(chunk))
            offs[:n_pk + 1].copy_(_dev(o.view(np.int64), torch.int64))
            sizes.copy_(torch.tensor([nb, n_pk], dtype=torch.int64, device=DEV))
            g.launch(s)
        s.synchronize()
        n = int(count.item())
        want = ac.scan_packets(chunk, o)
        assert n == len(want), (rep, n_pk, n, len(want))
        got = pfac.keys_to_numpy(keys[:n])
        assert np.array_equal(got, want), rep
        # eager work on the same automaton between replays
        eager = gpu_batch(a, chunk if nb else np.zeros(1, np.uint8), o)
        assert np.array_equal(eager, want)
    g.close()


def test_graph_text_mode():
    w = W.uniform_256(text_bytes=1 << 20)
    a = pfac.pfac_build(w.patterns, w.alphabet)
    ac = native.AhoCorasick(w.patterns, w.alphabet)
    text = _dev(w.text)
    keys = torch.zeros(10000, dtype=torch.int64, device=DEV)
    count = torch.zeros(1, dtype=torch.int64, device=DEV)
    sizes = torch.zeros(2, dtype=torch.int64, device=DEV)
    s = torch.cuda.Stream()
    g = pfac.pfac_graph_create(a, text, None, keys, count, sizes, s)
    for n in [len(w.text), 100000, 17, len(w.text), 0, 65537]:
        with torch.cuda.stream(s):
            sizes.copy_(torch.tensor([n, 0], dtype=torch.int64, device=DEV))
            g.launch(s)
        s.synchronize()
        want = ac.scan(w.text[:n])
        c = int(count.item())
        assert c == len(want), (n, c, len(want))
        assert np.array_equal(pfac.keys_to_numpy(keys[:c]), want), n
    g.close()
