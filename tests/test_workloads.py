"""The seeded generators: byte-identical reproduction and the statistics each workload
promises (small-scale variants, so the CPU suite stays fast)."""
import numpy as np

from paper_1704_02272_amd import workloads as W


def test_seed_reproduces_bytes():
    a = W.uniform_256(text_bytes=1 << 16, n_plants=10)
    b = W.uniform_256(text_bytes=1 << 16, n_plants=10)
    assert a.sha256() == b.sha256()
    c = W.uniform_256(seed=99, text_bytes=1 << 16, n_plants=10)
    assert c.sha256()["text"] != a.sha256()["text"]


def test_uniform_256_shape():
    w = W.uniform_256()
    assert len(w.text) == 1 << 20 and len(w.patterns) == 100
    assert all(4 <= len(p) <= 16 for p in w.patterns)
    assert len(w.plants) == 1000


def test_printable_256_statistics():
    w = W.printable_256(text_bytes=1 << 22)
    lens = np.array([len(p) for p in w.patterns])
    assert lens.min() >= 4 and lens.max() <= 64
    assert 11 <= np.median(lens) <= 13
    t = w.text
    printable = np.mean((t >= 0x20) & (t <= 0x7E))
    # 90 % printable-uniform plus 10 % uniform bytes that land in the printable range
    assert abs(printable - (0.9 + 0.1 * 95 / 256)) < 0.01
    allp = np.frombuffer(b"".join(w.patterns), dtype=np.uint8)
    pp = np.mean((allp >= 0x20) & (allp <= 0x7E))
    assert abs(pp - (0.7 + 0.3 * 95 / 256)) < 0.02
    heads = [p[:4] for p in w.patterns]
    shared = sum(1 for h in heads if heads.count(h) > 1)
    assert shared >= 0.3 * len(heads)  # 20 % takers + the donors they copied
    assert len(w.plants) == (1 << 22) // (1 << 16)
    for off, j in w.plants:
        assert off // (1 << 16) == (off + len(w.patterns[j]) - 1) // (1 << 16)


def test_dna_4_statistics():
    w = W.dna_4(text_bytes=1 << 20)
    assert w.text.max() <= 3
    assert all(8 <= len(p) <= 32 for p in w.patterns)
    assert all(max(p) <= 3 for p in w.patterns)
    # order-2 Markov: conditional next-symbol frequencies differ across contexts
    t = w.text.astype(np.int64)
    ctx = t[:-2] * 4 + t[1:-1]
    freq = np.array([np.bincount(t[2:][ctx == c], minlength=4) for c in range(16)], dtype=float)
    freq /= freq.sum(axis=1, keepdims=True)
    assert freq.std(axis=0).max() > 0.05
    assert len(w.plants) == 1


def test_packets_256_shape():
    w = W.packets_256(n_packets=4096, n_patterns=2000, plant_every=16)
    sizes = np.diff(w.offsets)
    assert set(np.unique(sizes)) <= {64, 576, 1500}
    frac64 = np.mean(sizes == 64)
    assert abs(frac64 - 0.4) < 0.03
    assert all(4 <= len(p) <= 128 for p in w.patterns)
    heads = {p[:6] for p in w.patterns if len(p) >= 6}
    assert len(heads) <= 729
    assert 0.03 < len(w.plants) / w.n_packets < 0.09
    for i, off, j in w.plants:
        p = w.patterns[j]
        assert off + len(p) <= sizes[i]


def test_serving_256_shape():
    w = W.serving_256(n_patterns=2000, pool_bytes=1 << 22, max_requests=300, plant_every=16)
    assert len(w.requests) == 300
    arr = np.array([r.arrival_s for r in w.requests])
    assert np.all(np.diff(arr) > 0)
    mean_req = w.packets_per_request * 2769.0
    lam = w.offered_bytes_per_s / mean_req
    gaps = np.diff(arr)
    assert abs(gaps.mean() * lam - 1) < 0.2
    for r in w.requests[:20]:
        sizes = np.diff(r.offsets)
        assert len(sizes) == 32 and set(np.unique(sizes)) <= {64, 512, 1500, 9000}


def test_serving_256_contiguous_views_share_the_pool():
    w = W.serving_256(n_patterns=500, pool_bytes=1 << 22, max_requests=200, plant_every=4, contiguous=True)
    assert len(w.requests) == 200
    for r in w.requests:
        assert r.data.base is w.pool or r.data.base is w.pool.base
        assert len(r.data) == int(r.offsets[-1])
        assert set(np.unique(np.diff(r.offsets))) <= {64, 512, 1500, 9000}
    # planted patterns exist in the pool
    hits = sum(1 for p in w.patterns[:500] if bytes(p) in w.pool.tobytes())
    assert hits > 0
