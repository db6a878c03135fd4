"""pfac_scan_noalloc (the entry point for callers that cannot allocate) against
pfac_scan_async on the same automaton and texts: two calls in a row, the second with a
smaller text, each checked key for key against the allocating entry point and against
the oracle; and its limits (no device copy, too many spans) as errors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_02272_amd.pfac as pfac  # noqa: E402
from oracle import native  # noqa: E402
from paper_1704_02272_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _keys(t, cnt):
    return t[: int(cnt.item())].cpu().numpy().view(np.uint64)


def _both(a, text, cap):
    dev = text.device
    k1 = torch.empty(cap, dtype=torch.int64, device=dev)
    c1 = torch.zeros(1, dtype=torch.int64, device=dev)
    pfac.pfac_scan_async(a, text, k1, c1)
    k2 = torch.full((cap,), -1, dtype=torch.int64, device=dev)
    c2 = torch.full((1,), -1, dtype=torch.int64, device=dev)
    pfac.pfac_scan_noalloc(a, text, k2, c2)
    torch.cuda.synchronize()
    assert int(c1.item()) <= cap and int(c2.item()) == int(c1.item())
    return _keys(k1, c1), _keys(k2, c2)


def test_noalloc_equals_scan_on_two_calls_second_smaller():
    w = W.printable_256(text_bytes=40 << 20, n_patterns=5000)
    a = pfac.pfac_build(w.patterns, 256)
    pfac.pfac_upload(a, 0)
    dev = torch.device("cuda:0")
    big = torch.from_numpy(w.text).to(dev)
    small = big[: (3 << 20) + 77]
    ac = native.AhoCorasick(w.patterns, 256)
    for text in (big, small):
        want = ac.scan(text.cpu().numpy())
        got_scan, got_noalloc = _both(a, text, max(4096, 2 * len(want)))
        assert np.array_equal(got_noalloc, got_scan)
        assert np.array_equal(got_noalloc, want)


def test_noalloc_dense_matches_past_the_records():
    # many matching starts per span: more than the 256 records a span keeps here, so
    # the placement walks those spans again
    rng = np.random.default_rng(31)
    pats = [bytes(rng.integers(0, 4, size=int(rng.integers(3, 7))).astype(np.uint8)) for _ in range(40)]
    a = pfac.pfac_build(pats, 4)
    pfac.pfac_upload(a, 0)
    dev = torch.device("cuda:0")
    ac = native.AhoCorasick(pats, 4)
    for n in ((5 << 20) + 3, (1 << 20) + 1):
        host = rng.integers(0, 4, size=n).astype(np.uint8)
        text = torch.from_numpy(host).to(dev)
        want = ac.scan(host)
        assert len(want) > n // 64
        got_scan, got_noalloc = _both(a, text, len(want) + 16)
        assert np.array_equal(got_noalloc, got_scan)
        assert np.array_equal(got_noalloc, want)


def test_noalloc_limits():
    a = pfac.pfac_build([b"abc", b"bcd"], 256)
    dev = torch.device("cuda:0")
    keys = torch.empty(16, dtype=torch.int64, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    text = torch.zeros(1 << 12, dtype=torch.uint8, device=dev)
    with pytest.raises(pfac.PfacError) as e:
        pfac.pfac_scan_noalloc(a, text, keys, cnt)  # no device copy yet
    assert e.value.code == pfac.PFAC_EINVAL
    pfac.pfac_upload(a, 0)
    # 2 KiB spans: a 16 MiB text takes 8,192 of them, more than the scratch holds
    pfac.pfac_set_tuning(a, span_log2=11)
    big = torch.zeros(16 << 20, dtype=torch.uint8, device=dev)
    with pytest.raises(pfac.PfacError) as e:
        pfac.pfac_scan_noalloc(a, big, keys, cnt)
    assert e.value.code == pfac.PFAC_ETOO_LARGE
    # the most the scratch holds with the library's span length: 256 MiB; one byte more
    pfac.pfac_set_tuning(a)
    edge = torch.zeros((256 << 20) + 1, dtype=torch.uint8, device=dev)
    edge[-4:-1] = torch.tensor(list(b"abc"), dtype=torch.uint8)
    with pytest.raises(pfac.PfacError) as e:
        pfac.pfac_scan_noalloc(a, edge, keys, cnt)
    assert e.value.code == pfac.PFAC_ETOO_LARGE
    pfac.pfac_scan_noalloc(a, edge[:-1], keys, cnt)
    torch.cuda.synchronize()
    assert _keys(keys, cnt).tolist() == [((256 << 20) - 3) << 32]
    del edge, big
    # within the limit, and the empty text
    small = torch.frombuffer(bytearray(b"xxabcdxxbcd"), dtype=torch.uint8).to(dev)
    pfac.pfac_scan_noalloc(a, small, keys, cnt)
    torch.cuda.synchronize()
    assert _keys(keys, cnt).tolist() == [(2 << 32) | 0, (3 << 32) | 1, (8 << 32) | 1]
    pfac.pfac_scan_noalloc(a, small[:0], keys, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0
