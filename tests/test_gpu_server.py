"""GPU tests of the serving loop: every request's result equals the oracle's scan of that
request, the same alone and in a mix of concurrent requests; admission by device memory
and by queue bytes; the rescan when a batch overflows its key buffer."""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_02272_amd.pfac as pfac  # noqa: E402
from oracle import native  # noqa: E402
from paper_1704_02272_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    w = W.serving_256(n_patterns=5000, pool_bytes=1 << 24, max_requests=400, plant_every=4,
                      contiguous=True)
    ac = native.AhoCorasick(w.patterns, w.alphabet)
    want = [ac.scan_packets(r.data, r.offsets) for r in w.requests]
    return w, want


def drain(srv, tickets, timeout_s=60.0):
    got = {}
    t0 = time.monotonic()
    while len(got) < len(tickets):
        for r in srv.poll(timeout_us=20000):
            got[r["ticket"]] = r
        assert time.monotonic() - t0 < timeout_s, "server did not finish"
    return got


@pytest.mark.parametrize("flags", [0, pfac.PFAC_SERVER_EAGER])
def test_alone_equals_in_mix_equals_oracle(served, flags):
    w, want = served
    torch.cuda.set_device(0)
    a = pfac.pfac_build(w.patterns, w.alphabet)
    srv = pfac.pfac_server_create(a, slots=3, max_batch_bytes=1 << 20, flags=flags)
    assert srv.config()["flags"] == flags
    assert srv.config()["slots"] == 3
    probe = 7
    t = srv.submit(w.requests[probe].data, w.requests[probe].offsets)
    alone = drain(srv, [t])[t]
    assert alone["status"] == 0
    assert np.array_equal(alone["keys"], want[probe])
    assert sum(len(x) for x in want) > 100  # plants give every batch real matches
    tickets = [srv.submit(r.data, r.offsets) for r in w.requests]
    got = drain(srv, tickets)
    for i, t in enumerate(tickets):
        r = got[t]
        assert r["status"] == 0 and r["n_pkts"] == 32
        assert np.array_equal(r["keys"], want[i]), i
        assert r["arrival_ns"] <= r["launch_ns"] <= r["done_ns"]
    assert np.array_equal(got[tickets[probe]]["keys"], alone["keys"])
    st = srv.stats()
    assert st["requests"] == len(w.requests) + 1 and st["packets"] == 32 * (len(w.requests) + 1)
    assert st["batches"] < st["requests"]  # requests were batched together
    assert 0 < st["p50_ns"] <= st["p99_ns"] <= st["max_ns"]
    srv.close()


def test_key_overflow_rescans(served):
    w, want = served
    a = pfac.pfac_build(w.patterns, w.alphabet)
    srv = pfac.pfac_server_create(a, slots=2, key_capacity=1, max_batch_bytes=1 << 20)
    tickets = [srv.submit(r.data, r.offsets) for r in w.requests[:60]]
    got = drain(srv, tickets)
    for i, t in enumerate(tickets):
        assert np.array_equal(got[t]["keys"], want[i]), i
    srv.close()


def test_admission_by_memory_and_queue(served):
    w, _ = served
    a = pfac.pfac_build(w.patterns, w.alphabet)
    with pytest.raises(pfac.PfacError) as e:
        pfac.pfac_server_create(a, device_memory_budget=1 << 20, max_batch_bytes=8 << 20)
    assert e.value.code == pfac.PFAC_ENOMEM
    srv = pfac.pfac_server_create(a, slots=8, max_batch_bytes=1 << 20, device_memory_budget=5 << 20)
    assert 1 <= srv.config()["slots"] < 8
    r = w.requests[0]
    # a request larger than a batch is refused
    big = np.zeros(2 << 20, dtype=np.uint8)
    with pytest.raises(pfac.PfacError) as e:
        srv.submit(big, np.array([0, len(big)], dtype=np.uint64))
    assert e.value.code == pfac.PFAC_ETOO_LARGE
    srv.close()
    # a small waiting queue turns a burst away with PFAC_EBUSY, and the rest completes
    srv = pfac.pfac_server_create(a, slots=1, max_batch_bytes=1 << 20, max_pending_bytes=len(r.data) * 2)
    codes = [srv.submit_raw(r.data.ctypes.data, r.offsets.ctypes.data, 32) for _ in range(200)]
    assert pfac.PFAC_EBUSY in codes
    ok = [c for c in codes if c == 0]
    seen = 0
    t0 = time.monotonic()
    while seen < len(ok):
        seen += len(srv.poll(timeout_us=20000, with_keys=False))
        assert time.monotonic() - t0 < 60
    assert srv.stats()["rejected"] == codes.count(pfac.PFAC_EBUSY)
    srv.close()


def test_empty_packets_and_empty_request(served):
    w, _ = served
    a = pfac.pfac_build(w.patterns, w.alphabet)
    srv = pfac.pfac_server_create(a, slots=1, max_batch_bytes=1 << 16)
    p = w.patterns[0]
    data = np.frombuffer(p + p, dtype=np.uint8)
    t1 = srv.submit(data, np.array([0, 0, len(p), len(p), 2 * len(p)], dtype=np.uint64))
    t2 = srv.submit(np.zeros(0, np.uint8), np.array([0], dtype=np.uint64))
    got = drain(srv, [t1, t2])
    want = native.AhoCorasick(w.patterns, 256).scan_packets(
        data, np.array([0, 0, len(p), len(p), 2 * len(p)], dtype=np.uint64))
    assert np.array_equal(got[t1]["keys"], want) and len(want) >= 2
    assert got[t2]["status"] == 0 and got[t2]["n_matches"] == 0
    srv.close()


@pytest.fixture(scope="module")
def served_full():
    """The serving workload's own pattern set: 50,000 patterns of 4-256 random bytes
    (the patterns are drawn before the payload pool, so a 64 MiB pool leaves them as in
    the full 1 GiB stream), 300 requests of 32 packets, one planted pattern in a quarter
    of the packets."""
    w = W.serving_256(pool_bytes=1 << 26, max_requests=300, plant_every=4, contiguous=True)
    assert len(w.patterns) == 50000 and w.max_len > 128
    ac = native.AhoCorasick(w.patterns, w.alphabet)
    want = [ac.scan_packets(r.data, r.offsets) for r in w.requests]
    return w, want


def test_full_pattern_set_alone_in_mix_and_batch(served_full):
    w, want = served_full
    print("serving_256 full pattern set: %d requests, %d keys expected"
          % (len(w.requests), sum(len(x) for x in want)), flush=True)
    assert sum(len(x) for x in want) > 500
    a = pfac.pfac_build(w.patterns, w.alphabet)
    info = pfac.pfac_table_info(a)
    assert info["n_patterns"] == 50000 and info["max_len"] == w.max_len
    srv = pfac.pfac_server_create(a, slots=4, max_batch_bytes=4 << 20)
    probes = [0, 11, 150, 299]
    alone = {}
    for p in probes:
        t = srv.submit(w.requests[p].data, w.requests[p].offsets)
        alone[p] = drain(srv, [t])[t]
        assert alone[p]["status"] == 0
        assert np.array_equal(alone[p]["keys"], want[p]), p
    tickets = [srv.submit(r.data, r.offsets) for r in w.requests]
    got = drain(srv, tickets)
    for i, t in enumerate(tickets):
        assert got[t]["status"] == 0
        assert np.array_equal(got[t]["keys"], want[i]), i
    for p in probes:
        assert np.array_equal(got[tickets[p]]["keys"], alone[p]["keys"])
    srv.close()
    # the same requests as one packet batch through pfac_scan_batch
    data = np.concatenate([r.data for r in w.requests])
    base = np.cumsum([0] + [len(r.data) for r in w.requests])
    offs = np.concatenate([r.offsets[:-1] + np.uint64(b) for r, b in zip(w.requests, base[:-1])]
                          + [np.array([base[-1]], dtype=np.uint64)])
    keys = pfac.keys_to_numpy(pfac.pfac_scan_batch(
        a, torch.from_numpy(data).cuda(), torch.from_numpy(offs.view(np.int64)).cuda()))
    expect = np.concatenate([k + np.uint64(int(b) << 32) for k, b in zip(want, base[:-1])])
    assert np.array_equal(keys, expect)
