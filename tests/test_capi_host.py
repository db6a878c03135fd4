"""The C ABI on the host (no GPU): the library loads and exports every symbol the header
declares; building validates its input; the table it builds is, bit for bit, the
Section 3.1 layout the oracle writes out from its definition."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1704_02272_amd.pfac as pfac
from oracle import trie
from paper_1704_02272_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfac.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"PFAC_API\s+[\w\s\*]*?\b(pfac_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 10
    L = C.CDLL(pfac.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_version():
    assert pfac.strerror(pfac.PFAC_OK) == "ok"
    for code in range(-10, 0):
        assert pfac.strerror(code) != "unknown status"
    assert pfac.pfac_version() >= 10000


@pytest.mark.parametrize("pats,alphabet,code", [
    ([b"ab", b""], 256, pfac.PFAC_EEMPTY_PATTERN),
    ([b"ab", b"\x04"], 4, pfac.PFAC_ESYMBOL),
    ([b"ab"], 0, pfac.PFAC_EINVAL),
    ([b"ab"], 257, pfac.PFAC_EINVAL),
])
def test_build_errors(pats, alphabet, code):
    with pytest.raises(pfac.PfacError) as e:
        pfac.pfac_build(pats, alphabet)
    assert e.value.code == code


def test_build_null_arguments():
    L = pfac.lib()
    h = C.c_void_p()
    assert L.pfac_build_csr(None, None, 3, 256, C.byref(h)) == pfac.PFAC_EINVAL
    assert L.pfac_build_csr(None, None, 0, 256, None) == pfac.PFAC_EINVAL
    assert L.pfac_table_info(None, None) == pfac.PFAC_EINVAL


def _paper_arrays(pats, alphabet):
    off, bms = trie.paper_layout(pats, alphabet)
    words = (alphabet + 31) // 32
    bm = np.array([[(b >> (32 * w)) & 0xFFFFFFFF for w in range(words)] for b in bms],
                  dtype=np.uint32).reshape(len(bms), words)
    return np.array(off, dtype=np.uint32), bm


def _check_table(pats, alphabet):
    a = pfac.pfac_build(pats, alphabet)
    off, bm = pfac.pfac_export_paper_table(a)
    want_off, want_bm = _paper_arrays(pats, alphabet)
    assert np.array_equal(off, want_off)
    assert np.array_equal(bm, want_bm)
    info = pfac.pfac_table_info(a)
    assert info["n_nodes"] == len(want_off)
    assert info["paper_table_bytes"] == trie.paper_table_bytes(len(want_off), alphabet)
    # pattern ids per node: the ids of the patterns that spell that node's string
    first, ids = pfac.pfac_export_outputs(a)
    nodes = trie.canonical_nodes(pats)
    for q, s in enumerate(nodes):
        want = [j for j, p in enumerate(pats) if p == s]
        assert list(ids[first[q]:first[q + 1]]) == want
    return a, info


def test_worked_example_table():
    a, info = _check_table([b"AB", b"AD", b"Z"], 256)
    off, bm = pfac.pfac_export_paper_table(a)
    assert off[1] == 3 and (bm[1][2] >> (66 - 64)) & 1 and (bm[1][2] >> (68 - 64)) & 1
    assert info["n_nodes"] == 5


def test_random_tables_match_layout_model():
    rng = np.random.default_rng(21)
    for trial in range(60):
        sigma = int(rng.choice([1, 2, 4, 5, 26, 32, 33, 64, 65, 128, 200, 256]))
        pats = [bytes(rng.integers(0, sigma, size=int(rng.integers(1, 10))).astype(np.uint8))
                for _ in range(int(rng.integers(1, 60)))]
        _check_table(pats, sigma)


def test_workload_tables_match_layout_model():
    _check_table(W.uniform_256().patterns, 256)
    _check_table(W.dna_4(text_bytes=1 << 12, n_patterns=2000).patterns, 4)
    _check_table(W.printable_256(text_bytes=1 << 16, n_patterns=1500).patterns, 256)


def test_node_layout_choice():
    assert pfac.pfac_table_info(pfac.pfac_build([b"\x01\x02"], 32))["node_layout"] == 0
    assert pfac.pfac_table_info(pfac.pfac_build([b"\x01\x02"], 33))["node_layout"] == 1


def test_empty_pattern_set():
    a = pfac.pfac_build([], 256)
    info = pfac.pfac_table_info(a)
    assert info["n_nodes"] == 1 and info["n_patterns"] == 0


def test_key_to_packet():
    # packets "a" | "bc" | "" | "ab" at offsets 0, 1, 3, 3; keys (start << 32) | id
    offsets = np.array([0, 1, 3, 3, 5], dtype=np.uint64)
    keys = np.array([(1 << 32) | 2, (3 << 32) | 0, (4 << 32) | 7, 0 | 9], dtype=np.uint64)
    pk, off, ids = pfac.pfac_key_to_packet(keys, offsets)
    assert pk.tolist() == [1, 3, 3, 0]      # an empty packet never owns a start
    assert off.tolist() == [0, 0, 1, 0]
    assert ids.tolist() == [2, 0, 7, 9]
    # against a plain search over random batches
    rng = np.random.default_rng(4)
    for _ in range(20):
        sizes = rng.integers(0, 9, size=int(rng.integers(1, 30)))
        offs = np.zeros(len(sizes) + 1, np.uint64)
        offs[1:] = np.cumsum(sizes)
        if offs[-1] == 0:
            continue
        starts = rng.integers(0, int(offs[-1]), size=50)
        ids_in = rng.integers(0, 1 << 32, size=50)
        k = (starts.astype(np.uint64) << np.uint64(32)) | ids_in.astype(np.uint64)
        pk, off, ids = pfac.pfac_key_to_packet(k, offs)
        for i, s in enumerate(starts):
            p = max(j for j in range(len(sizes)) if offs[j] <= s < offs[j + 1])
            assert (pk[i], off[i], ids[i]) == (p, s - offs[p], ids_in[i])
    # a start past the last packet's end, or NULL arrays, are refused
    with pytest.raises(pfac.PfacError) as e:
        pfac.pfac_key_to_packet(np.array([5 << 32], np.uint64), offsets)
    assert e.value.code == pfac.PFAC_EINVAL
    assert pfac.lib().pfac_key_to_packet(None, 1, None, 0, None, None, None) == pfac.PFAC_EINVAL
    assert pfac.lib().pfac_key_to_packet(None, 0, None, 0, None, None, None) == pfac.PFAC_OK


# --------------------------------------------------------------------------- save / load
def _same_automaton(a, b):
    ia, ib = pfac.pfac_table_info(a), pfac.pfac_table_info(b)
    assert ia == ib
    ta, tb = pfac.pfac_export_paper_table(a), pfac.pfac_export_paper_table(b)
    assert np.array_equal(ta[0], tb[0]) and np.array_equal(ta[1], tb[1])
    oa, ob = pfac.pfac_export_outputs(a), pfac.pfac_export_outputs(b)
    assert np.array_equal(oa[0], ob[0]) and np.array_equal(oa[1], ob[1])
    assert pfac.pfac_get_tuning(a) == pfac.pfac_get_tuning(b)
    assert pfac.pfac_save(a) == pfac.pfac_save(b)


def _pattern_sets():
    rng = np.random.default_rng(31)
    yield [], 256
    yield [b"AB", b"AD", b"Z"], 256
    yield [b"ab", b"abc", b"bc", b"c", b"ab"], 256           # duplicates, prefixes
    yield [bytes(rng.integers(0, 4, size=int(rng.integers(1, 12))).astype(np.uint8))
           for _ in range(300)], 4
    yield [bytes(rng.integers(0, 52, size=int(rng.integers(1, 9))).astype(np.uint8))
           for _ in range(200)], 52
    w = W.printable_256(text_bytes=1 << 12, n_patterns=2000)
    yield w.patterns, 256


@pytest.mark.parametrize("k", range(6))
def test_save_load_round_trip(k):
    pats, alphabet = list(_pattern_sets())[k]
    a = pfac.pfac_build(pats, alphabet)
    blob = pfac.pfac_save(a)
    b = pfac.pfac_load(blob)
    _same_automaton(a, b)
    # a second automaton built from the same patterns is the same too
    _same_automaton(pfac.pfac_build(pats, alphabet), b)


def test_save_keeps_tuning():
    pats = [b"abcd", b"abce", b"xyzw", b"qq12"]
    a = pfac.pfac_build(pats, 256)
    pfac.pfac_set_tuning(a, algo="tiled", grid=300, span_log2=13, root_depth=1, filter_k=3, lane_bytes=16)
    b = pfac.pfac_load(pfac.pfac_save(a))
    assert pfac.pfac_get_tuning(b) == pfac.pfac_get_tuning(a)
    assert pfac.pfac_get_tuning(b)["lane_bytes"] == 16 and pfac.pfac_get_tuning(b)["grid"] == 300
    assert pfac.pfac_table_info(b)["root_depth"] == 1 and pfac.pfac_table_info(b)["filter_k"] == 3


def test_save_capacity_and_arguments():
    a = pfac.pfac_build([b"ab"], 256)
    L = pfac.lib()
    size = C.c_uint64(0)
    assert L.pfac_save(a.handle, None, 0, C.byref(size)) == pfac.PFAC_ECAPACITY and size.value > 64
    small = (C.c_uint8 * 8)()
    assert L.pfac_save(a.handle, small, 8, C.byref(size)) == pfac.PFAC_ECAPACITY
    assert L.pfac_save(None, None, 0, C.byref(size)) == pfac.PFAC_EINVAL
    assert L.pfac_save(a.handle, None, 0, None) == pfac.PFAC_EINVAL
    h = C.c_void_p()
    assert L.pfac_load(None, 0, C.byref(h)) == pfac.PFAC_EINVAL
    assert L.pfac_load(small, 8, None) == pfac.PFAC_EINVAL


def _fnv1a(data: bytes) -> int:
    h = 0xcbf29ce484222325
    for b in data:
        h = ((h ^ b) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def _reseal(blob: bytearray) -> bytes:
    """Recompute the header checksum (64-bit FNV-1a over bytes 0..55 and the payload)."""
    blob[56:64] = _fnv1a(bytes(blob[:56]) + bytes(blob[64:])).to_bytes(8, "little")
    return bytes(blob)


def _expect_format_error(blob):
    with pytest.raises(pfac.PfacError) as e:
        pfac.pfac_load(blob)
    assert e.value.code == pfac.PFAC_EFORMAT


def test_load_rejects_truncated_and_flipped_blobs():
    pats = [b"he", b"she", b"his", b"hers", b"h"]
    blob = pfac.pfac_save(pfac.pfac_build(pats, 256))
    assert _reseal(bytearray(blob)) == blob  # the test's checksum is the library's
    for n in range(len(blob)):
        _expect_format_error(blob[:n])
    _expect_format_error(blob + b"\0" * 8)
    rng = np.random.default_rng(8)
    for pos in list(range(64)) + rng.integers(64, len(blob), size=200).tolist():
        for bit in (0, 5):
            bad = bytearray(blob)
            bad[pos] ^= 1 << bit
            _expect_format_error(bytes(bad))


def test_load_rejects_inconsistent_tables_with_valid_checksum():
    """Blobs whose checksum is right but whose table is not the trie of its patterns."""
    pats = [b"ab", b"ad", b"z"]
    a = pfac.pfac_build(pats, 256)
    blob = bytearray(pfac.pfac_save(a))
    Q, N = 5, 3
    off_pat = 64
    off_bytes = off_pat + (N + 1) * 8
    off_first = off_bytes + 8                     # 5 pattern bytes padded to 8
    off_bm = off_first + 24                       # 5 u32 padded to 24
    off_of = off_bm + Q * 4 * 8
    off_ids = off_of + 24
    assert len(blob) == off_ids + 16
    assert blob[off_bytes:off_bytes + 5] == b"abadz"

    def mutate(at, value, size=4):
        bad = bytearray(blob)
        bad[at:at + size] = value.to_bytes(size, "little")
        return _reseal(bad)

    assert pfac.pfac_load(_reseal(bytearray(blob))) is not None
    _expect_format_error(mutate(off_first + 4 * 1, 4))      # node 1's first child off by one
    _expect_format_error(mutate(off_first + 4 * 1, 99))     # past the table
    _expect_format_error(mutate(off_ids, 7))                # id out of range
    _expect_format_error(mutate(off_ids, 0))                # id 0 twice (ids are 2, 0, 1)
    _expect_format_error(mutate(off_of + 4 * 5, 2))         # a leaf that ends no pattern
    _expect_format_error(mutate(off_bytes + 1, ord("c"), 1))  # 'ac' is not in the trie
    _expect_format_error(mutate(16, 100))                   # alphabet below 'z'
    _expect_format_error(mutate(off_bm + 8 * 3, 1 << 32, 8))  # an extra child bit
    _expect_format_error(mutate(28, 9))                     # wrong longest pattern
    _expect_format_error(mutate(40, 3 << 16))               # root depth 3 > shortest pattern
    _expect_format_error(mutate(40, 9))                     # no such algorithm


def test_batch_and_graph_argument_errors():
    a = pfac.pfac_build([b"ab"], 256)
    L = pfac.lib()
    cnt = C.c_uint64(0)
    # offsets missing while packets are claimed; count pointer missing
    assert L.pfac_scan_batch(a.handle, None, None, 3, 10, None, 0, C.byref(cnt), None) == pfac.PFAC_EINVAL
    assert L.pfac_scan_batch_async(a.handle, None, None, 0, 0, None, 0, None, None) == pfac.PFAC_EINVAL
    g = C.c_void_p(123)
    # NULL stream, NULL buffers: rejected before any device work, *out cleared
    assert L.pfac_graph_create(a.handle, None, None, 10, 0, None, 0, None, None, None,
                               C.byref(g)) == pfac.PFAC_EINVAL
    assert g.value is None
    assert L.pfac_graph_launch(None, None) == pfac.PFAC_EINVAL
    L.pfac_graph_destroy(None)


def test_tuning_rebuilds_lds_image_on_host():
    pats = [b"abcdef", b"abxy", b"zzzz", b"qq12"]
    a = pfac.pfac_build(pats, 256)
    t0 = pfac.pfac_get_tuning(a)
    assert t0["span_log2"] == 0 and t0["root_depth"] == 2 and t0["filter_k"] >= 2
    pfac.pfac_set_tuning(a, span_log2=11, root_depth=1, filter_k=3)
    t1 = pfac.pfac_get_tuning(a)
    assert (t1["span_log2"], t1["root_depth"], t1["filter_k"]) == (11, 1, 3)
    info = pfac.pfac_table_info(a)
    assert info["root_depth"] == 1 and info["filter_k"] == 3
    # out of range: shorter than the root depth, longer than the shortest pattern allows,
    # a span outside 11..16; the previous tuning stays in force
    for bad in (dict(root_depth=1, filter_k=5), dict(root_depth=3), dict(root_depth=2, filter_k=1),
                dict(span_log2=10), dict(span_log2=17), dict(lane_bytes=8), dict(lane_bytes=64),
                dict(grid=1 << 24)):
        with pytest.raises(pfac.PfacError) as e:
            pfac.pfac_set_tuning(a, **bad)
        assert e.value.code == pfac.PFAC_EINVAL
        assert pfac.pfac_get_tuning(a) == t1
    # positions per thread: 16 or 32 for the hashed form; the sampled form (the builder's
    # choice here: bytes, no pattern shorter than 4) always takes 32
    assert t1["lane_bytes"] == 32
    pfac.pfac_set_tuning(a, span_log2=11, root_depth=1, filter_k=3, lane_bytes=16)
    assert pfac.pfac_get_tuning(a)["lane_bytes"] == 16
    pfac.pfac_set_tuning(a, lane_bytes=16)
    assert pfac.pfac_get_tuning(a)["lane_bytes"] == 32
    # back to the builder's choice
    pfac.pfac_set_tuning(a)
    assert pfac.pfac_get_tuning(a) == t0


def test_tuning_cache_key_separates_workloads():
    from paper_1704_02272_amd import tuning_cache as TC
    k1 = TC.cache_key([b"ab"], 256, 100, 0, "dev")
    assert k1 == TC.cache_key([b"ab"], 256, 100, 0, "dev")
    assert len({k1, TC.cache_key([b"ab"], 256, 101, 0, "dev"), TC.cache_key([b"ab"], 4, 100, 0, "dev"),
                TC.cache_key([b"ab", b"c"], 256, 100, 0, "dev"), TC.cache_key([b"ab"], 256, 100, 3, "dev"),
                TC.cache_key([b"ab"], 256, 100, 0, "other")}) == 6


def test_host_scan_argument_errors():
    a = pfac.pfac_build([b"ab"], 256)
    L = pfac.lib()
    m = pfac.Matches()
    assert L.pfac_scan_host(a.handle, None, 10, 0, C.byref(m)) == pfac.PFAC_EINVAL
    assert L.pfac_scan_host(None, None, 0, 0, C.byref(m)) == pfac.PFAC_EINVAL
    assert L.pfac_scan_host(a.handle, None, 0, 0, None) == pfac.PFAC_EINVAL
    assert L.pfac_scan_host(a.handle, None, 0, (1 << 32) - 1, C.byref(m)) == pfac.PFAC_ETOO_LARGE
    assert not m.matches and m.count == 0
    # an empty text needs no device and returns no match
    assert L.pfac_scan_host(a.handle, None, 0, 0, C.byref(m)) == pfac.PFAC_OK and m.count == 0
    L.pfac_matches_free(C.byref(m))
    L.pfac_matches_free(None)


def test_server_argument_errors():
    L = pfac.lib()
    h = C.c_void_p(7)
    empty = pfac.pfac_build([], 256)
    # no automaton, an automaton without patterns: rejected before any device work
    assert L.pfac_server_create(None, None, C.byref(h)) == pfac.PFAC_EINVAL and h.value is None
    assert L.pfac_server_create(empty.handle, None, C.byref(h)) == pfac.PFAC_EINVAL
    t = C.c_uint64(0)
    assert L.pfac_server_submit(None, None, None, 0, 0, C.byref(t)) == pfac.PFAC_EINVAL
    n = C.c_uint32(5)
    assert L.pfac_server_poll(None, None, 0, C.byref(n), 0) == pfac.PFAC_EINVAL
    st = pfac.ServerStats()
    assert L.pfac_server_stats(None, C.byref(st), 0) == pfac.PFAC_EINVAL
    L.pfac_server_destroy(None)
    L.pfac_result_free(None)
    assert pfac.strerror(pfac.PFAC_EBUSY) == "server queue is full"
