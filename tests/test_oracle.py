"""Pins for the CPU oracle: hand-derived answers, the paper's printed worked example and
byte accounting, closed forms, a library routine for overlapping occurrences, and
cross-checks between independently written algorithms. Planted mistakes (in copies of
the oracle, never in the product) show that each pin bites."""
import itertools
import json
import os
import re

import numpy as np
import pytest

from oracle import literal, native, trie

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _cases():
    return [(c["name"], c["alphabet"], [bytes.fromhex(p) for p in c["patterns"]],
             bytes.fromhex(c["text"]), [tuple(x) for x in c["expected"]])
            for c in _load("hand_cases.json")["cases"]]


def _pairs(keys):
    return [(int(k) >> 32, int(k) & 0xFFFFFFFF) for k in keys]


@pytest.fixture(scope="module", autouse=True)
def _built():
    native.build(force=False)


# ----------------------------------------------------------------------------- hand cases
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_hand_cases_all_oracles(case):
    name, alphabet, pats, text, expected = case
    assert literal.match_set(pats, text) == expected
    assert _pairs(native.brute(pats, text)) == expected
    assert _pairs(native.AhoCorasick(pats, alphabet).scan(text)) == expected
    assert trie.walk_matches(pats, alphabet, text) == expected


def test_overlapping_occurrences_via_regex_lookahead():
    """``re`` with a zero-width lookahead finds every (overlapping) occurrence of one
    pattern: a library routine the oracles did not use."""
    rng = np.random.default_rng(11)
    for _ in range(60):
        sigma = int(rng.choice([2, 3, 4]))
        pats = [bytes(rng.integers(0, sigma, size=int(rng.integers(1, 5))).astype(np.uint8))
                for _ in range(int(rng.integers(1, 6)))]
        text = bytes(rng.integers(0, sigma, size=int(rng.integers(0, 80))).astype(np.uint8))
        want = sorted((m.start(), j) for j, p in enumerate(pats)
                      for m in re.finditer(b"(?=" + re.escape(p) + b")", text))
        assert literal.match_set(pats, text) == want
        assert _pairs(native.brute(pats, text)) == want
        assert _pairs(native.AhoCorasick(pats, sigma).scan(text, chunk=7)) == want


def test_closed_form_all_binary_texts():
    """Over all 2^n binary texts, pattern p occurs (n - |p| + 1) * 2^(n - |p|) times in
    total: each start position fixes |p| bits and leaves the rest free."""
    pats = [b"\x00", b"\x01\x01", b"\x00\x01\x00", b"\x01\x01", b"\x01\x00\x01\x01"]
    n = 9
    want = sum((n - len(p) + 1) * 2 ** (n - len(p)) for p in pats if len(p) <= n)
    ac = native.AhoCorasick(pats, 2)
    got_ac = got_brute = 0
    for bits in itertools.product((0, 1), repeat=n):
        t = bytes(bits)
        got_ac += len(ac.scan(t, chunk=4))
        got_brute += len(native.brute(pats, t))
    assert got_ac == want
    assert got_brute == want


def test_random_small_cross_check():
    rng = np.random.default_rng(7)
    for trial in range(300):
        sigma = int(rng.choice([2, 4, 256]))
        npat = int(rng.integers(1, 51))
        pats = [bytes(rng.integers(0, sigma, size=int(rng.integers(1, 9))).astype(np.uint8))
                for _ in range(npat)]
        n = int(rng.integers(0, 2001)) if trial % 10 == 0 else int(rng.integers(0, 200))
        # text symbols sometimes exceed the alphabet (no transition)
        hi = sigma + (1 if sigma < 256 and trial % 3 == 0 else 0)
        text = bytes(rng.integers(0, hi, size=n).astype(np.uint8))
        want = literal.match_set(pats, text)
        assert _pairs(native.brute(pats, text)) == want
        chunk = int(rng.integers(1, 64))
        assert _pairs(native.AhoCorasick(pats, sigma).scan(text, chunk=chunk)) == want
        if trial % 5 == 0:
            assert trie.walk_matches(pats, sigma, text) == want


def test_uniform_workload_brute_equals_ac_and_contains_plants():
    from paper_1704_02272_amd import workloads as W
    w = W.uniform_256()
    b = native.brute(w.patterns, w.text)
    a = native.AhoCorasick(w.patterns, 256).scan(w.text, chunk=1 << 16)
    assert np.array_equal(a, b)
    keys = set(int(k) for k in a)
    t = w.text.tobytes()
    surviving = {(off << 32) | j for off, j in w.plants
                 if t[off:off + len(w.patterns[j])] == w.patterns[j]}
    # every plant still spelled in the final text is reported
    assert surviving <= keys
    # uniform text: expected natural matches sum_j (n-|p|+1) 256^-|p| is far below 1
    n = len(w.text)
    expect_natural = sum((n - len(p) + 1) * 256.0 ** (-len(p)) for p in w.patterns)
    assert expect_natural < 0.1
    assert len(keys - surviving) <= 3


# ------------------------------------------------------------------------- storage model
def test_worked_example_section_3_1():
    g = _load("worked_example_3_1.json")
    pats = [p.encode() for p in g["patterns"]]
    off, bm = trie.paper_layout(pats, g["alphabet"])
    a = g["node_of_A"]
    assert trie.canonical_nodes(pats)[a] == b"A"
    assert [c for c in range(256) if (bm[a] >> c) & 1] == g["children_bits_of_A"]
    assert off[a] == g["offset_of_A"]
    assert trie.child(off, bm, a, ord("B")) == g["node_of_B"]
    assert trie.popcount_below(bm[a], ord("D")) == g["popcount_below_D"]
    assert trie.child(off, bm, a, ord("D")) == g["node_of_D"]
    # the bitmap of 256 bits is 8 words of 32 bits; 'B' and 'D' sit in word 2
    assert g["bitmap_words"] * g["bitmap_word_bits"] == 256
    assert (66 // 32, 68 // 32) == (2, 2)


def test_layout_is_breadth_first_queue_order():
    rng = np.random.default_rng(3)
    for _ in range(40):
        sigma = int(rng.choice([2, 4, 26, 256]))
        pats = [bytes(rng.integers(0, sigma, size=int(rng.integers(1, 7))).astype(np.uint8))
                for _ in range(int(rng.integers(1, 40)))]
        assert trie.paper_layout(pats, sigma) == trie.bfs_queue_layout(pats, sigma)


def test_layout_offsets_count_children():
    """Breadth-first numbering: the first child of the k-th node that has children
    comes right after the children of all earlier nodes, so
    offset[k] = 1 + (sum of degrees of nodes before k); leaves keep offset 0."""
    rng = np.random.default_rng(5)
    pats = [bytes(rng.integers(0, 4, size=int(rng.integers(1, 9))).astype(np.uint8))
            for _ in range(200)]
    off, bm = trie.paper_layout(pats, 4)
    deg = [bin(b).count("1") for b in bm]
    run = 1
    for k in range(len(off)):
        if deg[k]:
            assert off[k] == run
        else:
            assert off[k] == 0
        run += deg[k]
    assert run == len(off)  # every node but the root is somebody's child
    # node count = 1 + number of distinct non-empty prefixes
    prefixes = {p[:d] for p in pats for d in range(1, len(p) + 1)}
    assert len(off) == 1 + len(prefixes)


def test_memory_accounting_section_3_1():
    g = _load("memory_accounting_3_1.json")
    for sigma, b in g["bytes_per_node"].items():
        assert trie.paper_node_bytes(int(sigma)) == b
    mib = 1 << 20
    t256, t32 = g["tries"]
    size256 = trie.paper_table_bytes(t256["nodes"], 256) / mib
    size32 = trie.paper_table_bytes(t32["nodes"], 32) / mib
    assert int(size256 * 10) / 10 == t256["printed_mb"]
    assert int(size32 * 10) / 10 == t32["printed_mb"]
    assert round(t256["other_system_mb"] / t256["printed_mb"], 1) == t256["printed_ratio"]
    for k, ratio in t32["printed_ratios"].items():
        assert round(t32["other_systems_mb"][k] / t32["printed_mb"], 2) == ratio


def test_global_final_node_count_eq_2():
    """Eq. 2 on a set where every pattern ends in its own childless leaf (prefix-free,
    no duplicates): merging all final nodes into one removes |P| - 1 nodes. Counted
    here directly on the node set."""
    rng = np.random.default_rng(9)
    pats = set()
    while len(pats) < 60:
        pats.add(bytes(rng.integers(0, 4, size=6).astype(np.uint8)))  # equal length: prefix-free
    pats = sorted(pats)
    nodes = trie.canonical_nodes(pats)
    leaves = [s for s in nodes if s in pats]
    merged = len(nodes) - len(leaves) + 1
    assert trie.global_final_nodes(len(nodes), len(pats)) == merged


# ---------------------------------------------------------------------- planted mistakes
def test_pins_catch_planted_mistakes_in_c_oracle(tmp_path):
    cases = _cases()

    def hand_ok(lib):
        for name, alphabet, pats, text, expected in cases:
            if _pairs(native.brute(pats, text, lib=lib)) != expected:
                return False
            if _pairs(native.AhoCorasick(pats, alphabet, lib=lib).scan(text)) != expected:
                return False
        return True

    for define in ("ORC_MUTANT_BRUTE_END", "ORC_MUTANT_NO_DICT", "ORC_MUTANT_ROOT_FAIL"):
        lib = native.build_mutant(define, str(tmp_path))
        assert not hand_ok(lib), define
    # a too-short chunk overlap only shows when a match crosses a chunk end
    lib = native.build_mutant("ORC_MUTANT_SHORT_OVERLAP", str(tmp_path))
    pats = [b"abcd"]
    text = b"xxabcdxx"
    assert _pairs(native.AhoCorasick(pats, 256, lib=lib).scan(text, chunk=3)) != \
        literal.match_set(pats, text)


def test_pins_catch_planted_mistakes_in_python_oracle(monkeypatch):
    cases = _cases()

    def off_by_one(patterns, text):  # stops one start early
        text = bytes(text)
        return [(s, j) for s in range(len(text) - 1) for j, p in enumerate(patterns)
                if p and s + len(p) <= len(text) and text[s:s + len(p)] == p]

    def popcount_inclusive(bitmap, c):  # counts bit c itself
        return bin(bitmap & ((1 << (c + 1)) - 1)).count("1")

    assert any(off_by_one(p, t) != e for _, _, p, t, e in cases)
    monkeypatch.setattr(trie, "popcount_below", popcount_inclusive)
    g = _load("worked_example_3_1.json")
    pats = [p.encode() for p in g["patterns"]]
    off, bm = trie.paper_layout(pats, 256)
    assert trie.child(off, bm, 1, ord("D")) != g["node_of_D"]


# ------------------------------------------------------------------------ packet batches
def _batch_cases():
    out = []
    for c in _load("packet_batches.json")["cases"]:
        data = b"".join(bytes.fromhex(p) for p in c["data_parts"])
        offs = np.array(c["offsets"], dtype=np.uint64)
        # the parts are the packets: the offsets must cut the data at their ends
        ends = np.cumsum([0] + [len(bytes.fromhex(p)) for p in c["data_parts"]])
        assert list(ends) == c["offsets"]
        out.append((c["name"], c["alphabet"], [bytes.fromhex(p) for p in c["patterns"]],
                    data, offs, [tuple(x) for x in c["expected"]]))
    return out


def _random_batch(rng, sigma, n_pk, max_pk):
    sizes = rng.integers(0, max_pk + 1, size=n_pk)
    sizes[rng.random(n_pk) < 0.2] = 0          # empty packets
    sizes[rng.random(n_pk) < 0.1] = 1          # one-byte packets
    offs = np.zeros(n_pk + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(sizes)
    data = rng.integers(0, sigma, size=int(offs[-1])).astype(np.uint8)
    return data, offs


def _per_packet_literal(pats, data, offs):
    """Each packet matched alone with the plain definition, starts moved by the
    packet's first byte: written out here, independent of both oracle helpers."""
    out = []
    raw = bytes(data)
    for i in range(len(offs) - 1):
        a, b = int(offs[i]), int(offs[i + 1])
        out.extend((a + s, j) for s, j in literal.match_set(pats, raw[a:b]))
    return out


@pytest.mark.parametrize("case", _batch_cases(), ids=lambda c: c[0])
def test_packet_batch_hand_cases(case):
    name, alphabet, pats, data, offs, expected = case
    arr = np.frombuffer(data, dtype=np.uint8)
    assert _pairs(native.AhoCorasick(pats, alphabet).scan_packets(arr, offs)) == expected
    assert literal.match_set_packets(pats, data, offs) == expected
    assert literal.keys(expected) == [(s << 32) | j for s, j in expected]


def test_packet_batch_random_against_per_packet_definition():
    rng = np.random.default_rng(21)
    for trial in range(120):
        sigma = int(rng.choice([2, 4, 256]))
        pats = [bytes(rng.integers(0, sigma, size=int(rng.integers(1, 7))).astype(np.uint8))
                for _ in range(int(rng.integers(1, 25)))]
        data, offs = _random_batch(rng, sigma, int(rng.integers(1, 40)), int(rng.integers(1, 60)))
        want = _per_packet_literal(pats, data, offs)
        assert _pairs(native.AhoCorasick(pats, sigma).scan_packets(data, offs)) == want
        assert literal.match_set_packets(pats, data.tobytes(), offs) == want
        # brute force over each packet, keys shifted by the packet's first byte
        parts = [native.brute(pats, data[int(offs[i]):int(offs[i + 1])]) + np.uint64(int(offs[i]) << 32)
                 for i in range(len(offs) - 1)]
        got = np.concatenate(parts) if parts else np.zeros(0, np.uint64)
        assert _pairs(np.sort(got)) == want


def test_keys_hand_values():
    """(s << 32) | j: start in the high word, id in the low word, so numeric order is
    (start, id) order."""
    assert literal.keys([(0, 5), (1, 2), (1, 7), (4294967295, 4294967295)]) == [
        5, 4294967298, 4294967303, 18446744073709551615]
    assert literal.keys([]) == []
    k = literal.keys([(3, 9), (2, 100), (3, 1)])
    assert sorted(k) == literal.keys([(2, 100), (3, 1), (3, 9)])


def test_packet_pins_catch_planted_mistakes():
    """Copies of the packet scan with a plausible mistake each fail a pin above."""
    cases = _batch_cases()

    class ByIndex(native.AhoCorasick):       # shifts starts by the packet index
        def scan_packets(self, data, offsets, threads=0):
            parts = []
            for i in range(len(offsets) - 1):
                k = self.scan(np.asarray(data)[int(offsets[i]):int(offsets[i + 1])], threads=1)
                parts.append(k + np.uint64(i << 32))
            return np.concatenate(parts) if parts else np.zeros(0, np.uint64)

    class DropLast(native.AhoCorasick):      # forgets the last packet
        def scan_packets(self, data, offsets, threads=0):
            return super().scan_packets(data, offsets[:-1], threads)

    class Concatenated(native.AhoCorasick):  # scans the batch as one text
        def scan_packets(self, data, offsets, threads=0):
            return self.scan(np.asarray(data)[:int(offsets[-1])])

    for bad in (ByIndex, DropLast, Concatenated):
        caught = any(_pairs(bad(p, a).scan_packets(np.frombuffer(d, np.uint8), o)) != e
                     for _, a, p, d, o, e in cases)
        assert caught, bad.__name__

    def literal_no_shift(patterns, data, offsets):   # forgets the packet base
        out = []
        for i in range(len(offsets) - 1):
            a, b = int(offsets[i]), int(offsets[i + 1])
            out.extend(literal.match_set(patterns, bytes(data)[a:b]))
        return sorted(out)

    assert any(literal_no_shift(p, d, o) != e for _, _, p, d, o, e in cases)


# ------------------------------------------------------------- compression (Section 3.2)
from oracle import reduce  # noqa: E402


def _reduction_cases():
    g = _load("reduction_3_2.json")
    return [(c["name"], [bytes.fromhex(p) for p in c["patterns"]], c["trie_nodes"],
             {int(k): v for k, v in c["by_levels"].items()}) for c in g["cases"]]


@pytest.mark.parametrize("case", _reduction_cases(), ids=lambda c: c[0])
def test_reduction_hand_cases(case):
    name, pats, q, by_levels = case
    assert len(trie.canonical_nodes(pats)) == q
    for levels, want in by_levels.items():
        assert reduce.reduced_node_count(pats, levels) == want, levels


def _moore_minimal_states(patterns, alphabet):
    """States of the minimal DFA of the finite pattern language, by Moore's partition
    refinement on the trie automaton completed with a dead state (a textbook algorithm
    that shares nothing with the suffix-language count). The dead state is excluded."""
    nodes = trie.canonical_nodes(patterns)
    index = {s: i for i, s in enumerate(nodes)}
    dead = len(nodes)
    pset = {bytes(p) for p in patterns}
    syms = sorted({c for p in patterns for c in p})
    delta = [[index.get(s + bytes([c]), dead) for c in syms] for s in nodes] + [[dead] * len(syms)]
    cls = [1 if s in pset else 0 for s in nodes] + [0]
    while True:
        sig = [(cls[q],) + tuple(cls[t] for t in delta[q]) for q in range(len(delta))]
        ids = {}
        new = [ids.setdefault(x, len(ids)) for x in sig]
        if len(ids) == len(set(cls)):
            break
        cls = new
    return len(set(cls)) - 1


def test_full_reduction_is_the_minimal_automaton():
    rng = np.random.default_rng(13)
    for _ in range(60):
        sigma = int(rng.choice([2, 3, 4, 26]))
        pats = [bytes(rng.integers(0, sigma, size=int(rng.integers(1, 9))).astype(np.uint8))
                for _ in range(int(rng.integers(1, 40)))]
        assert reduce.reduced_node_count(pats, 64) == _moore_minimal_states(pats, sigma)


def test_reduction_step_1_is_eq_2():
    """levels = 1 merges only the final nodes: on prefix-free sets without duplicates
    this is Eq. 2, Q - (|P| - 1)."""
    rng = np.random.default_rng(17)
    for _ in range(20):
        sigma = int(rng.choice([2, 4, 52]))
        m = int(rng.integers(2, 10))
        pats = sorted({bytes(rng.integers(0, sigma, size=m).astype(np.uint8))
                       for _ in range(int(rng.integers(1, 200)))})
        q = len(trie.canonical_nodes(pats))
        assert reduce.reduced_node_count(pats, 1) == trie.global_final_nodes(q, len(pats))


def test_reduction_is_monotone_and_bounded():
    rng = np.random.default_rng(19)
    pats = [bytes(rng.integers(0, 4, size=int(rng.integers(3, 12))).astype(np.uint8)) for _ in range(300)]
    q = len(trie.canonical_nodes(pats))
    counts = [reduce.reduced_node_count(pats, k) for k in range(0, 14)]
    assert counts[0] == q                       # nothing merged
    assert all(a >= b for a, b in zip(counts, counts[1:]))
    assert counts[-1] == _moore_minimal_states(pats, 4)


def test_eq_4_occupancy_law():
    """P(g = i) from adding patterns one at a time equals the closed occupancy form
    C(r, i) i! S(n, i) / r^n (S: Stirling numbers of the second kind, from scipy), sums
    to 1, and its mean is r (1 - (1 - 1/r)^n)."""
    from math import comb, factorial
    from fractions import Fraction
    from scipy.special import stirling2
    for n, r in [(1, 16), (5, 16), (12, 16), (30, 16), (20, 2704), (40, 9)]:
        p = reduce.distinct_chain_distribution(n, r)
        assert sum(p) == 1
        for i in range(n + 1):
            closed = Fraction(comb(r, i) * factorial(i) * int(stirling2(n, i, exact=True)), r ** n)
            assert p[i] == closed, (n, r, i)
        mean = sum(i * pi for i, pi in enumerate(p))
        assert mean == r * (1 - (1 - Fraction(1, r)) ** n)
    assert reduce.chains(4) == 16 and reduce.chains(52) == 2704


def test_eq_4_against_monte_carlo():
    """Two-symbol suffixes of random equal-length patterns: the mean number of distinct
    ones over many draws approaches E[g] (and 2 E[g] is Eq. 4's node estimate)."""
    rng = np.random.default_rng(23)
    for sigma, n in [(4, 10), (4, 40), (8, 100)]:
        trials = 3000
        tails = rng.integers(0, sigma, size=(trials, n, 2))
        g = np.array([len({(int(a), int(b)) for a, b in t}) for t in tails])
        want = float(reduce.expected_reduced_tail_nodes(n, sigma)) / 2
        sd = g.std() / np.sqrt(trials)
        assert abs(g.mean() - want) < 5 * sd + 1e-9, (sigma, n, g.mean(), want)


def test_reduction_planted_mistakes_fail_pins():
    """A count that merges by height alone (ignoring the suffixes), and one that also
    merges nodes of height `levels`, each fail the hand cases."""
    cases = _reduction_cases()

    def by_height_only(pats, levels):
        h = reduce.heights(pats)
        return sum(1 for s in h if h[s] >= levels) + len({h[s] for s in h if h[s] < levels})

    def off_by_one(pats, levels):
        return reduce.reduced_node_count(pats, levels + 1)

    for bad in (by_height_only, off_by_one):
        assert any(bad(p, k) != v for _, p, _, bl in cases for k, v in bl.items()), bad.__name__
