"""Pins of the oracle's prefix depths (the quantity behind Section 2.4's truncated trie
and Section 4.2's prefix-length study): hand-derived histograms, a closed form, the
trie walk of Section 2.3 as an independent second computation, and a planted mistake."""
import numpy as np
import pytest

from oracle import prefix, trie


def test_hand_case():
    # patterns abc, abd, b; text "abcabxb"
    # s=0 "abc" -> 3; s=1 "b" -> 1 ("bc" no); s=2 "c" -> 0; s=3 "ab" then "abx" no -> 2;
    # s=4 "b" -> 1; s=5 "x" -> 0; s=6 "b" -> 1
    h = prefix.depth_histogram([b"abc", b"abd", b"b"], b"abcabxb", cap=5)
    assert h == [2, 3, 1, 1, 0, 0]
    assert prefix.survivors(h, 0) == 7 and prefix.survivors(h, 2) == 2 and prefix.survivors(h, 3) == 1
    # capped: depths of 3 or more land in the last bin
    assert prefix.depth_histogram([b"abc", b"abd", b"b"], b"abcabxb", cap=2) == [2, 3, 2]


def test_closed_form_single_run():
    # one pattern a^L over the text a^n: the depth at s is min(L, n - s, cap)
    for L, n, cap in ((3, 10, 5), (5, 4, 8), (4, 9, 2), (1, 1, 1)):
        h = prefix.depth_histogram([b"a" * L], b"a" * n, cap)
        want = [0] * (cap + 1)
        for s in range(n):
            want[min(L, n - s, cap)] += 1
        assert h == want, (L, n, cap)


def test_equals_trie_walk_on_random_sets():
    rng = np.random.default_rng(17)
    for trial in range(40):
        alphabet = int(rng.choice([2, 4, 26, 256]))
        pats = [bytes(rng.integers(0, alphabet, size=int(rng.integers(1, 9))).astype(np.uint8))
                for _ in range(int(rng.integers(1, 30)))]
        text = bytes(rng.integers(0, min(256, alphabet + 1), size=int(rng.integers(0, 300))).astype(np.uint8))
        cap = int(rng.integers(1, 10))
        offs, bms = trie.paper_layout(pats, alphabet)
        want = [0] * (cap + 1)
        for s in range(len(text)):
            want[min(cap, len(trie.walk_depths(offs, bms, text, s, alphabet)))] += 1
        assert prefix.depth_histogram(pats, text, cap) == want
        assert sum(want) == len(text)


def test_planted_mistake_fails_a_pin(monkeypatch):
    # a depth that ignores the end of the text (reads one symbol past it as a match)
    def wrong(prefixes, text, s, cap):
        d = 0
        while d < cap and bytes(text[s:s + d + 1]) in prefixes:
            d += 1
            if s + d >= len(text):
                d += 1
                break
        return min(d, cap)
    monkeypatch.setattr(prefix, "depth_at", wrong)
    with pytest.raises(AssertionError):
        test_closed_form_single_run()
