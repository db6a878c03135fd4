"""The match set from its definition, in plain Python (test infrastructure only).

Section 2.2 states the problem: find every occurrence of every pattern of a set in a
text. A failure-less walk from start s (Section 2.3) reaches the terminal state of
pattern j exactly when the text from s spells p_j, so the result of the method is

    M(T) = { (s, j) : s + |p_j| <= |T| and T[s : s + |p_j|] == p_j },

reported in increasing (s, j) order. This module computes M by comparing every pattern at
every start; it is quadratic and meant for inputs of a few thousand bytes.
"""
from __future__ import annotations


def match_set(patterns, text) -> list:
    """All (start, pattern_id) pairs with the pattern spelled at start, sorted."""
    text = bytes(text)
    n = len(text)
    out = []
    for s in range(n):
        for j, p in enumerate(patterns):
            L = len(p)
            if L and s + L <= n and text[s:s + L] == p:
                out.append((s, j))
    return out


def match_set_packets(patterns, data, offsets) -> list:
    """Per-packet match sets, each start shifted to its global byte offset: a match
    never crosses a packet end."""
    data = bytes(data)
    out = []
    for i in range(len(offsets) - 1):
        a, b = int(offsets[i]), int(offsets[i + 1])
        out.extend((a + s, j) for s, j in match_set(patterns, data[a:b]))
    return out


def keys(pairs) -> list:
    """Pairs (s, j) as the 64-bit keys (s << 32) | j, whose numeric order is (s, j)."""
    return [(s << 32) | j for s, j in pairs]
