"""Prefix depths of a text against a pattern set (test infrastructure only).

Section 2.4 truncates the trie to its first k levels and lets a second stage confirm
the candidates; Section 4.2 measures how long the prefix must be before that first stage
stops producing false positives, for each alphabet. Both rest on one quantity per start
position s: the length of the longest prefix of some pattern that the text spells from
s, i.e. how deep a failure-less walk (Section 2.3) gets before a transition is missing.

This module computes it from the definition (the set of all pattern prefixes), not from
any trie, and summarises it as a histogram: hist[d] = number of starts whose depth is d,
for d < cap, and hist[cap] = number of starts of depth cap or more.
"""
from __future__ import annotations


def prefix_set(patterns) -> set:
    """Every non-empty prefix of every pattern, as bytes."""
    out = set()
    for p in patterns:
        p = bytes(p)
        for k in range(1, len(p) + 1):
            out.add(p[:k])
    return out


def depth_at(prefixes: set, text: bytes, s: int, cap: int) -> int:
    """Length of the longest pattern prefix spelled by text from s, at most cap."""
    d = 0
    while d < cap and s + d < len(text) and bytes(text[s:s + d + 1]) in prefixes:
        d += 1
    return d


def depth_histogram(patterns, text, cap: int) -> list:
    """hist[d] for d = 0 .. cap (the last bin holds depths >= cap)."""
    pre = prefix_set(patterns)
    text = bytes(text)
    hist = [0] * (cap + 1)
    for s in range(len(text)):
        hist[depth_at(pre, text, s, cap)] += 1
    return hist


def survivors(hist, k: int) -> int:
    """Starts that a trie truncated after k levels lets through: depth >= k."""
    return sum(hist[k:])
