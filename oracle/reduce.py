"""The paper's trie compression (Section 3.2) as a node count (test infrastructure only).

Section 3.2 shrinks the trie of Section 3.1 in two steps. Step 1 merges the final node
of every pattern into one global final node; Eq. 2 counts what remains,
Q_final = Q - (|P| - 1), which holds when every pattern ends in its own childless node.
Step 2 merges nodes of the last three levels whose suffixes agree. Eq. 3 and Eq. 4
estimate step 2's result for random patterns: with r = |Sigma|^2 possible chains of two
symbols, the expected size of the merged bottom levels is the sum over i of
P(g = i) * 2i, where g is the number of distinct two-symbol suffix chains.

Reading used here (the figure of Section 3.2 is missing and Eq. 4 is garbled):

* Two nodes may be merged when everything below them is the same: the same set of
  suffixes that complete a pattern from there (their "suffix language"), which also
  fixes whether the node itself ends a pattern. Merging them changes no match.
* "The last three levels" are the nodes whose height -- the longest path down to a
  leaf -- is 0, 1 or 2. For patterns of one length (the paper's experiments use
  20-symbol patterns) these are exactly the bottom three depths. ``levels`` generalises
  this: nodes of height below ``levels`` are merged; ``levels = 1`` merges only the
  leaves, which is step 1 alone; a large ``levels`` merges everything mergeable (the
  minimal acyclic automaton of the pattern set).
* Eq. 4 is read as an occupancy law: n patterns drop their last two symbols into
  r = |Sigma|^2 equally likely chains; g is the number of chains hit. Its distribution
  is computed here by adding the patterns one at a time (each new pattern lands on a
  chain already hit with probability i / r), and 2 * E[g] is the expected node count.

The node count is the paper's own measure (Figs. 4 and 5 plot trie sizes); bytes are
nodes x (4 + ceil(|Sigma| / 8)) as in Section 3.1.
"""
from __future__ import annotations

from fractions import Fraction

from . import trie


def suffix_languages(patterns):
    """{prefix string: frozenset of suffixes w with prefix + w a pattern} for every trie
    node (the empty prefix is the root). Duplicates collapse: a language is a set."""
    pset = {bytes(p) for p in patterns}
    nodes = trie.canonical_nodes(patterns)
    kids = {s: [] for s in nodes}
    for s in nodes:
        if s:
            kids[s[:-1]].append(s)
    lang = {}
    # deepest first, so a node's children are done before it
    for s in sorted(nodes, key=len, reverse=True):
        words = set()
        if s in pset:
            words.add(b"")
        for child in kids[s]:
            c = child[-1:]
            words.update(c + w for w in lang[child])
        lang[s] = frozenset(words)
    return lang


def heights(patterns):
    """{prefix string: longest distance from that node down to a leaf}."""
    lang = suffix_languages(patterns)
    return {s: max(len(w) for w in L) for s, L in lang.items()}


def reduced_node_count(patterns, levels: int = 3) -> int:
    """Nodes left after merging every group of nodes with height < ``levels`` that have
    the same suffix language (nodes of height >= ``levels`` stay as they are)."""
    lang = suffix_languages(patterns)
    kept = 0
    merged = set()
    for s, L in lang.items():
        h = max(len(w) for w in L)
        if h < levels:
            merged.add(L)
        else:
            kept += 1
    return kept + len(merged)


def reduced_table_bytes(patterns, alphabet: int, levels: int = 3) -> int:
    return reduced_node_count(patterns, levels) * trie.paper_node_bytes(alphabet)


def chains(alphabet: int) -> int:
    """Eq. 3: two-symbol chains over the alphabet."""
    return alphabet * alphabet


def distinct_chain_distribution(n: int, r: int) -> list:
    """P(g = i) for i = 0..n: the number of distinct chains hit when n patterns each land
    on one of r equally likely chains, by adding the patterns one at a time. Exact
    fractions."""
    p = [Fraction(1)] + [Fraction(0)] * n
    for k in range(n):
        q = [Fraction(0)] * (n + 1)
        for i in range(k + 1):
            if p[i]:
                q[i] += p[i] * Fraction(i, r)              # a chain already hit
                if i + 1 <= n:
                    q[i + 1] += p[i] * Fraction(r - i, r)  # a new chain
        p = q
    return p


def expected_reduced_tail_nodes(n: int, alphabet: int) -> Fraction:
    """Eq. 4 in the occupancy reading: sum over i of P(g = i) * 2i."""
    r = chains(alphabet)
    return sum(2 * i * pi for i, pi in enumerate(distinct_chain_distribution(n, r)))
