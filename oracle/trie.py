"""The paper's storage model of the trie (test infrastructure only).

Section 3.1 builds the trie from the patterns sorted alphabetically, breadth-first, into
one contiguous array of nodes. A node keeps only

  * the offset of (index of) its first child, 0 when it has no child, and
  * a child bitmap with one bit per alphabet symbol.

Eq. 1 walks it: the child for symbol c of node q is node offset(q) + i, where i is the
number of bits of q's bitmap that are set below bit c. Section 3.1 also prices a node at
4 bytes of offset plus |Sigma| bits of bitmap (36 bytes at |Sigma| = 256, 8 bytes at 32).

This module writes that array out from its definition: the node set is the empty prefix
plus every distinct non-empty prefix of a pattern; breadth-first numbering with children
taken in increasing symbol order numbers the nodes by (depth, lexicographic order of the
prefix). Pattern identity is not part of the paper's node (a node is "final" when it has
no child); the walker below therefore reports, for each start, the depths at which it
reaches a state that spells a whole pattern, using the pattern set itself.
"""
from __future__ import annotations


def canonical_nodes(patterns) -> list:
    """Node strings in breadth-first order: the empty prefix, then all distinct
    non-empty prefixes sorted by (length, bytes)."""
    pre = set()
    for p in patterns:
        for d in range(1, len(p) + 1):
            pre.add(bytes(p[:d]))
    return [b""] + sorted(pre, key=lambda x: (len(x), x))


def paper_layout(patterns, alphabet: int):
    """(offsets, bitmaps) of the Section 3.1 array. ``bitmaps[q]`` is a Python int whose
    bit c is set when node q has a child on symbol c."""
    nodes = canonical_nodes(patterns)
    index = {s: i for i, s in enumerate(nodes)}
    first = [0] * len(nodes)
    bitmaps = [0] * len(nodes)
    for s, i in index.items():
        if not s:
            continue
        parent = index[s[:-1]]
        c = s[-1]
        if c >= alphabet:
            raise ValueError("pattern symbol outside the alphabet")
        bitmaps[parent] |= 1 << c
        if first[parent] == 0 or i < first[parent]:
            first[parent] = i
    return first, bitmaps


def bfs_queue_layout(patterns, alphabet: int):
    """The same array built the way Section 3.1 describes it: an explicit queue,
    breadth-first, children enqueued in increasing symbol order. Used to check that the
    (depth, lexicographic) numbering of ``paper_layout`` is the breadth-first one."""
    children = {b"": set()}
    for p in patterns:
        for d in range(1, len(p) + 1):
            children.setdefault(bytes(p[:d]), set())
            children[bytes(p[:d - 1])].add(p[d - 1])
    order = []
    queue = [b""]
    head = 0
    offsets, bitmaps = [], []
    next_free = 1
    while head < len(queue):
        s = queue[head]
        head += 1
        order.append(s)
        kids = sorted(children[s])
        bm = 0
        for c in kids:
            bm |= 1 << c
            queue.append(s + bytes([c]))
        offsets.append(next_free if kids else 0)
        bitmaps.append(bm)
        next_free += len(kids)
    return offsets, bitmaps


def popcount_below(bitmap: int, c: int) -> int:
    """The i of Eq. 1: set bits of ``bitmap`` strictly below bit c."""
    return bin(bitmap & ((1 << c) - 1)).count("1")


def child(offsets, bitmaps, q: int, c: int):
    """Eq. 1: the node reached from q on symbol c, or None when the bit is clear."""
    if c < 0 or not (bitmaps[q] >> c) & 1:
        return None
    return offsets[q] + popcount_below(bitmaps[q], c)


def walk_depths(offsets, bitmaps, text, s: int, alphabet: int) -> list:
    """Failure-less walk from start s (Section 2.3): follow Eq. 1 while the next text
    symbol has a child; return the nodes visited (node after 1, 2, ... symbols)."""
    q = 0
    visited = []
    for d in range(s, len(text)):
        c = text[d]
        if c >= alphabet:
            break
        nq = child(offsets, bitmaps, q, c)
        if nq is None:
            break
        q = nq
        visited.append(q)
    return visited


def walk_matches(patterns, alphabet: int, text) -> list:
    """M(T) via failure-less walks over the Section 3.1 array. A walk that has consumed
    d symbols from s has spelled text[s:s+d]; every pattern equal to that string is a
    match (pattern identity comes from the pattern list, not the node)."""
    offsets, bitmaps = paper_layout(patterns, alphabet)
    by_string = {}
    for j, p in enumerate(patterns):
        by_string.setdefault(bytes(p), []).append(j)
    text = bytes(text)
    out = []
    for s in range(len(text)):
        visited = walk_depths(offsets, bitmaps, text, s, alphabet)
        found = []
        for d in range(1, len(visited) + 1):
            found.extend(by_string.get(text[s:s + d], ()))
        out.extend((s, j) for j in sorted(found))
    return out


def paper_node_bytes(alphabet: int) -> int:
    """Section 3.1 accounting: 4 bytes of offset plus |Sigma| bits of bitmap."""
    return 4 + (alphabet + 7) // 8


def paper_table_bytes(n_nodes: int, alphabet: int) -> int:
    return n_nodes * paper_node_bytes(alphabet)


def global_final_nodes(n_nodes: int, n_patterns: int) -> int:
    """Eq. 2: node count after merging every pattern's (childless) final node into one."""
    return n_nodes - (n_patterns - 1)
