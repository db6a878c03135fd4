"""The compressed table of Section 3.2 on the host (no GPU): the builder's node counts
equal the oracle's suffix-language count, and a walker written here over the exported
records -- Eq. 1 for every step, pattern ids from the rank of the spelled string --
finds exactly the oracle's match set at every compression level. It checks the
encoding the GPU walks before any GPU run."""
import numpy as np
import pytest

import paper_1704_02272_amd.pfac as pfac
from oracle import literal, native, reduce, trie


def _child(rec, words, q, c):
    """Eq. 1 over the exported records: first child + set bits below c, or None."""
    bm = rec["bitmaps"][q]
    if not (int(bm[c >> 5]) >> (c & 31)) & 1:
        return None
    below = sum(bin(int(bm[w])).count("1") for w in range(c >> 5))
    below += bin(int(bm[c >> 5]) & ((1 << (c & 31)) - 1)).count("1")
    return int(rec["first"][q]) + below


def host_walk(a, text, alphabet):
    rec = pfac.pfac_export_records(a)
    words = (alphabet + 31) // 32
    S = rec["shared_base"]
    out = []
    text = bytes(text)
    for s in range(len(text)):
        q, u, add = 0, 0, 0
        for i in range(s, len(text)):
            c = text[i]
            if c >= alphabet:
                break
            y = _child(rec, words, q, c)
            if y is None:
                break
            if y < S:
                u = y
            else:
                add += int(rec["term"][q]) + int(rec["rank"][y])
            q = y
            if rec["term"][q]:
                r = int(rec["rank"][q]) if q < S else int(rec["rank"][u]) + add
                ids = rec["rank_ids"][rec["rank_first"][r]:rec["rank_first"][r + 1]]
                out.extend((s, int(j)) for j in ids)
    return sorted(out)


def _sets():
    rng = np.random.default_rng(41)
    yield "hand", [b"ab", b"abc", b"bc", b"c", b"ab", b"xbc", b"bbc"], 256
    yield "dna_pairs", [bytes([0, 0, 0, 1]), bytes([0, 1, 0, 1]), bytes([1, 0, 0, 1]), bytes([1, 1, 0, 1])], 4
    for sigma in (2, 4, 26, 256):
        pats = [bytes(rng.integers(0, sigma, size=int(rng.integers(1, 9))).astype(np.uint8))
                for _ in range(int(rng.integers(5, 120)))]
        yield "rand%d" % sigma, pats, sigma
    pats = sorted({bytes(rng.integers(0, 4, size=12).astype(np.uint8)) for _ in range(400)})
    yield "eq_len_dna", pats, 4


SETS = list(_sets())


@pytest.mark.parametrize("levels", [0, 1, 2, 3, 5, 255])
@pytest.mark.parametrize("case", SETS, ids=lambda c: c[0])
def test_reduced_counts_and_walk(case, levels):
    name, pats, alphabet = case
    a = pfac.pfac_build(pats, alphabet, merge_levels=levels)
    info = pfac.pfac_table_info(a)
    q = len(trie.canonical_nodes(pats))
    assert info["n_nodes"] == q
    assert info["reduced_nodes"] == reduce.reduced_node_count(pats, levels)
    assert info["reduced_paper_bytes"] == info["reduced_nodes"] * trie.paper_node_bytes(alphabet)
    assert info["table_records"] <= q
    # the paper layout export is the uncompressed trie whatever the level
    off, bm = pfac.pfac_export_paper_table(a)
    want_off, _ = trie.paper_layout(pats, alphabet)
    assert off.tolist() == want_off
    # the levels the LDS root image folds keep their breadth-first indices and bitmaps
    rec = pfac.pfac_export_records(a)
    d0 = min(min(len(p) for p in pats), 8 if alphabet <= 4 else 2)
    top = sum(1 for s in trie.canonical_nodes(pats) if len(s) <= d0)
    assert rec["shared_base"] >= top
    assert np.array_equal(rec["bitmaps"][:top], bm[:top])
    rng = np.random.default_rng(len(pats) + levels)
    hi = alphabet + (1 if alphabet < 256 else 0)
    text = bytes(rng.integers(0, hi, size=600).astype(np.uint8))
    # plant some patterns so every level sees real matches
    t = bytearray(text)
    for k in range(20):
        p = pats[int(rng.integers(0, len(pats)))]
        o = int(rng.integers(0, len(t) - len(p)))
        t[o:o + len(p)] = p
    text = bytes(t)
    want = literal.match_set(pats, text)
    assert host_walk(a, text, alphabet) == want


def test_step_1_table_keeps_one_final_block():
    """levels 1 on a prefix-free set: the final nodes become one shared block as wide as
    the widest node whose children are all final, i.e. Eq. 2's count plus the width - 1
    that Eq. 1's consecutive children need."""
    rng = np.random.default_rng(3)
    pats = sorted({bytes(rng.integers(0, 4, size=10).astype(np.uint8)) for _ in range(500)})
    a = pfac.pfac_build(pats, 4, merge_levels=1)
    info = pfac.pfac_table_info(a)
    q = len(trie.canonical_nodes(pats))
    assert info["reduced_nodes"] == trie.global_final_nodes(q, len(pats))
    off, bm = trie.paper_layout(pats, 4)
    width = max(bin(b).count("1") for b, o in zip(bm, off) if o and all(bm[c] == 0 for c in range(o, o + bin(b).count("1"))))
    assert info["table_records"] == q - len(pats) + width


def test_compression_shrinks_small_alphabets_more():
    """Section 4.1: the compression saves more with a small alphabet than with a large
    one (20-symbol random patterns)."""
    rng = np.random.default_rng(5)
    red = {}
    for sigma in (4, 52):
        pats = sorted({bytes(rng.integers(0, sigma, size=20).astype(np.uint8)) for _ in range(2000)})
        a = pfac.pfac_build(pats, sigma, merge_levels=3)
        info = pfac.pfac_table_info(a)
        red[sigma] = 1 - info["reduced_nodes"] / info["n_nodes"]
        assert 1 - info["table_records"] / info["n_nodes"] > 0.05
    assert red[4] > red[52] > 0


def test_reduced_round_trip_save_load():
    pats = [b"abc", b"bbc", b"cbc", b"ab", b"zz"]
    a = pfac.pfac_build(pats, 256, merge_levels=3)
    b = pfac.pfac_load(pfac.pfac_save(a))
    assert pfac.pfac_table_info(b) == pfac.pfac_table_info(a)
    ra, rb = pfac.pfac_export_records(a), pfac.pfac_export_records(b)
    for k in ("first", "bitmaps", "term", "rank", "rank_first", "rank_ids"):
        assert np.array_equal(ra[k], rb[k]), k


def test_merge_levels_out_of_range():
    with pytest.raises(pfac.PfacError) as e:
        pfac.pfac_build([b"ab"], 256, merge_levels=256)
    assert e.value.code == pfac.PFAC_EINVAL
