"""GPU parity of the plain table's collapsed unary paths: a node below the root image's
levels whose subtree is one path to its only terminal is stored as one tail record, and
walks compare the rest of the path at once. Cases built around that record, each
compared key for key with the oracle: paths that start right at the root image's depth
and deeper, texts ending inside a path or one symbol short of its end, a mismatch at the
path's last symbol, duplicate patterns at a path's end, a pattern that is a prefix of a
longer one (a terminal above the path), bytes outside the alphabet, packet ends inside a
path; tail lengths around the 16 path bytes kept beside each record; for the tiled scan,
the plain baseline and the prefix depths."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1704_02272_amd.pfac as pfac  # noqa: E402
from oracle import native, prefix  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _keys(a, text):
    got = pfac.keys_to_numpy(pfac.pfac_scan(a, torch.from_numpy(np.ascontiguousarray(text)).to(DEV)))
    torch.cuda.synchronize()
    return got


def _pattern_set(rng, alphabet, n):
    pats = []
    for _ in range(n):
        L = int(rng.integers(1, 40))
        pats.append(bytes(rng.integers(0, alphabet, size=L).astype(np.uint8)))
    # nested: prefixes of longer patterns, and duplicates of whole patterns
    for p in list(pats[: n // 4]):
        if len(p) > 3:
            pats.append(p[: len(p) // 2])
        pats.append(p)
    return pats


def _text_around(rng, pats, alphabet, n):
    text = rng.integers(0, min(256, alphabet + 1), size=n).astype(np.uint8)
    for _ in range(n // 40):
        p = pats[int(rng.integers(0, len(pats)))]
        o = int(rng.integers(0, max(1, n - len(p))))
        cut = int(rng.integers(0, 3))  # whole, or one / two symbols short
        q = np.frombuffer(p, np.uint8)[: max(1, len(p) - cut)].copy()
        if cut == 0 and len(p) > 2 and rng.random() < 0.2:
            q[-1] = (int(q[-1]) + 1) % max(1, alphabet)  # mismatch at the path's last symbol
        text[o:o + len(q)] = q
    return text


@pytest.mark.parametrize("alphabet", [2, 4, 26, 256])
def test_collapsed_paths_tiled_and_plain(alphabet):
    rng = np.random.default_rng(900 + alphabet)
    pats = _pattern_set(rng, alphabet, 300)
    a = pfac.pfac_build(pats, alphabet)
    info = pfac.pfac_table_info(a)
    assert info["device_tails"] > 0 and info["device_records"] < info["n_nodes"]
    ac = native.AhoCorasick(pats, alphabet)
    for n in (1, 37, 4096 + 5, 300_000):
        text = _text_around(rng, pats, alphabet, n)
        want = ac.scan(text)
        assert np.array_equal(_keys(a, text), want), n
        # the text ending inside a path: every prefix length near the end of a plant
        p = max(pats, key=len)
        for cut in range(1, min(len(p), 6)):
            t2 = np.concatenate([text, np.frombuffer(p[:-cut], np.uint8)])
            assert np.array_equal(_keys(a, t2), ac.scan(t2))
    pfac.pfac_set_tuning(a, algo="plain")
    text = _text_around(rng, pats, alphabet, 50_000)
    assert np.array_equal(_keys(a, text), ac.scan(text))
    pfac.pfac_set_tuning(a)
    h = pfac.pfac_prefix_histogram(a, torch.from_numpy(text[:20_000]).to(DEV), 40)
    assert h.cpu().tolist() == prefix.depth_histogram(pats, text[:20_000], 40)


def test_paths_at_every_depth_and_packet_ends():
    # Sigma = 4: the root image covers depth min(min_len, 8); patterns branch at depths 8..20
    rng = np.random.default_rng(77)
    base = rng.integers(0, 4, size=24).astype(np.uint8)
    pats = []
    for d in range(8, 21):
        for x in range(4):
            if x == base[d]:
                continue
            p = base.copy()
            p[d] = x
            pats.append(bytes(p[: d + 1 + int(rng.integers(0, 4))]))
    pats.append(bytes(base))
    a = pfac.pfac_build(pats, 4)
    ac = native.AhoCorasick(pats, 4)
    text = rng.integers(0, 4, size=200_000).astype(np.uint8)
    for i in range(0, len(text) - 30, 997):
        p = pats[(i // 997) % len(pats)]
        text[i:i + len(p)] = np.frombuffer(p, np.uint8)
    assert np.array_equal(_keys(a, text), ac.scan(text))
    # packets cut inside plants: no match crosses a packet end
    cuts = np.unique(np.concatenate([[0], rng.integers(1, len(text), size=3000), [len(text)]])).astype(np.uint64)
    data = torch.from_numpy(text).to(DEV)
    offs = torch.from_numpy(cuts.astype(np.int64)).to(DEV)
    got = pfac.keys_to_numpy(pfac.pfac_scan_batch(a, data, offs))
    torch.cuda.synchronize()
    assert np.array_equal(got, ac.scan_packets(text, cuts))


@pytest.mark.parametrize("alphabet", [4, 256])
def test_tail_lengths_around_the_copied_path_bytes(alphabet):
    """A walk at a tail head compares the first 16 bytes of the path from a copy kept
    beside the record and the rest from the pattern bytes: tails of 15 to 17 and 31 to
    33 bytes, mismatches at the first, 16th, 17th and last tail byte, and texts that end
    0 to 3 bytes short of a whole match, with 16 and 32 starts a lane."""
    rng = np.random.default_rng(31 + alphabet)
    head = 8 if alphabet == 4 else 2  # the root image's depth: tails start below it
    pats = []
    for i, tl in enumerate((1, 8, 15, 16, 17, 31, 32, 33, 47)):
        lead = [(i >> (2 * k)) & 3 for k in range(head)] if alphabet == 4 else [65 + i, 66]
        body = rng.integers(0, alphabet, size=tl).astype(np.uint8)
        pats.append(bytes(lead) + bytes(body))
    pieces = []
    for p in pats:
        for k in (None, head, head + 15, head + 16, len(p) - 1):
            q = bytearray(p)
            if k is not None and k < len(q):
                q[k] = (q[k] + 1) % alphabet
            pieces.append(bytes(q))
    sep = bytes([3, 2, 1, 0, 3, 3]) if alphabet == 4 else b"#~"
    body = sep.join(pieces) + sep
    ac = native.AhoCorasick(pats, alphabet)
    a = pfac.pfac_build(pats, alphabet)
    for lb in (16, 32):
        pfac.pfac_set_tuning(a, lane_bytes=lb)
        for p in pats:
            for cut in range(4):
                text = np.frombuffer(body + p[: len(p) - cut], np.uint8).copy()
                assert np.array_equal(_keys(a, text), ac.scan(text)), (alphabet, lb, len(p), cut)
