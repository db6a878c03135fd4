"""Seeded synthetic inputs for the matcher: pattern sets, texts, packet batches and
request streams.

This module holds no part of the matching method. It only draws random bytes, so the
oracle (under ``oracle/``) and the HIP path can both be fed from it without sharing any
arithmetic of the method.

The paper measures on synthetic files made with a Mersenne Twister generator and
checks their distinctness with SHA-256 (Section 4, opening paragraphs). Here every
workload is drawn from ``numpy.random.default_rng(seed)`` and carries the SHA-256 of
its buffers, so a run can state exactly which bytes it scanned.

Workloads (sizes are the defaults; each generator takes its sizes as keyword arguments
so tests can draw small variants of the same shape):

* ``uniform_256``      -- alphabet 256, 100 patterns of uniform bytes (length 4-16),
                          1 MiB uniform text, 1,000 planted pattern copies.
* ``printable_256``    -- alphabet 256, 5,000 patterns (log-normal length, median 12,
                          clipped 4-64, 70 % printable bytes, 20 % sharing a 4-byte
                          prefix with another pattern), 256 MiB text 90 % printable,
                          one planted copy per 64 KiB.
* ``dna_4``            -- alphabet 4 (byte codes 0-3), 10,000 patterns (length 8-32),
                          1 GiB order-2 Markov text, one planted copy per MiB.
* ``packets_256``      -- 65,536 packets of 64 / 576 / 1500 bytes (40/20/40 %), 80 %
                          printable; 20,000 patterns (length 4-128) whose first bytes
                          follow a random branching-3 trie of depth 6.
* ``serving_256``      -- Poisson request stream of 32-packet batches, packet sizes
                          uniform over {64, 512, 1500, 9000}, 50,000 patterns
                          (log-normal length, median 16, clipped 4-256).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

PRINTABLE_LO = 0x20
PRINTABLE_HI = 0x7E  # inclusive: 95 printable ASCII values
_CHUNK = 1 << 24


def sha256_of(buf) -> str:
    h = hashlib.sha256()
    mv = memoryview(np.ascontiguousarray(buf)).cast("B")
    for i in range(0, len(mv), 1 << 26):
        h.update(mv[i:i + (1 << 26)])
    return h.hexdigest()


def mixed_bytes(rng: np.random.Generator, n: int, p_printable: float) -> np.ndarray:
    """``n`` bytes; each independently printable-uniform with probability
    ``p_printable``, else uniform over 0..255. Generated in chunks to bound memory."""
    out = np.empty(n, dtype=np.uint8)
    thr = int(round(p_printable * 65536))
    for a in range(0, n, _CHUNK):
        m = min(_CHUNK, n - a)
        u = rng.integers(0, 256, size=m, dtype=np.uint8)
        pr = rng.integers(PRINTABLE_LO, PRINTABLE_HI + 1, size=m, dtype=np.uint8)
        sel = rng.integers(0, 65536, size=m, dtype=np.uint16) < thr
        np.copyto(u, pr, where=sel)
        out[a:a + m] = u
    return out


def lognormal_lengths(rng, count, median, sigma, lo, hi) -> np.ndarray:
    x = np.exp(rng.normal(np.log(median), sigma, size=count))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


@dataclass
class TextWorkload:
    """A pattern set plus one contiguous text."""
    name: str
    alphabet: int
    patterns: list            # list[bytes]
    text: np.ndarray          # uint8[n]
    seed: int
    plants: list = field(default_factory=list)   # (offset, pattern_id), in apply order
    recipe: str = ""

    @property
    def max_len(self) -> int:
        return max((len(p) for p in self.patterns), default=0)

    def sha256(self) -> dict:
        return {"text": sha256_of(self.text),
                "patterns": hashlib.sha256(b"".join(len(p).to_bytes(4, "little") + p
                                                    for p in self.patterns)).hexdigest()}


@dataclass
class PacketWorkload:
    """A pattern set plus a CSR batch of packets: packet i is
    ``data[offsets[i]:offsets[i+1]]``."""
    name: str
    alphabet: int
    patterns: list
    data: np.ndarray          # uint8[total]
    offsets: np.ndarray       # uint64[n_packets + 1]
    seed: int
    plants: list = field(default_factory=list)   # (packet, offset-in-packet, pattern_id)
    recipe: str = ""

    @property
    def n_packets(self) -> int:
        return len(self.offsets) - 1

    @property
    def max_len(self) -> int:
        return max((len(p) for p in self.patterns), default=0)

    def packet(self, i: int) -> np.ndarray:
        return self.data[int(self.offsets[i]):int(self.offsets[i + 1])]


def _plant(rng, text, patterns, count, block=None):
    """Copy ``count`` uniformly chosen patterns into ``text``. Without ``block`` the
    offset is uniform over the whole text; with ``block`` there is one copy per block,
    placed wholly inside it. Plants are applied in order, so a later one may overwrite
    part of an earlier one; the match set of the final text is what counts."""
    n = len(text)
    plants = []
    for b in range(count):
        j = int(rng.integers(0, len(patterns)))
        p = patterns[j]
        if block is None:
            if len(p) > n:
                continue
            off = int(rng.integers(0, n - len(p) + 1))
        else:
            lo = b * block
            hi = min(n, lo + block)
            if len(p) > hi - lo:
                continue
            off = lo + int(rng.integers(0, hi - lo - len(p) + 1))
        text[off:off + len(p)] = np.frombuffer(p, dtype=np.uint8)
        plants.append((off, j))
    return plants


def uniform_256(seed: int = 1, text_bytes: int = 1 << 20, n_patterns: int = 100,
                n_plants: int = 1000) -> TextWorkload:
    """Alphabet 256: uniform-byte patterns of length 4..16, uniform text, planted copies
    at uniform offsets."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(4, 17, size=n_patterns)
    pats = [rng.integers(0, 256, size=int(L), dtype=np.uint8).tobytes() for L in lens]
    text = rng.integers(0, 256, size=text_bytes, dtype=np.uint8)
    plants = _plant(rng, text, pats, n_plants)
    return TextWorkload("uniform_256", 256, pats, text, seed, plants,
                        "patterns U{4..16} x U{0..255}; text U{0..255}; plants at U offsets")


def printable_256(seed: int = 2, text_bytes: int = 1 << 28, n_patterns: int = 5000,
                  plant_block: int = 1 << 16) -> TextWorkload:
    """Alphabet 256, text and patterns biased to printable ASCII (the shape of IDS
    signatures and traffic)."""
    rng = np.random.default_rng(seed)
    lens = lognormal_lengths(rng, n_patterns, 12.0, 0.5, 4, 64)
    pats = [bytearray(mixed_bytes(rng, int(L), 0.70).tobytes()) for L in lens]
    # 20 % of the patterns take their first 4 bytes from another, uniformly chosen one.
    n_share = n_patterns // 5
    takers = rng.choice(n_patterns, size=n_share, replace=False)
    for t in takers:
        d = int(rng.integers(0, n_patterns - 1))
        d = d + 1 if d >= t else d
        pats[t][0:4] = pats[d][0:4]
    pats = [bytes(p) for p in pats]
    text = mixed_bytes(rng, text_bytes, 0.90)
    plants = _plant(rng, text, pats, text_bytes // plant_block, block=plant_block)
    return TextWorkload("printable_256", 256, pats, text, seed, plants,
                        "patterns lognormal(ln 12, 0.5) clip 4..64, 70% printable, 20% share "
                        "a 4-byte prefix; text 90% printable; 1 plant per 64 KiB block")


def markov2_dna(rng: np.random.Generator, n: int, segment: int = 1 << 14) -> np.ndarray:
    """Order-2 Markov text over codes 0..3. The 16 two-symbol contexts each get a
    next-symbol distribution drawn from Dirichlet(1,1,1,1). The text is generated as
    independent chain segments of ``segment`` symbols (first two symbols of each
    uniform) so the loop runs over positions-in-segment with all segments vectorised."""
    probs = rng.dirichlet(np.ones(4), size=16)
    cum = np.cumsum(probs, axis=1)[:, :3]
    thr = np.minimum(np.floor(cum * 2.0 ** 32), 2.0 ** 32 - 1).astype(np.uint64)
    nseg = -(-n // segment)
    out = np.empty((segment, nseg), dtype=np.uint8)
    out[0] = rng.integers(0, 4, size=nseg, dtype=np.uint8)
    if segment > 1:
        out[1] = rng.integers(0, 4, size=nseg, dtype=np.uint8)
    t0, t1, t2 = thr[:, 0], thr[:, 1], thr[:, 2]
    for i in range(2, segment):
        ctx = (out[i - 2].astype(np.intp) << 2) | out[i - 1]
        r = rng.integers(0, 1 << 32, size=nseg, dtype=np.uint64)
        out[i] = ((r >= t0[ctx]).astype(np.uint8) + (r >= t1[ctx]) + (r >= t2[ctx]))
    return np.ascontiguousarray(out.T).reshape(-1)[:n]


def dna_4(seed: int = 3, text_bytes: int = 1 << 30, n_patterns: int = 10000,
          plant_block: int = 1 << 20, segment: int = 1 << 14) -> TextWorkload:
    """Alphabet 4 (DNA, one byte per base, codes 0..3): uniform patterns of length 8..32,
    order-2 Markov text, one planted copy per MiB."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(8, 33, size=n_patterns)
    pats = [rng.integers(0, 4, size=int(L), dtype=np.uint8).tobytes() for L in lens]
    text = markov2_dna(rng, text_bytes, segment)
    plants = _plant(rng, text, pats, max(1, text_bytes // plant_block), block=plant_block)
    return TextWorkload("dna_4", 4, pats, text, seed, plants,
                        "patterns U{8..32} x U{0..3}; text order-2 Markov, Dirichlet(1,1,1,1) "
                        "rows, independent 16 Ki-symbol segments; 1 plant per MiB")


def _prefix_tree_paths(rng, depth, branching, p_printable):
    """All root-to-leaf paths of a random tree of the given depth where every node has
    ``branching`` distinct child bytes (each drawn printable with ``p_printable``)."""
    paths = [b""]
    for _ in range(depth):
        nxt = []
        for pre in paths:
            kids = set()
            while len(kids) < branching:
                kids.add(int(mixed_bytes(rng, 1, p_printable)[0]))
            for c in sorted(kids):
                nxt.append(pre + bytes([c]))
        paths = nxt
    return paths


def packets_256(seed: int = 4, n_packets: int = 65536, n_patterns: int = 20000,
                plant_every: int = 0) -> PacketWorkload:
    """Alphabet 256 packet batch. Sizes 64 / 576 / 1500 B with probabilities
    0.4 / 0.2 / 0.4, bytes 80 % printable. Patterns of length 4..128 whose first
    min(len, 6) bytes follow one of the 729 paths of a random tree with 3 children per
    node. ``plant_every = k > 0`` plants one whole fitting pattern into each packet with
    probability 1/k (the planted variant)."""
    rng = np.random.default_rng(seed)
    paths = _prefix_tree_paths(rng, 6, 3, 0.80)
    lens = rng.integers(4, 129, size=n_patterns)
    pats = []
    for L in lens:
        L = int(L)
        head = paths[int(rng.integers(0, len(paths)))][:min(L, 6)]
        tail = mixed_bytes(rng, L - len(head), 0.80).tobytes()
        pats.append(head + tail)
    sizes = rng.choice(np.array([64, 576, 1500]), size=n_packets, p=[0.4, 0.2, 0.4])
    offsets = np.zeros(n_packets + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    data = mixed_bytes(rng, int(offsets[-1]), 0.80)
    plants = []
    if plant_every:
        order = np.argsort([len(p) for p in pats], kind="stable")
        sorted_lens = np.array([len(pats[i]) for i in order])
        for i in range(n_packets):
            if rng.integers(0, plant_every) != 0:
                continue
            size = int(sizes[i])
            fit = int(np.searchsorted(sorted_lens, size, side="right"))
            if fit == 0:
                continue
            j = int(order[int(rng.integers(0, fit))])
            p = pats[j]
            off = int(rng.integers(0, size - len(p) + 1))
            base = int(offsets[i])
            data[base + off:base + off + len(p)] = np.frombuffer(p, dtype=np.uint8)
            plants.append((i, off, j))
    name = "packets_256" + ("_planted" if plant_every else "")
    return PacketWorkload(name, 256, pats, data, offsets, seed, plants,
                          "sizes {64:.4,576:.2,1500:.4}; 80% printable; patterns U{4..128} "
                          "headed by a depth-6 branching-3 random tree")


@dataclass
class Request:
    """One serving request: a batch of packets, with its arrival time (seconds from
    the start of the stream)."""
    arrival_s: float
    data: np.ndarray      # uint8, packets back to back
    offsets: np.ndarray   # uint64[n_packets + 1]


@dataclass
class ServingWorkload:
    name: str
    alphabet: int
    patterns: list
    seed: int
    offered_bytes_per_s: float
    packets_per_request: int
    pool: np.ndarray
    requests: list        # list[Request]
    recipe: str = ""

    @property
    def max_len(self) -> int:
        return max((len(p) for p in self.patterns), default=0)


SERVING_SIZES = np.array([64, 512, 1500, 9000])


def serving_256(seed: int = 5, n_patterns: int = 50000, offered_gbit_s: float = 40.0,
                duration_s: float = 2.0, packets_per_request: int = 32,
                pool_bytes: int = 1 << 30, plant_every: int = 0,
                max_requests: int | None = None, contiguous: bool = False) -> ServingWorkload:
    """Open-loop Poisson request stream at ``offered_gbit_s``. Each request is a batch
    of ``packets_per_request`` packets with sizes uniform over {64, 512, 1500, 9000};
    payloads are slices of a seeded uniform random pool (optionally with one planted
    whole pattern per packet with probability 1/``plant_every``).

    ``contiguous=True`` makes each request one slice of the pool, held as a view (no
    copy), with plants written into the pool itself: a 2 s stream at 40 Gbit/s is then
    10 GB of requests over a 1 GiB pool without 10 GB of copies. Later plants may land
    in earlier requests' slices; the bytes a request finally views are its payload."""
    rng = np.random.default_rng(seed)
    lens = lognormal_lengths(rng, n_patterns, 16.0, 0.5, 4, 256)
    pats = [rng.integers(0, 256, size=int(L), dtype=np.uint8).tobytes() for L in lens]
    pool = rng.integers(0, 256, size=pool_bytes, dtype=np.uint8)
    offered = offered_gbit_s * 1e9 / 8.0
    mean_req = packets_per_request * float(SERVING_SIZES.mean())
    lam = offered / mean_req
    n_req = int(np.ceil(lam * duration_s))
    if max_requests is not None:
        n_req = min(n_req, max_requests)
    gaps = rng.exponential(1.0 / lam, size=n_req)
    arrivals = np.cumsum(gaps)
    order = np.argsort(lens, kind="stable")
    sorted_lens = lens[order]
    reqs = []
    if contiguous:
        sizes = SERVING_SIZES[rng.integers(0, 4, size=(n_req, packets_per_request))]
        offs = np.zeros((n_req, packets_per_request + 1), dtype=np.uint64)
        np.cumsum(sizes, axis=1, out=offs[:, 1:])
        starts = rng.integers(0, pool_bytes - offs[:, -1].astype(np.int64) + 1)
        for r in range(n_req):
            a = int(starts[r])
            data = pool[a:a + int(offs[r, -1])]
            if plant_every:
                for i in np.nonzero(rng.integers(0, plant_every, size=packets_per_request) == 0)[0]:
                    s = int(sizes[r, i])
                    fit = int(np.searchsorted(sorted_lens, s, side="right"))
                    if fit:
                        p = pats[int(order[int(rng.integers(0, fit))])]
                        o = int(offs[r, i]) + int(rng.integers(0, s - len(p) + 1))
                        data[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
            reqs.append(Request(float(arrivals[r]), data, offs[r]))
        name = "serving_256" + ("_planted" if plant_every else "")
        return ServingWorkload(name, 256, pats, seed, offered, packets_per_request, pool, reqs,
                               "Poisson arrivals; 32 packets/request U{64,512,1500,9000}, each "
                               "request one pool slice; patterns lognormal(ln 16, 0.5) clip "
                               "4..256 x U{0..255}")
    for r in range(n_req):
        sizes = SERVING_SIZES[rng.integers(0, 4, size=packets_per_request)]
        offs = np.zeros(packets_per_request + 1, dtype=np.uint64)
        np.cumsum(sizes, out=offs[1:])
        data = np.empty(int(offs[-1]), dtype=np.uint8)
        for i, s in enumerate(sizes):
            a = int(rng.integers(0, pool_bytes - int(s) + 1))
            data[int(offs[i]):int(offs[i + 1])] = pool[a:a + int(s)]
            if plant_every and rng.integers(0, plant_every) == 0:
                fit = int(np.searchsorted(sorted_lens, int(s), side="right"))
                if fit:
                    j = int(order[int(rng.integers(0, fit))])
                    p = pats[j]
                    o = int(offs[i]) + int(rng.integers(0, int(s) - len(p) + 1))
                    data[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
        reqs.append(Request(float(arrivals[r]), data, offs))
    name = "serving_256" + ("_planted" if plant_every else "")
    return ServingWorkload(name, 256, pats, seed, offered, packets_per_request, pool, reqs,
                           "Poisson arrivals; 32 packets/request U{64,512,1500,9000}; "
                           "patterns lognormal(ln 16, 0.5) clip 4..256 x U{0..255}")
