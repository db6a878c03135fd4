"""Python binding of ``libpfac.so`` (argument marshalling only).

Each function has the name of the C entry point it calls (``include/pfac.h``). Device
buffers are torch tensors on a ROCm device; their ``data_ptr()`` and the current HIP
stream are passed straight to the library, and every step of the matching runs in the
library's HIP kernels. If the library is not built, or the device is not a gfx950,
these functions raise: there is no fallback.

Keys are returned in int64 tensors used as raw 64-bit storage: key = (start << 32) | id,
which numpy reads back as uint64 (``keys.cpu().numpy().view(np.uint64)``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfac.so")

PFAC_OK = 0
PFAC_EINVAL = -1
PFAC_EEMPTY_PATTERN = -2
PFAC_ESYMBOL = -3
PFAC_ETOO_LARGE = -4
PFAC_ENOMEM = -5
PFAC_EHIP = -6
PFAC_ECAPACITY = -7
PFAC_ENODEVICE = -8
PFAC_EFORMAT = -9
PFAC_ETIMEOUT = -10
PFAC_EINTERNAL = -11
PFAC_EBUSY = -12

_lib = None


class PfacError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s: %s (%d)" % (where, strerror(code) if _lib else "error", code))


class TableInfo(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in (
        "alphabet", "n_patterns", "n_nodes", "n_terminal_nodes", "min_len", "max_len",
        "depth", "node_layout")] + [
        ("paper_table_bytes", C.c_uint64), ("device_table_bytes", C.c_uint64)] + [
        (n, C.c_uint32) for n in ("root_depth", "filter_k", "filter_log2_bits",
                                  "lds_image_bytes", "merge_levels", "reduced_nodes",
                                  "table_records", "shared_base")] + [
        ("reduced_paper_bytes", C.c_uint64), ("node_array_bytes", C.c_uint64),
        ("stream_scratch", C.c_uint64), ("device_records", C.c_uint32), ("device_tails", C.c_uint32)]


class BuildOptions(C.Structure):
    _fields_ = [("merge_levels", C.c_uint32), ("reserved", C.c_uint32 * 7)]


class Match(C.Structure):
    _fields_ = [("start", C.c_uint64), ("pattern_id", C.c_uint32), ("reserved", C.c_uint32)]


class Matches(C.Structure):
    _fields_ = [("matches", C.POINTER(Match)), ("count", C.c_uint64)]


class ServerConfig(C.Structure):
    _fields_ = [("slots", C.c_uint32), ("max_batch_packets", C.c_uint32), ("max_batch_bytes", C.c_uint64),
                ("key_capacity", C.c_uint64), ("max_pending_bytes", C.c_uint64),
                ("device_memory_budget", C.c_uint64), ("flags", C.c_uint32), ("reserved", C.c_uint32 * 3)]


class Result(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("n_pkts", C.c_uint32),
                ("n_bytes", C.c_uint64), ("n_matches", C.c_uint64), ("keys", C.POINTER(C.c_uint64)),
                ("arrival_ns", C.c_uint64), ("launch_ns", C.c_uint64), ("done_ns", C.c_uint64)]


class ServerStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("requests", "packets", "bytes", "matches", "batches", "rejected",
                                          "pending_requests")] + [
        ("slots", C.c_uint32), ("reserved0", C.c_uint32), ("bytes_per_s", C.c_double),
        ("mean_batch_bytes", C.c_double), ("p50_ns", C.c_uint64), ("p99_ns", C.c_uint64),
        ("max_ns", C.c_uint64)]


MATCH_DTYPE = np.dtype([("start", np.uint64), ("pattern_id", np.uint32), ("reserved", np.uint32)])

PFAC_ALGO_AUTO, PFAC_ALGO_PLAIN, PFAC_ALGO_TILED = 0, 1, 2
PFAC_SERVER_EAGER = 1
ALGOS = {"auto": PFAC_ALGO_AUTO, "plain": PFAC_ALGO_PLAIN, "tiled": PFAC_ALGO_TILED}


class Tuning(C.Structure):
    _fields_ = [("algo", C.c_uint32), ("grid", C.c_uint32), ("span_log2", C.c_uint32),
                ("root_depth", C.c_uint32), ("filter_k", C.c_uint32), ("lane_bytes", C.c_uint32),
                ("reserved", C.c_uint32 * 2)]


TUNING_FIELDS = ("algo", "grid", "span_log2", "root_depth", "filter_k", "lane_bytes")


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpfac.so is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P8, P64, P32 = C.POINTER(C.c_uint8), C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)
        VP = C.c_void_p
        sig = {
            "pfac_strerror": (C.c_char_p, [C.c_int]),
            "pfac_version": (C.c_int, []),
            "pfac_build_csr": (C.c_int, [P8, P64, C.c_uint32, C.c_uint32, C.POINTER(VP)]),
            "pfac_build": (C.c_int, [C.POINTER(P8), P64, C.c_uint32, C.c_uint32, C.POINTER(VP)]),
            "pfac_build_ex": (C.c_int, [P8, P64, C.c_uint32, C.c_uint32, C.POINTER(BuildOptions),
                                        C.POINTER(VP)]),
            "pfac_export_records": (C.c_int, [VP, P32, P32, P8, P32, C.c_uint64]),
            "pfac_export_rank_ids": (C.c_int, [VP, P32, C.c_uint64, P32, C.c_uint64]),
            "pfac_destroy": (None, [VP]),
            "pfac_table_info": (C.c_int, [VP, C.POINTER(TableInfo)]),
            "pfac_export_paper_table": (C.c_int, [VP, P32, C.c_uint64, P32, C.c_uint64]),
            "pfac_export_outputs": (C.c_int, [VP, P32, C.c_uint64, P32, C.c_uint64]),
            "pfac_upload": (C.c_int, [VP, C.c_int]),
            "pfac_save": (C.c_int, [VP, P8, C.c_uint64, P64]),
            "pfac_load": (C.c_int, [P8, C.c_uint64, C.POINTER(VP)]),
            "pfac_key_to_packet": (C.c_int, [P64, C.c_uint64, P64, C.c_uint32, P32, P32, P32]),
            "pfac_scan_async": (C.c_int, [VP, VP, C.c_uint64, VP, C.c_uint64, VP, VP]),
            "pfac_scan_noalloc": (C.c_int, [VP, VP, C.c_uint64, VP, C.c_uint64, VP, VP]),
            "pfac_prefix_histogram": (C.c_int, [VP, VP, C.c_uint64, C.c_uint32, VP, VP]),
            "pfac_scan": (C.c_int, [VP, VP, C.c_uint64, VP, C.c_uint64, P64, VP]),
            "pfac_scan_batch_async": (C.c_int, [VP, VP, VP, C.c_uint32, C.c_uint64, VP, C.c_uint64,
                                                VP, VP]),
            "pfac_scan_batch": (C.c_int, [VP, VP, VP, C.c_uint32, C.c_uint64, VP, C.c_uint64,
                                          P64, VP]),
            "pfac_graph_create": (C.c_int, [VP, VP, VP, C.c_uint64, C.c_uint32, VP, C.c_uint64,
                                            VP, VP, VP, C.POINTER(VP)]),
            "pfac_graph_launch": (C.c_int, [VP, VP]),
            "pfac_graph_destroy": (None, [VP]),
            "pfac_scan_host": (C.c_int, [VP, VP, C.c_uint64, C.c_uint64, C.POINTER(Matches)]),
            "pfac_matches_free": (None, [C.POINTER(Matches)]),
            "pfac_server_create": (C.c_int, [VP, C.POINTER(ServerConfig), C.POINTER(VP)]),
            "pfac_server_config_get": (C.c_int, [VP, C.POINTER(ServerConfig)]),
            "pfac_server_submit": (C.c_int, [VP, VP, VP, C.c_uint32, C.c_uint64, P64]),
            "pfac_server_poll": (C.c_int, [VP, C.POINTER(Result), C.c_uint32, P32, C.c_uint32]),
            "pfac_result_free": (None, [C.POINTER(Result)]),
            "pfac_server_stats": (C.c_int, [VP, C.POINTER(ServerStats), C.c_int]),
            "pfac_server_destroy": (None, [VP]),
            "pfac_set_tuning": (C.c_int, [VP, C.POINTER(Tuning)]),
            "pfac_get_tuning": (C.c_int, [VP, C.POINTER(Tuning)]),
            "pfac_tune": (C.c_int, [VP, VP, C.c_uint64, VP, C.c_uint32, C.c_uint32, VP,
                                    C.POINTER(Tuning), C.POINTER(C.c_float)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().pfac_strerror(code).decode()


def pfac_version() -> int:
    return lib().pfac_version()


def _check(rc: int, where: str):
    if rc != PFAC_OK:
        raise PfacError(rc, where)


class Automaton:
    """Owns a ``pfac_automaton*``; freed with ``pfac_destroy`` on close / collection."""

    def __init__(self, handle: int, patterns_max_len: int):
        self.handle = handle
        self.max_len = patterns_max_len

    def close(self):
        if self.handle:
            lib().pfac_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def pfac_build(patterns, alphabet: int = 256, merge_levels: int = 0) -> Automaton:
    """Build the table of ``patterns`` (a list of bytes): the trie of Section 3.1, or with
    ``merge_levels`` > 0 its compressed form of Section 3.2 (``pfac_build_ex``)."""
    offs = np.zeros(len(patterns) + 1, dtype=np.uint64)
    if patterns:
        np.cumsum([len(p) for p in patterns], out=offs[1:])
    data = np.frombuffer(b"".join(bytes(p) for p in patterns) or b"\0", dtype=np.uint8).copy()
    h = C.c_void_p()
    P8, P64 = C.POINTER(C.c_uint8), C.POINTER(C.c_uint64)
    if merge_levels:
        opt = BuildOptions(merge_levels)
        rc = lib().pfac_build_ex(data.ctypes.data_as(P8), offs.ctypes.data_as(P64), len(patterns), alphabet,
                                 C.byref(opt), C.byref(h))
    else:
        rc = lib().pfac_build_csr(data.ctypes.data_as(P8), offs.ctypes.data_as(P64), len(patterns),
                                  alphabet, C.byref(h))
    _check(rc, "pfac_build")
    return Automaton(h.value, max((len(p) for p in patterns), default=0))


def pfac_export_records(a: Automaton) -> dict:
    """The walked table: first, bitmaps (records x ceil(alphabet/32) uint32), term, rank,
    plus shared_base and the ids by rank (rank_first, rank_ids)."""
    info = pfac_table_info(a)
    n, words = info["table_records"], (info["alphabet"] + 31) // 32
    first = np.zeros(n, np.uint32)
    bm = np.zeros((n, words), np.uint32)
    term = np.zeros(n, np.uint8)
    rank = np.zeros(n, np.uint32)
    P32 = C.POINTER(C.c_uint32)
    _check(lib().pfac_export_records(a.handle, first.ctypes.data_as(P32), bm.ctypes.data_as(P32),
                                     term.ctypes.data_as(C.POINTER(C.c_uint8)), rank.ctypes.data_as(P32), n),
           "pfac_export_records")
    rf = np.zeros(info["n_patterns"] + 1, np.uint32)
    ri = np.zeros(max(info["n_patterns"], 1), np.uint32)
    _check(lib().pfac_export_rank_ids(a.handle, rf.ctypes.data_as(P32), len(rf), ri.ctypes.data_as(P32), len(ri)),
           "pfac_export_rank_ids")
    return {"first": first, "bitmaps": bm, "term": term, "rank": rank, "shared_base": info["shared_base"],
            "rank_first": rf, "rank_ids": ri[:info["n_patterns"]]}


def pfac_table_info(a: Automaton) -> dict:
    info = TableInfo()
    _check(lib().pfac_table_info(a.handle, C.byref(info)), "pfac_table_info")
    return {name: getattr(info, name) for name, _ in TableInfo._fields_}


def pfac_export_paper_table(a: Automaton):
    """(offsets uint32[n_nodes], bitmaps uint32[n_nodes, ceil(alphabet/32)])."""
    info = pfac_table_info(a)
    n, words = info["n_nodes"], (info["alphabet"] + 31) // 32
    off = np.zeros(n, dtype=np.uint32)
    bm = np.zeros((n, words), dtype=np.uint32)
    P32 = C.POINTER(C.c_uint32)
    _check(lib().pfac_export_paper_table(a.handle, off.ctypes.data_as(P32), n,
                                         bm.ctypes.data_as(P32), bm.size),
           "pfac_export_paper_table")
    return off, bm


def pfac_export_outputs(a: Automaton):
    info = pfac_table_info(a)
    first = np.zeros(info["n_nodes"] + 1, dtype=np.uint32)
    ids = np.zeros(max(info["n_patterns"], 1), dtype=np.uint32)
    P32 = C.POINTER(C.c_uint32)
    _check(lib().pfac_export_outputs(a.handle, first.ctypes.data_as(P32), len(first),
                                     ids.ctypes.data_as(P32), len(ids)), "pfac_export_outputs")
    return first, ids[:info["n_patterns"]]


def pfac_set_tuning(a: Automaton, algo: str = "auto", grid: int = 0, span_log2: int = 0,
                    root_depth: int = 0, filter_k: int = 0, lane_bytes: int = 0):
    t = Tuning(ALGOS[algo], grid, span_log2, root_depth, filter_k, lane_bytes)
    _check(lib().pfac_set_tuning(a.handle, C.byref(t)), "pfac_set_tuning")


def _tuning_dict(t: Tuning) -> dict:
    d = {f: int(getattr(t, f)) for f in TUNING_FIELDS}
    d["algo"] = {v: k for k, v in ALGOS.items()}[t.algo]
    return d


def pfac_get_tuning(a: Automaton) -> dict:
    t = Tuning()
    _check(lib().pfac_get_tuning(a.handle, C.byref(t)), "pfac_get_tuning")
    return _tuning_dict(t)


def pfac_tune(a: Automaton, data, offsets=None, reps: int = 5, stream=None) -> dict:
    """Run the library's autotuner on a device-resident sample (a text, or a packet
    batch when ``offsets`` is given) and keep the best tuning. Returns it, with the mean
    milliseconds per scan under ``"ms"``."""
    data = _device_u8(data)
    if offsets is not None:
        offsets = _device_u64(offsets, "offsets")
    t = Tuning()
    ms = C.c_float(0)
    rc = lib().pfac_tune(a.handle, _ptr(data), data.numel(), _ptr(offsets),
                         offsets.numel() - 1 if offsets is not None else 0, reps,
                         _stream_handle(stream), C.byref(t), C.byref(ms))
    _check(rc, "pfac_tune")
    d = _tuning_dict(t)
    d["ms"] = float(ms.value)
    return d


def pfac_upload(a: Automaton, device: int = 0):
    _check(lib().pfac_upload(a.handle, device), "pfac_upload")


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _device_u8(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.uint8 and t.is_contiguous()):
        raise TypeError("text must be a contiguous uint8 tensor on a ROCm device")
    return t


def pfac_scan_async(a: Automaton, text, keys, count, stream=None):
    """Enqueue a scan of ``text`` (uint8 device tensor). ``keys``: int64 device tensor
    (capacity = its numel); ``count``: int64 device tensor with one element."""
    text = _device_u8(text)
    rc = lib().pfac_scan_async(a.handle, C.c_void_p(text.data_ptr()), text.numel(),
                               C.c_void_p(keys.data_ptr() if keys.numel() else 0), keys.numel(),
                               C.c_void_p(count.data_ptr()), _stream_handle(stream))
    _check(rc, "pfac_scan_async")


def pfac_scan_noalloc(a: Automaton, text, keys, count, stream=None):
    """Enqueue a scan that allocates nothing (the library's fixed per-device scratch;
    the automaton must already be on the device). Arguments as ``pfac_scan_async``."""
    text = _device_u8(text)
    rc = lib().pfac_scan_noalloc(a.handle, C.c_void_p(text.data_ptr()), text.numel(),
                                 C.c_void_p(keys.data_ptr() if keys.numel() else 0), keys.numel(),
                                 C.c_void_p(count.data_ptr()), _stream_handle(stream))
    _check(rc, "pfac_scan_noalloc")


def pfac_prefix_histogram(a: Automaton, text, cap: int, stream=None):
    """Prefix depths of ``text`` (uint8 device tensor): int64 device tensor of cap + 1
    bins, bin d = starts whose longest spelled pattern prefix has length d (the last bin:
    cap or more)."""
    import torch
    text = _device_u8(text)
    hist = torch.empty(cap + 1, dtype=torch.int64, device=text.device)
    rc = lib().pfac_prefix_histogram(a.handle, C.c_void_p(text.data_ptr() if text.numel() else 0), text.numel(),
                                     cap, C.c_void_p(hist.data_ptr()), _stream_handle(stream))
    _check(rc, "pfac_prefix_histogram")
    return hist


def pfac_scan(a: Automaton, text, keys=None, stream=None):
    """Blocking scan. Returns the keys of all matches as an int64 device tensor (raw
    uint64 keys, sorted). If ``keys`` is given it is used as the output buffer first;
    on PFAC_ECAPACITY a buffer of the needed size is allocated and the scan repeated."""
    import torch
    text = _device_u8(text)
    if keys is None:
        keys = torch.empty(max(1024, text.numel() // 256), dtype=torch.int64, device=text.device)
    cnt = C.c_uint64(0)
    for _ in range(2):
        rc = lib().pfac_scan(a.handle, C.c_void_p(text.data_ptr()), text.numel(),
                             C.c_void_p(keys.data_ptr()), keys.numel(), C.byref(cnt),
                             _stream_handle(stream))
        if rc == PFAC_ECAPACITY:
            keys = torch.empty(int(cnt.value), dtype=torch.int64, device=text.device)
            continue
        _check(rc, "pfac_scan")
        return keys[:int(cnt.value)]
    raise PfacError(PFAC_ECAPACITY, "pfac_scan")


def _device_u64(t, what):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int64 and t.is_contiguous()):
        raise TypeError("%s must be a contiguous int64 tensor on a ROCm device" % what)
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)


def pfac_scan_batch_async(a: Automaton, data, offsets, keys, count, stream=None):
    """Enqueue a scan of a packet batch: ``data`` uint8 device tensor holding the packets
    back to back, ``offsets`` int64 device tensor of n_pkts + 1 packet offsets."""
    data = _device_u8(data)
    offsets = _device_u64(offsets, "offsets")
    rc = lib().pfac_scan_batch_async(a.handle, _ptr(data), _ptr(offsets), max(offsets.numel() - 1, 0),
                                     data.numel(), _ptr(keys), keys.numel(), _ptr(count),
                                     _stream_handle(stream))
    _check(rc, "pfac_scan_batch_async")


def pfac_scan_batch(a: Automaton, data, offsets, keys=None, stream=None):
    """Blocking packet-batch scan; returns the sorted keys (global byte offset << 32 | id)
    as an int64 device tensor, growing ``keys`` on PFAC_ECAPACITY as pfac_scan does."""
    import torch
    data = _device_u8(data)
    offsets = _device_u64(offsets, "offsets")
    if keys is None:
        keys = torch.empty(max(1024, data.numel() // 256), dtype=torch.int64, device=data.device)
    cnt = C.c_uint64(0)
    for _ in range(2):
        rc = lib().pfac_scan_batch(a.handle, _ptr(data), _ptr(offsets), max(offsets.numel() - 1, 0),
                                   data.numel(), _ptr(keys), keys.numel(), C.byref(cnt),
                                   _stream_handle(stream))
        if rc == PFAC_ECAPACITY:
            keys = torch.empty(int(cnt.value), dtype=torch.int64, device=data.device)
            continue
        _check(rc, "pfac_scan_batch")
        return keys[:int(cnt.value)]
    raise PfacError(PFAC_ECAPACITY, "pfac_scan_batch")


class Graph:
    """Owns a ``pfac_graph*`` (a captured scan, replayed with :meth:`launch`). Keeps the
    tensors it was recorded on alive."""

    def __init__(self, handle, tensors):
        self.handle = handle
        self._tensors = tensors

    def launch(self, stream=None):
        _check(lib().pfac_graph_launch(self.handle, _stream_handle(stream)), "pfac_graph_launch")

    def close(self):
        if self.handle:
            lib().pfac_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pfac_graph_create(a: Automaton, data, offsets, keys, count, sizes, stream) -> Graph:
    """Record a scan of ``data`` (uint8 device tensor; its numel is the byte bound) as a
    packet batch over ``offsets`` (int64 device tensor, max packets + 1; None for one
    text) into a HIP graph. ``sizes``: int64 device tensor {bytes, packets} read at each
    replay. ``stream`` must be a non-default torch stream."""
    data = _device_u8(data)
    if offsets is not None:
        offsets = _device_u64(offsets, "offsets")
    sizes = _device_u64(sizes, "sizes")
    h = C.c_void_p()
    n_pk = offsets.numel() - 1 if offsets is not None else 0
    rc = lib().pfac_graph_create(a.handle, _ptr(data), _ptr(offsets), data.numel(), n_pk, _ptr(keys),
                                 keys.numel(), _ptr(count), _ptr(sizes), _stream_handle(stream), C.byref(h))
    _check(rc, "pfac_graph_create")
    return Graph(h.value, (data, offsets, keys, count, sizes, a))


def pfac_key_to_packet(keys, offsets):
    """(packet index, start within packet, pattern id) of uint64 batch keys (host numpy)
    for packets given by ``offsets`` (uint64, n_pkts + 1), as three uint32 arrays."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = len(keys)
    pk, st, ids = (np.zeros(max(n, 1), dtype=np.uint32) for _ in range(3))
    P32, P64 = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
    rc = lib().pfac_key_to_packet(keys.ctypes.data_as(P64), n, offs.ctypes.data_as(P64), len(offs) - 1,
                                  pk.ctypes.data_as(P32), st.ctypes.data_as(P32), ids.ctypes.data_as(P32))
    _check(rc, "pfac_key_to_packet")
    return pk[:n], st[:n], ids[:n]


def pfac_save(a: Automaton) -> bytes:
    """The automaton serialized by the library (see ``pfac_save`` in pfac.h)."""
    size = C.c_uint64(0)
    rc = lib().pfac_save(a.handle, None, 0, C.byref(size))
    if rc not in (PFAC_OK, PFAC_ECAPACITY):
        _check(rc, "pfac_save")
    buf = np.zeros(int(size.value), dtype=np.uint8)
    _check(lib().pfac_save(a.handle, buf.ctypes.data_as(C.POINTER(C.c_uint8)), len(buf), C.byref(size)),
           "pfac_save")
    return buf.tobytes()


def pfac_load(blob) -> Automaton:
    """An automaton rebuilt by the library from bytes written by ``pfac_save``."""
    buf = np.frombuffer(bytes(blob), dtype=np.uint8)
    h = C.c_void_p()
    arr = buf if len(buf) else np.zeros(1, dtype=np.uint8)
    _check(lib().pfac_load(arr.ctypes.data_as(C.POINTER(C.c_uint8)), len(buf), C.byref(h)), "pfac_load")
    a = Automaton(h.value, 0)
    a.max_len = pfac_table_info(a)["max_len"]
    return a


def pfac_scan_host(a: Automaton, text, chunk_bytes: int = 0) -> np.ndarray:
    """Scan a host buffer (numpy uint8 array, or any object exposing a uint8 buffer, e.g.
    a pinned torch CPU tensor's numpy view). Returns a structured array with fields
    ``start`` (uint64) and ``pattern_id`` (uint32), sorted."""
    arr = np.ascontiguousarray(np.asarray(text, dtype=np.uint8))
    m = Matches()
    rc = lib().pfac_scan_host(a.handle, C.c_void_p(arr.ctypes.data if arr.size else 0), arr.size,
                              chunk_bytes, C.byref(m))
    _check(rc, "pfac_scan_host")
    try:
        if m.count == 0:
            return np.zeros(0, dtype=MATCH_DTYPE)
        buf = C.cast(m.matches, C.POINTER(C.c_uint8 * (int(m.count) * MATCH_DTYPE.itemsize))).contents
        return np.frombuffer(buf, dtype=MATCH_DTYPE).copy()
    finally:
        lib().pfac_matches_free(C.byref(m))


class Server:
    """Owns a ``pfac_server*`` (the serving loop; see ``pfac_server_create``)."""

    def __init__(self, handle, automaton):
        self.handle = handle
        self._a = automaton  # the automaton must outlive the server
        self._buf = (Result * 1024)()

    def config(self) -> dict:
        c = ServerConfig()
        _check(lib().pfac_server_config_get(self.handle, C.byref(c)), "pfac_server_config_get")
        return {n: getattr(c, n) for n, _ in ServerConfig._fields_ if n != "reserved"}

    def submit(self, data: np.ndarray, offsets: np.ndarray, arrival_ns: int = 0) -> int:
        """Submit one request (host numpy arrays: uint8 bytes, uint64 packet offsets)."""
        data = np.ascontiguousarray(data, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        t = C.c_uint64(0)
        rc = lib().pfac_server_submit(self.handle, C.c_void_p(data.ctypes.data if data.size else 0),
                                      C.c_void_p(offsets.ctypes.data), len(offsets) - 1, arrival_ns,
                                      C.byref(t))
        _check(rc, "pfac_server_submit")
        return t.value

    def submit_raw(self, data_ptr: int, offsets_ptr: int, n_pkts: int, arrival_ns: int = 0) -> int:
        """Submit from raw host pointers (no conversion; returns the status, ticket in .last)."""
        t = C.c_uint64(0)
        rc = lib().pfac_server_submit(self.handle, C.c_void_p(data_ptr), C.c_void_p(offsets_ptr), n_pkts,
                                      arrival_ns, C.byref(t))
        self.last = t.value
        return rc

    def poll(self, timeout_us: int = 0, with_keys: bool = True, keys_for=None) -> list:
        """Finished requests: dicts with ticket, status, n_pkts, n_bytes, n_matches, keys
        (uint64 numpy array), arrival_ns, launch_ns, done_ns. ``keys_for``: a predicate on
        the ticket; keys are copied out only for the tickets it accepts (else None)."""
        n = C.c_uint32(0)
        _check(lib().pfac_server_poll(self.handle, self._buf, len(self._buf), C.byref(n), timeout_us),
               "pfac_server_poll")
        out = []
        for i in range(n.value):
            r = self._buf[i]
            keys = None
            if with_keys and (keys_for is None or keys_for(r.ticket)):
                keys = (np.ctypeslib.as_array(r.keys, shape=(int(r.n_matches),)).copy()
                        if r.n_matches else np.zeros(0, dtype=np.uint64))
            out.append({"ticket": r.ticket, "status": r.status, "n_pkts": r.n_pkts, "n_bytes": r.n_bytes,
                        "n_matches": r.n_matches, "keys": keys, "arrival_ns": r.arrival_ns,
                        "launch_ns": r.launch_ns, "done_ns": r.done_ns})
            lib().pfac_result_free(C.byref(r))
        return out

    def stats(self, reset: bool = False) -> dict:
        st = ServerStats()
        _check(lib().pfac_server_stats(self.handle, C.byref(st), int(reset)), "pfac_server_stats")
        return {n: getattr(st, n) for n, _ in ServerStats._fields_ if n != "reserved0"}

    def close(self):
        if self.handle:
            lib().pfac_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pfac_server_create(a: Automaton, **cfg) -> Server:
    c = ServerConfig()
    for k, v in cfg.items():
        setattr(c, k, v)
    h = C.c_void_p()
    _check(lib().pfac_server_create(a.handle, C.byref(c), C.byref(h)), "pfac_server_create")
    return Server(h.value, a)


def keys_to_numpy(keys) -> np.ndarray:
    """Device int64 key tensor -> host uint64 array."""
    return keys.cpu().numpy().view(np.uint64)
