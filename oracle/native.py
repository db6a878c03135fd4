"""ctypes wrapper over ``oracle.c`` (test infrastructure only).

``build()`` compiles ``oracle.c`` with gcc (OpenMP) into ``_liboracle.so`` next to it.
``brute`` is the length-bucketed brute force, ``AhoCorasick`` the textbook automaton with
failure and dictionary links scanned in overlapped chunks (Section 2.2). Both return the
sorted 64-bit keys (start << 32) | pattern_id as a numpy uint64 array.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle library. Always recompiles when ``force``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def build_mutant(define: str, outdir: str) -> str:
    """Compile ``oracle.c`` with one of its planted-mistake macros (``ORC_MUTANT_*``)
    into ``outdir``. Used only by tests that show the pins catch such a mistake."""
    out = os.path.join(outdir, "_liboracle_%s.so" % define.lower())
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-D" + define, _SRC, "-o", out])
    return load(out)


def load(path: str):
    """Load and bind an oracle library at ``path``."""
    lib = C.CDLL(path)
    _bind(lib)
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = load(_LIB)
    return _lib


def _bind(lib):
    P8, P64 = C.POINTER(C.c_uint8), C.POINTER(C.c_uint64)
    lib.orc_brute.argtypes = [P8, P64, C.c_uint32, P8, C.c_uint64, C.c_int,
                              C.POINTER(P64), P64]
    lib.orc_brute.restype = C.c_int
    lib.orc_ac_build.argtypes = [P8, P64, C.c_uint32]
    lib.orc_ac_build.restype = C.c_void_p
    lib.orc_ac_free.argtypes = [C.c_void_p]
    lib.orc_ac_nodes.argtypes = [C.c_void_p]
    lib.orc_ac_nodes.restype = C.c_uint32
    lib.orc_ac_scan.argtypes = [C.c_void_p, P8, C.c_uint64, C.c_uint32, C.c_uint64, C.c_int,
                                C.POINTER(P64), P64]
    lib.orc_ac_scan.restype = C.c_int
    lib.orc_free.argtypes = [C.c_void_p]
    lib.orc_threads.restype = C.c_int


def threads() -> int:
    return _load().orc_threads()


def _csr(patterns):
    offs = np.zeros(len(patterns) + 1, dtype=np.uint64)
    if patterns:
        np.cumsum([len(p) for p in patterns], out=offs[1:])
    data = np.frombuffer(b"".join(patterns) or b"\0", dtype=np.uint8).copy()
    return data, offs


def _ptr8(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _ptr64(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def _take(lib, outp, cnt):
    n = int(cnt.value)
    res = np.ctypeslib.as_array(outp, shape=(max(n, 1),))[:n].copy()
    lib.orc_free(C.cast(outp, C.c_void_p))
    return res


def _text(text):
    t = np.ascontiguousarray(np.frombuffer(bytes(text), dtype=np.uint8)
                             if isinstance(text, (bytes, bytearray)) else text, dtype=np.uint8)
    return t if len(t) else np.zeros(1, dtype=np.uint8), len(t)


def brute(patterns, text, threads: int = 0, lib=None) -> np.ndarray:
    """Sorted keys of every (start, id) with T[start:start+|p|] == p."""
    lib = lib or _load()
    pd, po = _csr(patterns)
    t, n = _text(text)
    outp, cnt = C.POINTER(C.c_uint64)(), C.c_uint64(0)
    rc = lib.orc_brute(_ptr8(pd), _ptr64(po), len(patterns), _ptr8(t), n, threads,
                       C.byref(outp), C.byref(cnt))
    if rc != 0:
        raise MemoryError("oracle brute force failed")
    return _take(lib, outp, cnt)


class AhoCorasick:
    """Textbook automaton over ``patterns`` (goto + failure + dictionary links)."""

    def __init__(self, patterns, alphabet: int = 256, lib=None):
        self._lib = lib or _load()
        self.alphabet = alphabet
        self.max_len = max((len(p) for p in patterns), default=0)
        pd, po = _csr(patterns)
        self._h = self._lib.orc_ac_build(_ptr8(pd), _ptr64(po), len(patterns))
        if not self._h:
            raise MemoryError("oracle automaton build failed")

    @property
    def n_nodes(self) -> int:
        return int(self._lib.orc_ac_nodes(self._h))

    def scan(self, text, chunk: int = 1 << 22, threads: int = 0) -> np.ndarray:
        t, n = _text(text)
        outp, cnt = C.POINTER(C.c_uint64)(), C.c_uint64(0)
        rc = self._lib.orc_ac_scan(self._h, _ptr8(t), n, self.alphabet, chunk, threads,
                                   C.byref(outp), C.byref(cnt))
        if rc != 0:
            raise MemoryError("oracle scan failed")
        return _take(self._lib, outp, cnt)

    def scan_packets(self, data, offsets, threads: int = 0) -> np.ndarray:
        """Per-packet scan; starts are global offsets into ``data``."""
        parts = []
        data = np.asarray(data, dtype=np.uint8)
        for i in range(len(offsets) - 1):
            a, b = int(offsets[i]), int(offsets[i + 1])
            k = self.scan(data[a:b], threads=1)
            if len(k):
                parts.append(k + np.uint64(a << 32))
        return np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint64)

    def close(self):
        if self._h:
            self._lib.orc_ac_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
