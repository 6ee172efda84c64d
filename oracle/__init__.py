"""CPU oracle for the MaxSSmap hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.  The arithmetic lives in ``maxss_oracle.c`` (plain C,
nested loops, int32); this module only builds it with gcc and marshals
arguments through ctypes.  ``mlp.py`` holds the float64 oracle of the learned
proposal (4-mer profiles and the 512-256-1 MLP).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "maxss_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
ONE_STRAND = 1
FAST = 2
EXCL_ADJ = 4   # the second-best fragment is never a neighbour of the best
NW_FIT = 0
NW_GLOBAL = 1

# 32-byte scan record (same field order as the library's; compared field by field)
TOP2_DTYPE = np.dtype([("frag", "<i4", (2,)), ("score", "<i4", (2,)),
                       ("offset", "<i4", (2,)), ("strand", "i1", (2,)),
                       ("pad", "i1", (6,))])


class _Aln(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("strand", ctypes.c_int8),
                ("flags", ctypes.c_int8), ("pad_", ctypes.c_int8 * 2),
                ("ref_begin", ctypes.c_int64), ("ref_end", ctypes.c_int64),
                ("cigar_len", ctypes.c_uint32), ("pad2_", ctypes.c_uint32)]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L",
                               "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        c = ctypes
        L.oracle_num_fragments.restype = c.c_uint32
        L.oracle_num_fragments.argtypes = [c.c_uint64, c.c_uint32]
        L.oracle_maxss_seq.restype = c.c_int32
        L.oracle_maxss_seq.argtypes = [c.c_void_p, c.c_uint32]
        L.oracle_window_score.restype = c.c_int
        L.oracle_window_score.argtypes = [c.c_char_p, c.c_uint32, c.c_char_p, c.c_uint64,
                                          c.c_uint64, c.c_int32, c.c_int32, c.c_uint32,
                                          c.c_char_p, c.c_int32, c.POINTER(c.c_int32)]
        L.oracle_revcomp.restype = None
        L.oracle_revcomp.argtypes = [c.c_char_p, c.c_uint32, c.c_char_p]
        L.oracle_scan.restype = c.c_int
        L.oracle_scan.argtypes = [c.c_char_p, c.c_uint64, c.c_uint32, c.c_void_p, c.c_void_p,
                                  c.c_uint32, c.c_int32, c.c_int32, c.c_uint32, c.c_int,
                                  c.c_void_p, c.c_void_p, c.c_void_p, c.c_int32]
        L.oracle_nw.restype = c.c_int
        L.oracle_nw.argtypes = [c.c_char_p, c.c_uint32, c.c_char_p, c.c_uint32, c.c_int32,
                                c.c_int32, c.c_int32, c.c_int, c.c_char_p, c.c_int32,
                                c.POINTER(c.c_int32),
                                c.POINTER(c.c_int32), c.POINTER(c.c_int32), c.c_char_p,
                                c.c_uint32, c.POINTER(c.c_uint32)]
        L.oracle_cigar_rle.restype = c.c_int
        L.oracle_cigar_rle.argtypes = [c.c_char_p, c.c_char_p, c.c_uint32]
        L.oracle_align_one.restype = c.c_int
        L.oracle_align_one.argtypes = [c.c_char_p, c.c_uint64, c.c_uint32, c.c_char_p,
                                       c.c_uint32, c.c_int32, c.c_int32, c.c_uint32, c.c_int32,
                                       c.c_int32, c.c_int32, c.c_int, c.c_char_p, c.c_int32,
                                       c.POINTER(_Aln), c.c_char_p, c.c_uint32]
        _lib = L
    return _lib


def _b(s) -> bytes:
    if isinstance(s, str):
        return s.encode()
    if isinstance(s, np.ndarray):
        return s.tobytes()
    return bytes(s)


def num_fragments(G: int, F: int) -> int:
    return int(lib().oracle_num_fragments(G, F))


def maxss_seq(x) -> int:
    a = np.ascontiguousarray(x, dtype=np.int32)
    return int(lib().oracle_maxss_seq(a.ctypes.data, a.size))


def window_score(read, genome, p: int, M: int = 1, X: int = -1, step: int = 1, qual=None,
                 qscale: int = 0) -> int:
    """MaxSS of the window at p; step 2 scores every other read base (fast);
    `qual` (Phred+33, one per read base) scores with position-specific pairs
    in units of 1/qscale."""
    r, g = _b(read), _b(genome)
    qb = _b(qual) if qual is not None else None
    if qb is not None and len(qb) != len(r):
        raise ValueError("one quality per read base")
    out = ctypes.c_int32()
    st = lib().oracle_window_score(r, len(r), g, len(g), p, M, X, step, qb, qscale,
                                   ctypes.byref(out))
    if st != OK:
        raise ValueError("oracle_window_score failed: %d" % st)
    return out.value


def revcomp(read) -> bytes:
    r = _b(read)
    out = ctypes.create_string_buffer(len(r) + 1)
    lib().oracle_revcomp(r, len(r), out)
    return out.raw[:len(r)]


def scan(genome, F: int, seq, offsets, M: int = 1, X: int = -1, flags: int = 0,
         nthreads: int = 1, want_values: bool = False, quals=None, qscale: int = 0):
    """Top-2 record per read; optionally the n x NF matrix of fragment values.
    `quals` (Phred+33, laid out as `seq`) switches to position-specific
    scores in units of 1/qscale."""
    g = _b(genome)
    s = np.frombuffer(_b(seq), dtype=np.uint8)
    qa = np.frombuffer(_b(quals), dtype=np.uint8) if quals is not None else None
    if qa is not None and qa.size != s.size:
        raise ValueError("one quality per read base")
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    n = off.size - 1
    out = np.zeros(n, dtype=TOP2_DTYPE)
    NF = num_fragments(len(g), F)
    vals = np.zeros((n, NF), dtype=np.int32) if want_values else None
    st = lib().oracle_scan(g, len(g), F, s.ctypes.data, off.ctypes.data, n, M, X, flags,
                           nthreads, out.ctypes.data,
                           vals.ctypes.data if vals is not None else None,
                           qa.ctypes.data if qa is not None else None, qscale)
    if st != OK:
        raise ValueError("oracle_scan failed: %d" % st)
    return (out, vals) if want_values else out


def nw(read, ref, M: int = 1, X: int = -1, gap: int = -2, mode: int = NW_FIT, qual=None,
       qscale: int = 0):
    """(score, ref_begin_col, ref_end_col, expanded_ops)."""
    q, r = _b(read), _b(ref)
    qb = _b(qual) if qual is not None else None
    cap = len(q) + len(r) + 1
    ops = ctypes.create_string_buffer(cap)
    sc, jb, je, ol = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_uint32()
    st = lib().oracle_nw(q, len(q), r, len(r), M, X, gap, mode, qb, qscale, ctypes.byref(sc),
                         ctypes.byref(jb), ctypes.byref(je), ops, cap, ctypes.byref(ol))
    if st != OK:
        raise ValueError("oracle_nw failed: %d" % st)
    return sc.value, jb.value, je.value, ops.raw[:ol.value].decode()


def cigar_rle(ops: str) -> str:
    cap = 2 * len(ops) + 2
    out = ctypes.create_string_buffer(cap)
    st = lib().oracle_cigar_rle(ops.encode(), out, cap)
    if st != OK:
        raise ValueError("oracle_cigar_rle failed")
    return out.value.decode()


def align_one(genome, F: int, read, frag: int, strand: int, pad: int = 100, M: int = 1,
              X: int = -1, gap: int = -2, mode: int = NW_FIT, qual=None, qscale: int = 0):
    """dict(score, strand, ref_begin, ref_end, cigar) for the second phase."""
    g, q = _b(genome), _b(read)
    qb = _b(qual) if qual is not None else None
    rec = _Aln()
    cap = 2 * (len(q) + F + len(q) + 2 * pad) + 16
    cig = ctypes.create_string_buffer(cap)
    st = lib().oracle_align_one(g, len(g), F, q, len(q), frag, strand, pad, M, X, gap, mode,
                                qb, qscale, ctypes.byref(rec), cig, cap)
    if st != OK:
        raise ValueError("oracle_align_one failed: %d" % st)
    return dict(score=rec.score, strand=rec.strand, ref_begin=rec.ref_begin,
                ref_end=rec.ref_end, cigar=cig.value.decode())


def align_top(genome, F: int, seq, offsets, top2, pad: int = 100, M: int = 1, X: int = -1,
              gap: int = -2, mode: int = NW_FIT, idx=None, quals=None, qscale: int = 0):
    """align_one for each read i (or each i in idx) from its top-2 record."""
    sb = _b(seq)
    qb = _b(quals) if quals is not None else None
    off = np.asarray(offsets, dtype=np.uint64)
    ids = range(off.size - 1) if idx is None else idx
    res = []
    for i in ids:
        a, b = int(off[i]), int(off[i + 1])
        res.append(align_one(genome, F, sb[a:b], int(top2["frag"][i][0]),
                             int(top2["strand"][i][0]), pad, M, X, gap, mode,
                             qb[a:b] if qb is not None else None, qscale))
    return res
