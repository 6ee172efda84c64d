"""Python binding of libmaxss (MaxSSmap hot path on MI355X / gfx950).

Argument marshalling only: every step of the path runs in the HIP library
(``csrc/``, C ABI in ``include/maxss.h``).  PyTorch is used for device memory
and streams.  The functions keep the C names; ``Index`` is a small owner of
the opaque index handle.  Importing this module does not need a GPU, but every
call that computes fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmaxss.so")

MAXSS_OK = 0
MAXSS_EINVAL = -1
MAXSS_ENOMEM = -2
MAXSS_EDEVICE = -3
MAXSS_ETOOLONG = -4
MAXSS_ESTATE = -5
MAXSS_ONE_STRAND = 1
MAXSS_NW_GLOBAL = 2
MAXSS_FAST = 4
MAXSS_EXCLUDE_ADJACENT = 8
# scan kernel variants (maxss_scan_kernel_info), by VALU instructions per packed
# cell pair and step of their inner loop
MAXSS_KERNEL_STEP_MAX, MAXSS_KERNEL_TWO_STEP, MAXSS_KERNEL_REGISTER_BANK = 0, 1, 2
KERNEL_OPS_PER_CELL = {0: 3.0, 1: 2.5, 2: 1.75}
MAXSS_READ_INVALID = -2
MAXSS_ALN_TRUNCATED = 1
MAXSS_ALN_SKIPPED = 2

TOP2_DTYPE = np.dtype([("frag", "<i4", (2,)), ("score", "<i4", (2,)),
                       ("offset", "<i4", (2,)), ("strand", "i1", (2,)),
                       ("pad", "i1", (6,))])
ALN_DTYPE = np.dtype([("score", "<i4"), ("strand", "i1"), ("flags", "i1"), ("pad", "i1", (2,)),
                      ("ref_begin", "<i8"), ("ref_end", "<i8"), ("cigar_len", "<u4"),
                      ("pad2", "<u4")])
assert TOP2_DTYPE.itemsize == 32 and ALN_DTYPE.itemsize == 32


class MaxssError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("maxss status %d: %s" % (status, msg))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32), ("gap", ctypes.c_int32),
                ("frag_len", ctypes.c_uint32), ("max_read_len", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("qual_scale", ctypes.c_uint32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("np", ctypes.c_int32), ("reads_per_tile", ctypes.c_uint32),
                ("rounds", ctypes.c_uint32), ("best_ms", ctypes.c_float),
                ("default_ms", ctypes.c_float), ("tried", ctypes.c_uint32),
                ("rejected", ctypes.c_uint32), ("from_cache", ctypes.c_uint32)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint32), ("hard_negatives", ctypes.c_uint32),
                ("eval_every", ctypes.c_uint32), ("K", ctypes.c_uint32),
                ("val_fraction", ctypes.c_float), ("target_agreement", ctypes.c_float),
                ("loss_trace", ctypes.c_void_p), ("cand_trace", ctypes.c_void_p)]


class TrainStats(ctypes.Structure):
    _fields_ = [("n_train", ctypes.c_uint32), ("n_val", ctypes.c_uint32),
                ("steps_run", ctypes.c_uint32), ("best_step", ctypes.c_uint32),
                ("loss_first", ctypes.c_float), ("loss_last", ctypes.c_float),
                ("val_recall_init", ctypes.c_float), ("val_recall_best", ctypes.c_float),
                ("tau", ctypes.c_float), ("min_score", ctypes.c_int32),
                ("val_accept", ctypes.c_float), ("val_agreement", ctypes.c_float)]


class Reads(ctypes.Structure):
    _fields_ = [("seq", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("n", ctypes.c_uint32),
                ("on_device", ctypes.c_uint32), ("qual", ctypes.c_void_p)]


# every function declared in include/maxss.h
EXPORTS = ("maxss_index_genome", "maxss_index_free", "maxss_index_info", "maxss_scan_reads",
           "maxss_scan_reads_noalloc",
           "maxss_align_top", "maxss_plan_create", "maxss_plan_free", "maxss_plan_run",
           "maxss_plan_run_graph", "maxss_autotune", "maxss_index_set_tiles",
           "maxss_scan_kernel_info",
           "maxss_model_create", "maxss_model_from_params", "maxss_model_free",
           "maxss_model_get_params", "maxss_model_save",
           "maxss_model_load", "maxss_profiles", "maxss_proposal_scores",
           "maxss_proposal_candidates", "maxss_scan_reads_proposed", "maxss_model_train_step",
           "maxss_model_train", "maxss_choose_acceptance",
           "maxss_mapq", "maxss_sam_header", "maxss_sam_records",
           "maxss_profile_enable", "maxss_profile_read", "maxss_roof_int16",
           "maxss_fail_alloc_after", "maxss_last_error",
           "maxss_version")
MLP_PARAMS = 131585
MAXSS_INIT_GLOROT, MAXSS_INIT_PROFILE_MATCH = 0, 1

_lib = None


def lib():
    """The loaded library; raises if it was not built (no fallback path)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same soname as the system
        # one; loading torch first makes libmaxss bind to that copy, so that
        # torch's device memory and streams and this library share a runtime.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmaxss.so is not built (run __graft_entry__.build() or "
                               "python paper_1403_2136_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        c = ctypes
        L.maxss_index_genome.restype = c.c_int
        L.maxss_index_genome.argtypes = [c.c_void_p, c.c_uint64, c.POINTER(Params),
                                         c.POINTER(c.c_void_p)]
        L.maxss_index_free.restype = None
        L.maxss_index_free.argtypes = [c.c_void_p]
        L.maxss_index_info.restype = c.c_int
        L.maxss_index_info.argtypes = [c.c_void_p, c.POINTER(c.c_uint64), c.POINTER(c.c_uint32),
                                       c.POINTER(c.c_uint32)]
        L.maxss_scan_reads.restype = c.c_int
        L.maxss_scan_reads.argtypes = [c.c_void_p, c.POINTER(Reads), c.c_void_p, c.c_void_p]
        L.maxss_scan_reads_noalloc.restype = c.c_int
        L.maxss_scan_reads_noalloc.argtypes = [c.c_void_p, c.POINTER(Reads), c.c_void_p,
                                               c.c_void_p]
        L.maxss_align_top.restype = c.c_int
        L.maxss_align_top.argtypes = [c.c_void_p, c.POINTER(Reads), c.c_void_p, c.c_uint32,
                                      c.c_void_p, c.c_void_p, c.c_uint64, c.c_void_p]
        L.maxss_plan_create.restype = c.c_int
        L.maxss_plan_create.argtypes = [c.c_void_p, c.c_uint32, c.c_uint32, c.c_uint64,
                                        c.POINTER(c.c_void_p)]
        L.maxss_plan_free.restype = None
        L.maxss_plan_free.argtypes = [c.c_void_p]
        for fn in (L.maxss_plan_run, L.maxss_plan_run_graph):
            fn.restype = c.c_int
            fn.argtypes = [c.c_void_p, c.POINTER(Reads), c.c_void_p, c.c_void_p, c.c_void_p,
                           c.c_void_p]
        L.maxss_autotune.restype = c.c_int
        L.maxss_autotune.argtypes = [c.c_void_p, c.POINTER(Reads), c.c_char_p,
                                     c.POINTER(TuneResult)]
        L.maxss_index_set_tiles.restype = c.c_int
        L.maxss_index_set_tiles.argtypes = [c.c_void_p, c.c_int32, c.c_uint32, c.c_uint32]
        L.maxss_scan_kernel_info.restype = c.c_int
        L.maxss_scan_kernel_info.argtypes = [c.c_void_p, c.c_void_p, c.c_void_p]
        L.maxss_model_create.restype = c.c_int
        L.maxss_model_create.argtypes = [c.c_uint32, c.c_uint32, c.POINTER(c.c_void_p)]
        L.maxss_model_from_params.restype = c.c_int
        L.maxss_model_from_params.argtypes = [c.c_void_p, c.POINTER(c.c_void_p)]
        L.maxss_model_train.restype = c.c_int
        L.maxss_model_train.argtypes = [c.c_void_p, c.c_void_p, c.POINTER(Reads), c.c_void_p,
                                        c.POINTER(TrainOpts), c.POINTER(TrainStats), c.c_void_p]
        L.maxss_choose_acceptance.restype = c.c_int
        L.maxss_choose_acceptance.argtypes = [c.c_uint32, c.c_void_p, c.c_void_p, c.c_void_p,
                                              c.c_float, c.POINTER(c.c_float),
                                              c.POINTER(c.c_int32), c.POINTER(c.c_float),
                                              c.POINTER(c.c_float)]
        L.maxss_model_free.restype = None
        L.maxss_model_free.argtypes = [c.c_void_p]
        L.maxss_model_get_params.restype = c.c_int
        L.maxss_model_get_params.argtypes = [c.c_void_p, c.c_void_p]
        L.maxss_model_save.restype = c.c_int
        L.maxss_model_save.argtypes = [c.c_void_p, c.c_char_p]
        L.maxss_model_load.restype = c.c_int
        L.maxss_model_load.argtypes = [c.c_char_p, c.POINTER(c.c_void_p)]
        L.maxss_profiles.restype = c.c_int
        L.maxss_profiles.argtypes = [c.c_void_p, c.POINTER(Reads), c.c_void_p, c.c_void_p,
                                     c.c_void_p]
        L.maxss_proposal_scores.restype = c.c_int
        L.maxss_proposal_scores.argtypes = [c.c_void_p, c.c_void_p, c.POINTER(Reads), c.c_void_p,
                                            c.c_void_p]
        L.maxss_proposal_candidates.restype = c.c_int
        L.maxss_proposal_candidates.argtypes = [c.c_void_p, c.c_void_p, c.POINTER(Reads),
                                                c.c_uint32, c.c_float, c.c_void_p, c.c_void_p,
                                                c.c_void_p, c.c_void_p]
        L.maxss_scan_reads_proposed.restype = c.c_int
        L.maxss_scan_reads_proposed.argtypes = [c.c_void_p, c.c_void_p, c.POINTER(Reads),
                                                c.c_uint32, c.c_float, c.c_int32, c.c_void_p,
                                                c.c_void_p, c.c_void_p]
        L.maxss_model_train_step.restype = c.c_int
        L.maxss_model_train_step.argtypes = [c.c_void_p, c.c_void_p, c.POINTER(Reads), c.c_void_p,
                                             c.c_void_p, c.c_float, c.c_void_p, c.c_void_p,
                                             c.c_void_p]
        L.maxss_profile_enable.restype = c.c_int
        L.maxss_profile_enable.argtypes = [c.c_int]
        L.maxss_profile_read.restype = c.c_int
        L.maxss_profile_read.argtypes = [c.c_char_p, c.POINTER(c.c_double), c.POINTER(c.c_uint32)]
        L.maxss_fail_alloc_after.restype = c.c_int
        L.maxss_fail_alloc_after.argtypes = [c.c_uint32]
        L.maxss_roof_int16.restype = c.c_int
        L.maxss_roof_int16.argtypes = [c.POINTER(c.c_double), c.c_void_p]
        L.maxss_last_error.restype = c.c_char_p
        L.maxss_last_error.argtypes = []
        L.maxss_version.restype = c.c_char_p
        L.maxss_version.argtypes = []
        L.maxss_mapq.restype = c.c_int
        L.maxss_mapq.argtypes = [c.c_void_p, c.c_uint32, c.c_uint32, c.c_uint32, c.c_int32,
                                 c.c_void_p, c.c_void_p, c.c_void_p]
        L.maxss_sam_header.restype = c.c_int
        L.maxss_sam_header.argtypes = [c.c_void_p, c.c_char_p, c.c_void_p, c.c_uint64,
                                       c.POINTER(c.c_uint64)]
        L.maxss_sam_records.restype = c.c_int
        L.maxss_sam_records.argtypes = [c.POINTER(Reads), c.c_void_p, c.c_void_p, c.c_void_p,
                                        c.c_uint64, c.c_void_p, c.c_void_p, c.c_char_p,
                                        c.c_void_p, c.c_void_p, c.c_uint64,
                                        c.POINTER(c.c_uint64)]
        _lib = L
    return _lib


def _check(st: int):
    if st != MAXSS_OK:
        raise MaxssError(st, lib().maxss_last_error().decode(errors="replace"))


def _ptr(x):
    """Data pointer of a numpy array, torch tensor, bytes or int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    raise TypeError(type(x))


def _buf(x, nbytes: int, what: str, optional: bool = False):
    """Pointer of a buffer the library reads or writes nbytes of, after
    checking that the buffer (numpy array or torch tensor) is contiguous and
    large enough.  A raw int address is passed through unchecked."""
    if x is None:
        if optional:
            return None
        raise ValueError("%s is required" % what)
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        have, contig = x.nbytes, x.flags.c_contiguous
    elif hasattr(x, "data_ptr"):
        have, contig = x.numel() * x.element_size(), x.is_contiguous()
    else:
        raise TypeError(type(x))
    if not contig:
        raise ValueError("%s must be contiguous" % what)
    if have < nbytes:
        raise ValueError("%s holds %d bytes, %d needed" % (what, have, nbytes))
    return _ptr(x)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _as_u8(seq) -> np.ndarray:
    if isinstance(seq, (bytes, bytearray)):
        return np.frombuffer(bytes(seq), dtype=np.uint8)
    if isinstance(seq, str):
        return np.frombuffer(seq.encode(), dtype=np.uint8)
    return np.ascontiguousarray(seq, dtype=np.uint8)


def maxss_version() -> str:
    return lib().maxss_version().decode()


def maxss_profile_enable(on: bool) -> None:
    _check(lib().maxss_profile_enable(1 if on else 0))


def maxss_profile_read(name: str):
    """(total_ms, launches) of kernel `name` since profiling was enabled."""
    t, k = ctypes.c_double(), ctypes.c_uint32()
    _check(lib().maxss_profile_read(name.encode(), ctypes.byref(t), ctypes.byref(k)))
    return t.value, k.value


def maxss_fail_alloc_after(n: int) -> None:
    """Test hook: the n-th device allocation from now fails (0: off)."""
    _check(lib().maxss_fail_alloc_after(n))


def maxss_roof_int16(stream=None) -> float:
    """Measured packed 16-bit add issue rate of the current device (lane
    operations per second)."""
    v = ctypes.c_double()
    _check(lib().maxss_roof_int16(ctypes.byref(v), _stream_handle(stream)))
    return v.value


def maxss_index_genome(seq, frag_len: int, max_read_len: int, match: int = 1,
                       mismatch: int = -1, gap: int = -2, flags: int = 0,
                       qual_scale: int = 0) -> int:
    g = _as_u8(seq)
    p = Params(match, mismatch, gap, frag_len, max_read_len, flags, qual_scale)
    h = ctypes.c_void_p()
    _check(lib().maxss_index_genome(g.ctypes.data, g.size, ctypes.byref(p), ctypes.byref(h)))
    return h.value


def maxss_index_free(handle: int) -> None:
    lib().maxss_index_free(handle)


def maxss_index_info(handle: int):
    G, NF, F = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().maxss_index_info(handle, ctypes.byref(G), ctypes.byref(NF), ctypes.byref(F)))
    return G.value, NF.value, F.value


def _host_csr(seq, offsets):
    """Host reads as (uint8 array, uint64 offsets), with the offsets checked
    against the buffer so that the library never reads past it."""
    s = _as_u8(seq)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    if off.ndim != 1 or off.size < 1:
        raise ValueError("offsets must have n+1 >= 1 entries")
    if off.size > 1 and (int(off[-1]) > s.size or (np.diff(off.astype(np.int64)) < 0).any()):
        raise ValueError("offsets must be non-decreasing and end within the sequence buffer")
    return s, off


def _reads_struct(seq, offsets, on_device: bool, qual=None) -> Reads:
    n = (offsets.numel() if hasattr(offsets, "numel") else len(offsets)) - 1
    if qual is not None and hasattr(qual, "numel") and hasattr(seq, "numel"):
        if qual.numel() < seq.numel():
            raise ValueError("one quality per read base (%d qualities, %d bases)"
                             % (qual.numel(), seq.numel()))
    return Reads(_ptr(seq), _ptr(offsets), n, 1 if on_device else 0, _ptr(qual))


def _host_qual(qual, s: np.ndarray):
    """Host qualities as a uint8 array of the reads' size, or None."""
    if qual is None:
        return None
    q = _as_u8(qual)
    if q.size != s.size:
        raise ValueError("one quality per read base (%d qualities, %d bases)" % (q.size, s.size))
    return q


def maxss_scan_reads(handle: int, seq, offsets, out=None, stream=None, qual=None):
    """Top-2 records for a batch of reads.

    Host form: seq (bytes / uint8 array), offsets (uint64 array, n+1) ->
    returns a numpy array of TOP2_DTYPE.  Device form: seq and offsets are
    torch device tensors (uint8, int64 holding the offsets) and `out` a torch
    device tensor of n*32 bytes; the call is asynchronous on `stream`."""
    if hasattr(seq, "is_cuda") and seq.is_cuda:
        r = _reads_struct(seq, offsets, True, qual)
        if out is None:
            raise ValueError("device reads need a device `out` tensor of n*32 bytes")
        _check(lib().maxss_scan_reads(h_(handle), ctypes.byref(r), _buf(out, 32 * r.n, "out"),
                                      _stream_handle(stream)))
        return out
    s, off = _host_csr(seq, offsets)
    q = _host_qual(qual, s)
    n = off.size - 1
    res = np.zeros(n, dtype=TOP2_DTYPE) if out is None else out
    r = Reads(s.ctypes.data, off.ctypes.data, n, 0, _ptr(q))
    _check(lib().maxss_scan_reads(h_(handle), ctypes.byref(r), _buf(res, 32 * n, "out"),
                                  _stream_handle(stream)))
    return res


def maxss_scan_reads_noalloc(handle: int, seq, offsets, out, stream=None, qual=None):
    """maxss_scan_reads on device reads (torch tensors) with the library's
    fixed per-device scratch instead of allocations; `out` is a device tensor
    of n*32 bytes.  Calls that overlap on one device race."""
    r = _reads_struct(seq, offsets, True, qual)
    _check(lib().maxss_scan_reads_noalloc(h_(handle), ctypes.byref(r), _buf(out, 32 * r.n, "out"),
                                          _stream_handle(stream)))
    return out


def maxss_align_top(handle: int, seq, offsets, top, pad: int = 100, cigar_stride: int = 512,
                    out=None, cigar=None, stream=None, qual=None):
    """Second phase.  Host form returns (ALN_DTYPE array, list of CIGAR str);
    device form fills `out` (n*32 bytes) and `cigar` (n*cigar_stride bytes)."""
    if hasattr(seq, "is_cuda") and seq.is_cuda:
        r = _reads_struct(seq, offsets, True, qual)
        _check(lib().maxss_align_top(h_(handle), ctypes.byref(r), _buf(top, 32 * r.n, "top"), pad,
                                     _buf(out, 32 * r.n, "out"),
                                     _buf(cigar, cigar_stride * r.n, "cigar"), cigar_stride,
                                     _stream_handle(stream)))
        return out, cigar
    s, off = _host_csr(seq, offsets)
    q = _host_qual(qual, s)
    n = off.size - 1
    top = np.ascontiguousarray(top, dtype=TOP2_DTYPE)
    res = np.zeros(n, dtype=ALN_DTYPE)
    cig = np.zeros(n * cigar_stride, dtype=np.uint8)
    r = Reads(s.ctypes.data, off.ctypes.data, n, 0, _ptr(q))
    _check(lib().maxss_align_top(h_(handle), ctypes.byref(r), _buf(top, 32 * n, "top"), pad,
                                 res.ctypes.data, cig.ctypes.data, cigar_stride,
                                 _stream_handle(stream)))
    cigars = [decode_cigar(cig, i, cigar_stride) for i in range(n)]
    return res, cigars


def maxss_plan_create(handle, capacity: int, pad: int = 100, cigar_stride: int = 256) -> int:
    h = ctypes.c_void_p()
    _check(lib().maxss_plan_create(h_(handle), capacity, pad, cigar_stride, ctypes.byref(h)))
    return h.value


def maxss_plan_free(plan: int) -> None:
    lib().maxss_plan_free(plan)


def maxss_plan_run(plan: int, seq, offsets, top, aln=None, cigar=None, stream=None,
                   graph: bool = False, qual=None, cigar_stride: int | None = None):
    """One step on device reads (torch tensors); `graph` replays a captured
    HIP graph (needs a non-default stream).  With cigar_stride (the plan's),
    `cigar` is checked to hold n rows."""
    r = _reads_struct(seq, offsets, True, qual)
    fn = lib().maxss_plan_run_graph if graph else lib().maxss_plan_run
    cig = _buf(cigar, (cigar_stride or 0) * r.n, "cigar", optional=True)
    _check(fn(plan, ctypes.byref(r), _buf(top, 32 * r.n, "top"),
              _buf(aln, 32 * r.n, "aln", optional=True), cig, _stream_handle(stream)))


def maxss_autotune(handle, seq, offsets, cache_path: str | None = None, qual=None) -> dict:
    """Tune the index's tile shape on a sample (host arrays or device tensors)."""
    res = TuneResult()
    if hasattr(seq, "is_cuda") and seq.is_cuda:
        r = _reads_struct(seq, offsets, True, qual)
        keep = None
    else:
        s, off = _host_csr(seq, offsets)
        q = _host_qual(qual, s)
        r = Reads(s.ctypes.data, off.ctypes.data, off.size - 1, 0, _ptr(q))
        keep = (s, off, q)
    _check(lib().maxss_autotune(h_(handle), ctypes.byref(r),
                                cache_path.encode() if cache_path else None, ctypes.byref(res)))
    del keep
    return {f: getattr(res, f) for f, _ in TuneResult._fields_}


def maxss_index_set_tiles(handle, np_: int = 0, reads_per_tile: int = 0, rounds: int = 0) -> None:
    _check(lib().maxss_index_set_tiles(h_(handle), np_, reads_per_tile, rounds))


def maxss_scan_kernel_info(handle):
    """(offset pairs per lane, kernel variant) of the next scan on the index."""
    np_, kind = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().maxss_scan_kernel_info(h_(handle), ctypes.byref(np_), ctypes.byref(kind)))
    return np_.value, kind.value


def maxss_mapq(top, n: int, mapq, mapped=None, ratio_num: int = 9, ratio_den: int = 10,
               min_mapq: int = -1, stream=None) -> None:
    """Mapping quality of n top-2 records (device tensors: top n*32 bytes,
    mapq and mapped n bytes each)."""
    _check(lib().maxss_mapq(_buf(top, 32 * n, "top"), n, ratio_num, ratio_den, min_mapq,
                            _buf(mapq, n, "mapq"), _buf(mapped, n, "mapped", optional=True),
                            _stream_handle(stream)))


def _two_pass(call) -> str:
    """Run a formatting call once for its size, then into a buffer."""
    need = ctypes.c_uint64()
    st = call(None, 0, ctypes.byref(need))
    if st == 0:
        return ""
    buf = ctypes.create_string_buffer(max(1, need.value))
    _check(call(buf, need.value, ctypes.byref(need)))
    return buf.raw[:need.value].decode()


def maxss_sam_header(handle, rname: str) -> str:
    r = rname.encode()
    return _two_pass(lambda b, cap, ln: lib().maxss_sam_header(h_(handle), r, b, cap, ln))


def maxss_sam_records(seq, offsets, top: np.ndarray, aln: np.ndarray, cigar: np.ndarray,
                      cigar_stride: int, mapq: np.ndarray, mapped: np.ndarray, rname: str,
                      names=None, qual=None) -> str:
    """SAM lines from host copies of the records (numpy arrays); `qual`
    (Phred+33, one per read base) fills the QUAL column."""
    s, off = _host_csr(seq, offsets)
    n = off.size - 1
    q8 = _host_qual(qual, s)
    r = Reads(s.ctypes.data, off.ctypes.data, n, 0, q8.ctypes.data if q8 is not None else None)
    top = np.ascontiguousarray(top)
    aln = np.ascontiguousarray(aln)
    cig = np.ascontiguousarray(cigar, dtype=np.uint8)
    q = np.ascontiguousarray(mapq, dtype=np.uint8)
    mp = np.ascontiguousarray(mapped, dtype=np.uint8)
    if min(top.size, aln.size, q.size, mp.size) < n:
        raise ValueError("top, aln, mapq and mapped need one entry per read (%d reads)" % n)
    if cig.size < n * cigar_stride:
        raise ValueError("cigar holds %d bytes, %d reads x stride %d needed"
                         % (cig.size, n, cigar_stride))
    nm = None
    if names is not None:
        enc = [x.encode() for x in names]
        if len(enc) < n:
            raise ValueError("%d names for %d reads" % (len(enc), n))
        nm = (ctypes.c_char_p * len(enc))(*enc)
    rn = rname.encode()
    return _two_pass(lambda b, cap, ln: lib().maxss_sam_records(
        ctypes.byref(r), top.ctypes.data, aln.ctypes.data, cig.ctypes.data, cigar_stride,
        q.ctypes.data, mp.ctypes.data, rn, ctypes.cast(nm, ctypes.c_void_p) if nm else None,
        b, cap, ln))


def decode_cigar(buf: np.ndarray, i: int, stride: int) -> str:
    row = buf[i * stride:(i + 1) * stride]
    z = np.nonzero(row == 0)[0]
    end = int(z[0]) if z.size else stride
    return row[:end].tobytes().decode()


def h_(handle):
    if isinstance(handle, Index):
        return handle.handle
    return handle


class Plan:
    """Owner of a launch plan (all scratch of a step, preallocated)."""

    def __init__(self, index: "Index", capacity: int, pad: int = 100, cigar_stride: int = 256):
        self.index = index
        self.handle = maxss_plan_create(index.handle, capacity, pad, cigar_stride)
        self.capacity, self.pad, self.cigar_stride = capacity, pad, cigar_stride

    def run(self, seq, offsets, top, aln=None, cigar=None, stream=None, graph=False, qual=None):
        maxss_plan_run(self.handle, seq, offsets, top, aln, cigar, stream, graph, qual,
                       self.cigar_stride)

    def close(self):
        if getattr(self, "handle", None):
            maxss_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Model:
    """Owner of a proposal network (fp32 master + bf16 copies + Adam state):
    created in the library from a seed and an initialisation, from given
    parameters, or loaded from a file."""

    def __init__(self, params=None, path: str | None = None, seed: int = 0,
                 init: int = MAXSS_INIT_GLOROT):
        h = ctypes.c_void_p()
        if path is not None:
            _check(lib().maxss_model_load(path.encode(), ctypes.byref(h)))
        elif params is not None:
            p = np.ascontiguousarray(params, dtype=np.float32)
            if p.size != MLP_PARAMS:
                raise ValueError("expected %d parameters" % MLP_PARAMS)
            self._init = p
            _check(lib().maxss_model_from_params(p.ctypes.data, ctypes.byref(h)))
        else:
            _check(lib().maxss_model_create(seed, init, ctypes.byref(h)))
        self.handle = h.value

    def train(self, index, seq, offsets, labels, steps: int, batch: int = 256, lr: float = 1e-3,
              seed: int = 0, hard_negatives: int = 0, eval_every: int = 0, K: int = 64,
              val_fraction: float = 0.1, target_agreement: float = 0.995, loss_trace=None,
              cand_trace=None, stream=None, qual=None) -> dict:
        """maxss_model_train on device reads and their device top-2 records;
        returns the statistics as a dict.  loss_trace (float32, `steps`) and
        cand_trace (int32, steps*batch*64), host numpy arrays, are filled
        when given."""
        r = _reads_struct(seq, offsets, True, qual)
        tr = ct = None
        if loss_trace is not None:
            if not (isinstance(loss_trace, np.ndarray) and loss_trace.dtype == np.float32):
                raise ValueError("loss_trace must be a float32 numpy array")
            tr = _buf(loss_trace, 4 * steps, "loss_trace")
        if cand_trace is not None:
            if not (isinstance(cand_trace, np.ndarray) and cand_trace.dtype == np.int32):
                raise ValueError("cand_trace must be an int32 numpy array")
            ct = _buf(cand_trace, 4 * steps * batch * 64, "cand_trace")
        o = TrainOpts(steps, batch, lr, seed, hard_negatives, eval_every, K, val_fraction,
                      target_agreement, tr, ct)
        st = TrainStats()
        _check(lib().maxss_model_train(self.handle, h_(index), ctypes.byref(r),
                                       _buf(labels, 32 * r.n, "labels"), ctypes.byref(o),
                                       ctypes.byref(st), _stream_handle(stream)))
        return {f: getattr(st, f) for f, _ in TrainStats._fields_}

    def params(self) -> np.ndarray:
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(lib().maxss_model_get_params(self.handle, out.ctypes.data))
        return out

    def save(self, path: str):
        _check(lib().maxss_model_save(self.handle, path.encode()))

    def scores(self, index, seq, offsets, out, stream=None):
        r = _reads_struct(seq, offsets, True)
        nf = maxss_index_info(h_(index))[1]
        _check(lib().maxss_proposal_scores(h_(index), self.handle, ctypes.byref(r),
                                           _buf(out, 4 * r.n * nf, "scores"),
                                           _stream_handle(stream)))

    def candidates(self, index, seq, offsets, K, margin, cand, margins, fell_back, stream=None):
        r = _reads_struct(seq, offsets, True)
        _check(lib().maxss_proposal_candidates(h_(index), self.handle, ctypes.byref(r), K,
                                               margin, _buf(cand, 4 * r.n * K, "cand"),
                                               _buf(margins, 4 * r.n, "margins"),
                                               _buf(fell_back, r.n, "fell_back"),
                                               _stream_handle(stream)))

    def scan(self, index, seq, offsets, K, margin, out, fell_back=None, stream=None, qual=None,
             min_score: int = -1):
        r = _reads_struct(seq, offsets, True, qual)
        _check(lib().maxss_scan_reads_proposed(h_(index), self.handle, ctypes.byref(r), K, margin,
                                               min_score, _buf(out, 32 * r.n, "out"),
                                               _buf(fell_back, r.n, "fell_back", optional=True),
                                               _stream_handle(stream)))

    def train_step(self, index, seq, offsets, cand, strand, lr, loss=None, grad=None,
                   stream=None):
        r = _reads_struct(seq, offsets, True)
        _check(lib().maxss_model_train_step(self.handle, h_(index), ctypes.byref(r),
                                            _buf(cand, 4 * 64 * r.n, "cand"),
                                            _buf(strand, r.n, "strand"), lr,
                                            _buf(loss, 4, "loss", optional=True),
                                            _buf(grad, 4 * MLP_PARAMS, "grad", optional=True),
                                            _stream_handle(stream)))

    def close(self):
        if getattr(self, "handle", None):
            lib().maxss_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def maxss_choose_acceptance(margin, best_score, correct, target: float):
    """(tau, min_score, accept_frac, agreement) from held-out host arrays."""
    m = np.ascontiguousarray(margin, dtype=np.float32)
    b = np.ascontiguousarray(best_score, dtype=np.int32)
    c = np.ascontiguousarray(correct, dtype=np.uint8)
    if not (m.size == b.size == c.size):
        raise ValueError("margin, best_score and correct need one entry per read")
    tau, ms = ctypes.c_float(), ctypes.c_int32()
    acc, agr = ctypes.c_float(), ctypes.c_float()
    _check(lib().maxss_choose_acceptance(m.size, m.ctypes.data, b.ctypes.data, c.ctypes.data,
                                         target, ctypes.byref(tau), ctypes.byref(ms),
                                         ctypes.byref(acc), ctypes.byref(agr)))
    return tau.value, ms.value, acc.value, agr.value


def maxss_profiles(index, seq=None, offsets=None, read_prof=None, frag_prof=None, stream=None):
    r = _reads_struct(seq, offsets, True) if seq is not None else None
    nr = r.n if r is not None else 0
    nf = maxss_index_info(h_(index))[1]
    _check(lib().maxss_profiles(h_(index), ctypes.byref(r) if r is not None else None,
                                _buf(read_prof, 4 * 2 * 256 * nr, "read_prof", optional=True),
                                _buf(frag_prof, 4 * 256 * nf, "frag_prof", optional=True),
                                _stream_handle(stream)))


class Index:
    """Owner of a genome index (freed on close / garbage collection)."""

    def __init__(self, genome, frag_len: int, max_read_len: int, match: int = 1,
                 mismatch: int = -1, gap: int = -2, flags: int = 0, qual_scale: int = 0):
        self.handle = maxss_index_genome(genome, frag_len, max_read_len, match, mismatch, gap,
                                         flags, qual_scale)
        self.G, self.NF, self.F = maxss_index_info(self.handle)
        self.max_read_len = max_read_len
        self.params = dict(match=match, mismatch=mismatch, gap=gap, flags=flags,
                           qual_scale=qual_scale)

    def scan(self, seq, offsets, out=None, stream=None, qual=None):
        return maxss_scan_reads(self.handle, seq, offsets, out, stream, qual)

    def align(self, seq, offsets, top, pad: int = 100, cigar_stride: int = 512, out=None,
              cigar=None, stream=None, qual=None):
        return maxss_align_top(self.handle, seq, offsets, top, pad, cigar_stride, out, cigar,
                               stream, qual)

    def set_tiles(self, np_: int = 0, reads_per_tile: int = 0, rounds: int = 0):
        maxss_index_set_tiles(self.handle, np_, reads_per_tile, rounds)

    def kernel_info(self):
        return maxss_scan_kernel_info(self.handle)

    def autotune(self, seq, offsets, cache_path=None, qual=None):
        return maxss_autotune(self.handle, seq, offsets, cache_path, qual)

    def close(self):
        if getattr(self, "handle", None):
            maxss_index_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
