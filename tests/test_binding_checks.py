"""The binding checks every buffer the library reads or writes a known number
of bytes of (size and contiguity) before the call, so a short or strided
buffer raises instead of reaching a kernel or a host copy.  CPU only: each
check fires before any device work."""
import numpy as np
import pytest
import torch

import paper_1403_2136_amd as mx


def test_buf_accepts_exact_and_larger_buffers():
    a = np.zeros(4, dtype=mx.TOP2_DTYPE)
    assert mx._buf(a, 128, "a") == a.ctypes.data
    assert mx._buf(a, 64, "a") == a.ctypes.data
    t = torch.zeros(10, dtype=torch.float32)
    assert mx._buf(t, 40, "t") == t.data_ptr()
    assert mx._buf(1234, 1 << 40, "raw") == 1234        # raw addresses pass unchecked
    assert mx._buf(None, 8, "x", optional=True) is None


def test_buf_rejects_short_strided_and_missing_buffers():
    with pytest.raises(ValueError, match="holds 96 bytes, 128 needed"):
        mx._buf(np.zeros(3, dtype=mx.TOP2_DTYPE), 128, "out")
    with pytest.raises(ValueError, match="contiguous"):
        mx._buf(torch.zeros(8, 8)[:, 0], 4, "strided")
    with pytest.raises(ValueError, match="contiguous"):
        mx._buf(np.zeros(16, np.uint8)[::2], 4, "strided")
    with pytest.raises(ValueError, match="required"):
        mx._buf(None, 4, "mapq")


def test_calls_check_before_the_library_runs():
    # host scan with an `out` too small for the reads: raises before any
    # device call (the handle is never used)
    with pytest.raises(ValueError, match="out holds"):
        mx.maxss_scan_reads(0, b"ACGTACGT", [0, 4, 8], out=np.zeros(1, dtype=mx.TOP2_DTYPE))
    with pytest.raises(ValueError, match="top holds"):
        mx.maxss_align_top(0, b"ACGTACGT", [0, 4, 8], np.zeros(1, dtype=mx.TOP2_DTYPE))
    with pytest.raises(ValueError, match="mapq holds"):
        mx.maxss_mapq(np.zeros(5, dtype=mx.TOP2_DTYPE), 5, np.zeros(4, np.uint8))
    with pytest.raises(ValueError, match="one entry per read"):
        mx.maxss_sam_records(b"ACGTACGT", [0, 4, 8], np.zeros(1, dtype=mx.TOP2_DTYPE),
                             np.zeros(2, dtype=mx.ALN_DTYPE), np.zeros(16, np.uint8), 8,
                             np.zeros(2, np.uint8), np.zeros(2, np.uint8), "c")
    with pytest.raises(ValueError, match="cigar holds"):
        mx.maxss_sam_records(b"ACGTACGT", [0, 4, 8], np.zeros(2, dtype=mx.TOP2_DTYPE),
                             np.zeros(2, dtype=mx.ALN_DTYPE), np.zeros(15, np.uint8), 8,
                             np.zeros(2, np.uint8), np.zeros(2, np.uint8), "c")
    with pytest.raises(ValueError, match="names for"):
        mx.maxss_sam_records(b"ACGTACGT", [0, 4, 8], np.zeros(2, dtype=mx.TOP2_DTYPE),
                             np.zeros(2, dtype=mx.ALN_DTYPE), np.zeros(16, np.uint8), 8,
                             np.zeros(2, np.uint8), np.zeros(2, np.uint8), "c", names=["a"])
