"""The C-ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host before touching a device (no compute calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1403_2136_amd as mx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "maxss.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(maxss_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(mx.LIB_PATH):
        from paper_1403_2136_amd import build
        build.build()
    return mx.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert set(names) == set(mx.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_version(L):
    assert mx.maxss_version().startswith("maxss-gfx950")


def test_struct_sizes():
    assert ctypes.sizeof(mx.Params) == 28
    assert ctypes.sizeof(mx.Reads) == 32
    assert mx.TOP2_DTYPE.itemsize == 32 and mx.ALN_DTYPE.itemsize == 32


@pytest.mark.parametrize("kw,msg", [
    (dict(frag_len=0), "frag_len"),
    (dict(frag_len=40), "frag_len"),
    (dict(match=0), "match"),
    (dict(match=200), "match"),
    (dict(mismatch=1), "mismatch"),
    (dict(gap=1), "gap"),
    (dict(max_read_len=0), "max_read_len"),
    (dict(max_read_len=9000), "max_read_len"),
    (dict(match=127, max_read_len=1000), "65535"),
    (dict(flags=64), "flags"),
    (dict(qual_scale=128), "qual_scale"),
    (dict(mismatch=-4, qual_scale=100), "qual_scale"),
    (dict(qual_scale=100, max_read_len=1000), "65535"),
])
def test_index_rejects_bad_params(L, kw, msg):
    a = dict(frag_len=64, max_read_len=100, match=1, mismatch=-1, gap=-2, flags=0)
    a.update(kw)
    with pytest.raises(mx.MaxssError) as e:
        mx.maxss_index_genome(b"ACGT" * 100, **a)
    assert e.value.status == mx.MAXSS_EINVAL and msg in str(e.value)


def test_index_rejects_bad_genome(L):
    with pytest.raises(mx.MaxssError) as e:
        mx.maxss_index_genome(b"ACGTX", 16, 10)
    assert e.value.status == mx.MAXSS_EINVAL and "0x58" in str(e.value)
    with pytest.raises(mx.MaxssError) as e:
        mx.maxss_index_genome(b"", 16, 10)
    assert e.value.status == mx.MAXSS_EINVAL


def test_null_arguments(L):
    p = mx.Params(1, -1, -2, 16, 10, 0)
    assert L.maxss_index_genome(None, 4, ctypes.byref(p), None) == mx.MAXSS_EINVAL
    assert L.maxss_scan_reads(None, None, None, None) == mx.MAXSS_EINVAL
    assert L.maxss_scan_reads_noalloc(None, None, None, None) == mx.MAXSS_EINVAL
    assert L.maxss_align_top(None, None, None, 100, None, None, 16, None) == mx.MAXSS_EINVAL
    assert L.maxss_index_info(None, None, None, None) == mx.MAXSS_EINVAL
    L.maxss_index_free(None)   # no-op
    assert b"NULL" in L.maxss_last_error()


def test_host_offsets_checked_against_buffer(L):
    with pytest.raises(ValueError):
        mx._host_csr(b"ACGT", [0, 5])
    with pytest.raises(ValueError):
        mx._host_csr(b"ACGT", [0, 3, 2])
    s, off = mx._host_csr(b"ACGT", [0, 2, 4])
    assert s.size == 4 and off.tolist() == [0, 2, 4]


def test_header_constants_match_the_binding():
    txt = open(os.path.join(ROOT, "include", "maxss.h")).read()
    defs = dict(re.findall(r"#define\s+(MAXSS_[A-Z0-9_]+)\s+(-?\d+)u?\b", txt))
    assert {"MAXSS_ONE_STRAND", "MAXSS_NW_GLOBAL", "MAXSS_FAST", "MAXSS_EXCLUDE_ADJACENT",
            "MAXSS_KERNEL_REGISTER_BANK"} <= set(defs)
    for name, value in defs.items():
        if hasattr(mx, name):
            assert getattr(mx, name) == int(value), name
    flags = [int(defs[k]) for k in ("MAXSS_ONE_STRAND", "MAXSS_NW_GLOBAL", "MAXSS_FAST",
                                    "MAXSS_EXCLUDE_ADJACENT")]
    assert len(set(flags)) == 4 and all(f & (f - 1) == 0 for f in flags)  # distinct bits
