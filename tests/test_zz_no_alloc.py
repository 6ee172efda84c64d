"""maxss_scan_reads_noalloc (the first phase with the library's fixed
per-device scratch, for callers that cannot allocate) against
maxss_scan_reads: bit-exact records on two calls in a row, the second with a
smaller batch, for plain scores, the neighbour exclusion and quality scores;
one batch large enough that the scratch caps the fragment chunks per read;
and the host-side rejections (host reads, a batch beyond the scratch)."""
import numpy as np
import pytest

import gen
import oracle
import paper_1403_2136_amd as mx

pytestmark = pytest.mark.gpu
FIELDS = ("frag", "score", "offset", "strand")


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _dev(reads, qual=None):
    torch = _torch()
    d = torch.device("cuda:0")
    s = torch.from_numpy(np.ascontiguousarray(reads.seq, dtype=np.uint8)).to(d)
    o = torch.from_numpy(reads.offsets.astype(np.int64)).to(d)
    q = torch.from_numpy(np.ascontiguousarray(qual, dtype=np.uint8)).to(d) if qual is not None else None
    return s, o, q


def _both(ix, reads, qual=None):
    """(no-alloc records, maxss_scan_reads records) for the same device reads."""
    torch = _torch()
    s, o, q = _dev(reads, qual)
    n = reads.n
    a = torch.full((n * 32,), 0xA5, dtype=torch.uint8, device="cuda:0")
    b = torch.zeros(n * 32, dtype=torch.uint8, device="cuda:0")
    st = torch.cuda.current_stream()
    mx.maxss_scan_reads_noalloc(ix.handle, s, o, a, stream=st, qual=q)
    mx.maxss_scan_reads(ix.handle, s, o, b, stream=st, qual=q)
    torch.cuda.synchronize()
    return a.cpu().numpy().view(mx.TOP2_DTYPE), b.cpu().numpy().view(mx.TOP2_DTYPE)


def _same(got, ref, what):
    for f in FIELDS:
        bad = np.nonzero((got[f] != ref[f]).any(axis=1))[0]
        assert bad.size == 0, "%s: %s differs for %d reads, first %d: %s vs %s" % (
            what, f, bad.size, bad[0], got[bad[0]], ref[bad[0]])
    assert got.tobytes() == ref.tobytes(), what


def test_noalloc_two_calls_second_smaller():
    g = gen.uniform_genome(500_000, 61)
    ix = mx.Index(g.seq, 2048, 128)
    big = gen.sample_reads(g, 220_000, 62, [36, 51, 100, 128], 0.1, 0.3, indel_max=2)
    small = gen.sample_reads(g, 1_000, 63, [36, 51, 100, 128], 0.1, 0.3, indel_max=2)
    print("no-alloc: %d reads (scratch caps the chunks), then %d" % (big.n, small.n), flush=True)
    a, b = _both(ix, big)
    _same(a, b, "first call, %d reads" % big.n)
    a, b = _both(ix, small)
    _same(a, b, "second call, %d reads" % small.n)
    sub = small.subset(np.arange(200))
    ref = oracle.scan(g.seq, 2048, sub.seq, sub.offsets, 1, -1, nthreads=16)
    _same(a[:200], ref, "second call against the oracle")
    ix.close()


def test_noalloc_exclusion_and_quality():
    g = gen.uniform_genome(200_000, 71)
    seq = g.seq.copy()
    seq[150_000:152_000] = seq[10_000:12_000]      # an exact repeat
    g = gen.Genome(seq, "noalloc")
    ix = mx.Index(g.seq, 1024, 150, flags=mx.MAXSS_EXCLUDE_ADJACENT)
    for n, seed in ((5_000, 72), (600, 73)):
        r = gen.sample_reads(g, n, seed, [40, 100, 150], 0.05, 0.3, indel_max=2)
        print("no-alloc exclusion: %d reads" % n, flush=True)
        a, b = _both(ix, r)
        _same(a, b, "exclusion, %d reads" % n)
    ix.close()
    ixq = mx.Index(g.seq, 2048, 150, 5, -4, -26, qual_scale=10)
    for n, seed in ((3_000, 74), (400, 75)):
        r = gen.sample_reads(g, n, seed, [40, 100, 150], 0.05, 0.3, indel_max=2)
        q = gen.sample_qualities(r, seed + 100)
        print("no-alloc quality: %d reads" % n, flush=True)
        a, b = _both(ixq, r, q)
        _same(a, b, "quality, %d reads" % n)
    ixq.close()


def test_noalloc_rejections():
    torch = _torch()
    g = gen.uniform_genome(50_000, 81)
    r = gen.sample_reads(g, 10, 82, [100], 0.1, 0.1)
    ix = mx.Index(g.seq, 2048, 8192)
    # 5,000 reads of stride 8192 need about 82 MB of encoded reads alone
    many = gen.sample_reads(g, 5_000, 83, [100], 0.1, 0.1)
    s, o, _ = _dev(many)
    out = torch.empty(many.n * 32, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(mx.MaxssError) as e:
        mx.maxss_scan_reads_noalloc(ix.handle, s, o, out)
    assert e.value.status == mx.MAXSS_EINVAL and "scratch" in str(e.value)
    # host reads are refused
    hs = np.ascontiguousarray(r.seq)
    ho = np.ascontiguousarray(r.offsets)
    hout = np.zeros(r.n, dtype=mx.TOP2_DTYPE)
    rs = mx.Reads(hs.ctypes.data, ho.ctypes.data, r.n, 0, None)
    import ctypes
    st = mx.lib().maxss_scan_reads_noalloc(ix.handle, ctypes.byref(rs), hout.ctypes.data, None)
    assert st == mx.MAXSS_EINVAL
    # a batch that fits still runs on the same index after the rejection
    s, o, _ = _dev(r)
    a = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda:0")
    mx.maxss_scan_reads_noalloc(ix.handle, s, o, a)
    torch.cuda.synchronize()
    ref = oracle.scan(g.seq, 2048, r.seq, r.offsets, 1, -1, nthreads=8)
    _same(a.cpu().numpy().view(mx.TOP2_DTYPE), ref, "after a rejection")
    ix.close()
