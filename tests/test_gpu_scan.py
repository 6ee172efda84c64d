"""GPU parity of the first phase (scan + top-2) against the CPU oracle.

Bit-exact on every field of every record: fragment ids, scores, offsets and
strands of the best and second-best fragments.
"""
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


def assert_same(got, ref, what=""):
    for f in FIELDS:
        bad = np.nonzero((got[f] != ref[f]).any(axis=1))[0]
        assert bad.size == 0, "%s: field %s differs for %d reads, first %d: gpu %s oracle %s" % (
            what, f, bad.size, bad[0], got[bad[0]], ref[bad[0]])


def scan_device(ix, seq, offsets):
    torch = _torch()
    dev = torch.device("cuda:0")
    s = torch.from_numpy(np.ascontiguousarray(seq, dtype=np.uint8)).to(dev)
    o = torch.from_numpy(np.ascontiguousarray(offsets).astype(np.int64)).to(dev)
    n = len(offsets) - 1
    out = torch.empty(max(n, 1) * 32, dtype=torch.uint8, device=dev)
    ix.scan(s, o, out, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    return out.cpu().numpy()[:n * 32].view(mx.TOP2_DTYPE)


def csr(reads):
    reads = [r if isinstance(r, bytes) else r.encode() for r in reads]
    off = np.zeros(len(reads) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(r) for r in reads])
    return b"".join(reads), off


@pytest.fixture(scope="module")
def tiny():
    w = gen.workload("tiny")
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap)
    ref = oracle.scan(w.genome.seq, w.F, w.reads.seq, w.reads.offsets, w.M, w.X, nthreads=8)
    yield w, ix, ref
    ix.close()


def test_tiny_full_parity_host_reads(tiny):
    w, ix, ref = tiny
    got = ix.scan(w.reads.seq, w.reads.offsets)
    assert_same(got, ref, "tiny/host")


def test_tiny_full_parity_device_reads(tiny):
    w, ix, ref = tiny
    got = scan_device(ix, w.reads.seq, w.reads.offsets)
    assert_same(got, ref, "tiny/device")


def test_deterministic_repeat(tiny):
    w, ix, ref = tiny
    a = scan_device(ix, w.reads.seq, w.reads.offsets)
    b = scan_device(ix, w.reads.seq, w.reads.offsets)
    assert a.tobytes() == b.tobytes()


def _edge_case(G, F, lens, seed, M=1, X=-1, flags=0, n_runs=0, rate=0.15, max_len=None,
               repeats=0):
    g = gen.uniform_genome(G, seed)
    if n_runs:
        g = gen.with_n_runs(g, seed + 7, n_runs, 1, 60)
    seq = g.seq.copy()
    st = gen.Stream(seed, "edge.repeats")
    for _ in range(repeats):
        L = int(st.integers(20, 300, 1)[0])
        if G <= 2 * L:
            break
        a = int(st.integers(0, G - L, 1)[0])
        b = int(st.integers(0, G - L, 1)[0])
        seq[b:b + L] = seq[a:a + L]
    g = gen.Genome(seq, g.name)
    r = gen.sample_reads(g, len(lens), seed + 1, lens, rate, rate, length_mode="choice") \
        if len(set(lens)) == 1 else None
    if r is None:
        parts = []
        for i, m in enumerate(lens):
            rr = gen.sample_reads(g, 1, seed + 100 + i, [m], rate, rate)
            parts.append(rr.read(0))
        s, off = csr(parts)
    else:
        s, off = r.seq.tobytes(), r.offsets
    ml = max_len or max(lens)
    ix = mx.Index(g.seq, F, ml, M, X, -2, flags)
    ref = oracle.scan(g.seq, F, s, off, M, X, flags=flags, nthreads=8)
    got = ix.scan(s, off)
    ix.close()
    return got, ref


@pytest.mark.parametrize("G,F,lens", [
    (50_000, 2048, [100] * 40),                       # G % F != 0, several fragments
    (4096, 4096, [36, 250, 100]),                     # exactly one fragment (no second)
    (3000, 4096, [80, 5, 1]),                          # G < F
    (20_000, 48, [30, 47, 48, 49]),                   # small F (paper's E. coli choice)
    (20_000, 16, [1, 2, 15, 16, 17]),                  # F = 16, reads around F
    (30_000, 2064, [33, 100, 151]),                   # F not a multiple of 128
    (70_000, 4096, [36, 51, 100, 150, 250] * 4),      # mixed lengths, wide tiles
    (40_000, 1024, list(range(1, 130, 7))),           # ragged lengths across unroll
    (30_000, 2048, list(range(1, 34)) + [95, 100, 111, 112, 113]),   # every m % 16
    (40_000, 4096, list(range(1, 66, 2)) + [96, 127, 128, 129, 250]),  # m % 32, wide
])
def test_edge_shapes(G, F, lens):
    got, ref = _edge_case(G, F, lens, seed=G % 997 + F)
    assert_same(got, ref, "G=%d F=%d" % (G, F))


@pytest.mark.parametrize("F", [512, 2048])
def test_n_runs_and_paper_scores(F):
    got, ref = _edge_case(30_000, F, [100] * 24, seed=5, M=5, X=-4, n_runs=40)
    assert_same(got, ref, "N runs, 5/-4")


def test_exact_repeats_ties():
    got, ref = _edge_case(40_000, 256, [60] * 30, seed=9, repeats=60, rate=0.0)
    assert_same(got, ref, "repeats")
    assert (got["score"][:, 0] == 60).all()


@pytest.mark.parametrize("F", [1024, 2048])
def test_one_strand_flag(F):
    got, ref = _edge_case(30_000, F, [90] * 20, seed=13, flags=mx.MAXSS_ONE_STRAND)
    assert_same(got, ref, "one strand")


def test_bank_kernel_n_in_every_block_position():
    # reads with N at each step of a 16-step block, in full blocks and in the
    # m % 16 tail, and reads that are N up to one base (register-bank path)
    g = gen.uniform_genome(40_000, 41)
    src = g.seq[3000:3000 + 90].tobytes()
    reads = []
    # m = 90: blocks 0-3 stage the window ahead, block 4 (64-79) is the last
    # block (no staging), 80-89 the tail
    for p in list(range(0, 48)) + [64, 70, 79, 80, 85, 89]:
        r = bytearray(src)
        r[p] = ord("N")
        reads.append(bytes(r))
    reads += [b"N" * 89 + src[:1], src[:1] + b"N" * 40, b"N" * 16 + src[16:64]]
    s, off = csr(reads)
    ix = mx.Index(g.seq, 2048, 90)
    assert ix.kernel_info()[1] == mx.MAXSS_KERNEL_REGISTER_BANK
    got = ix.scan(s, off)
    ref = oracle.scan(g.seq, 2048, s, off, nthreads=8)
    ix.close()
    assert_same(got, ref, "N positions")


@pytest.mark.parametrize("F", [1024, 2048])
def test_reads_with_n_and_all_n(F):
    g = gen.uniform_genome(20_000, 17)
    reads = [b"N" * 50, b"ACGTN" * 10, g.seq[100:180].tobytes().replace(b"A", b"N"),
             b"acgt" * 12, g.seq[5000:5100].tobytes().lower(),
             g.seq[7000:7037].tobytes()[:20] + b"N" + g.seq[7021:7037].tobytes()]
    s, off = csr(reads)
    ix = mx.Index(g.seq, F, 100)
    got = ix.scan(s, off)
    ref = oracle.scan(g.seq, F, s, off, nthreads=4)
    ix.close()
    assert_same(got, ref, "N reads")
    assert got["score"][0].tolist() == [0, 0]


def test_max_score_range_limit():
    # max_read_len * match = 65535: the largest exact 16-bit case
    g = gen.uniform_genome(12_000, 23)
    read = g.seq[1000:1000 + 8191].tobytes()
    s, off = csr([read, read[:4000]])
    ix = mx.Index(g.seq, 4096, 8191, 8, -8)
    got = ix.scan(s, off)
    ref = oracle.scan(g.seq, 4096, s, off, 8, -8, nthreads=2)
    ix.close()
    assert_same(got, ref, "max range")
    assert got["score"][0][0] == 8191 * 8


@pytest.mark.parametrize("np_", [8, 16, 32])
def test_narrow_score_range_limit(np_):
    # max_read_len * match = 31744: the largest bound that takes the two-step
    # kernels (a full-length exact copy scores 0xFC00 - 0x8000 in biased form)
    g = gen.uniform_genome(12_000, 31)
    read = g.seq[700:700 + 3968].tobytes()
    mut = bytearray(read[:3000])
    mut[1500] = ord("A") if mut[1500] != ord("A") else ord("C")
    s, off = csr([read, bytes(mut), read[:1]])
    ix = mx.Index(g.seq, 4096, 3968, 8, -8)
    mx.maxss_index_set_tiles(ix.handle, np_, 0, 0)
    got = ix.scan(s, off)
    ref = oracle.scan(g.seq, 4096, s, off, 8, -8, nthreads=2)
    ix.close()
    assert_same(got, ref, "narrow range NP=%d" % np_)
    assert got["score"][0][0] == 31744


def test_device_invalid_reads_marked():
    torch = _torch()
    g = gen.uniform_genome(10_000, 29)
    good = g.seq[200:300].tobytes()
    s, off = csr([good, b"ACGX" * 5, good[:50], b"A" * 120])
    off = np.concatenate([off[:2], off[1:2], off[2:]])   # insert an empty read at index 1
    ix = mx.Index(g.seq, 512, 100)
    got = scan_device(ix, np.frombuffer(s, np.uint8), off)
    ix.close()
    assert got["frag"][1][0] == mx.MAXSS_READ_INVALID      # empty
    assert got["frag"][2][0] == mx.MAXSS_READ_INVALID      # bad character
    assert got["frag"][4][0] == mx.MAXSS_READ_INVALID      # too long
    ref = oracle.scan(g.seq, 512, good + good[:50], [0, 100, 150])
    assert_same(got[[0, 3]], ref, "valid reads among invalid ones")


def test_host_reads_errors():
    g = gen.uniform_genome(5000, 31)
    ix = mx.Index(g.seq, 512, 50)
    with pytest.raises(mx.MaxssError) as e:
        ix.scan(b"A" * 51, [0, 51])
    assert e.value.status == mx.MAXSS_ETOOLONG
    with pytest.raises(mx.MaxssError) as e:
        ix.scan(b"AC", [0, 0, 2])
    assert e.value.status == mx.MAXSS_ETOOLONG
    with pytest.raises(mx.MaxssError) as e:
        ix.scan(b"ACGU", [0, 4])
    assert e.value.status == mx.MAXSS_EINVAL
    assert ix.scan(b"", [0]).size == 0
    ix.close()


@pytest.mark.slow
def test_bacterial_full_size_sampled():
    """The full 100,000-read bacterial workload in one call, in the bench's
    launch configuration; 64 sampled reads are checked against the oracle."""
    w = gen.workload("bacterial")
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap)
    got = scan_device(ix, w.reads.seq, w.reads.offsets)
    ix.close()
    idx = np.sort(gen.Stream(77, "parity.sample").integers(0, w.reads.n, 64))
    sub = w.reads.subset(idx)
    ref = oracle.scan(w.genome.seq, w.F, sub.seq, sub.offsets, w.M, w.X, nthreads=16)
    assert_same(got[idx], ref, "bacterial sample")
    # properties over every read
    assert (got["score"][:, 0] >= got["score"][:, 1]).all()
    assert (got["score"][:, 0] <= 100).all() and (got["score"][:, 1] >= 0).all()
    assert (got["frag"][:, 0] != got["frag"][:, 1]).all()


def test_kernel_info_follows_tiles_and_scores():
    g = gen.uniform_genome(20_000, 37)
    ix = mx.Index(g.seq, 2048, 100)
    assert ix.kernel_info() == (16, mx.MAXSS_KERNEL_REGISTER_BANK)
    ix.set_tiles(8, 0, 0)
    assert ix.kernel_info() == (8, mx.MAXSS_KERNEL_TWO_STEP)
    ix.set_tiles(0, 0, 0)
    ix.close()
    ix = mx.Index(g.seq, 4096, 4000, 8, -8)             # bound 32000 > 31744
    assert ix.kernel_info() == (32, mx.MAXSS_KERNEL_STEP_MAX)
    ix.close()
    # quality scores: the register banks for reads with one score pair (a
    # two-step launch for the others)
    ix = mx.Index(g.seq, 2048, 100, 5, -4, -26, qual_scale=10)
    assert ix.kernel_info() == (16, mx.MAXSS_KERNEL_REGISTER_BANK)
    ix.set_tiles(8, 0, 0)
    assert ix.kernel_info() == (8, mx.MAXSS_KERNEL_TWO_STEP)
    ix.close()
