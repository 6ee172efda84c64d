"""Base-quality scoring on the GPU (position-specific match / mismatch from
Phred qualities, both phases): records, alignments and CIGARs bit-exact
against the oracle for every tile shape, host and device reads, the fast
scan, one strand, the plan and its graph, and the error paths."""
import numpy as np
import pytest

import gen
import oracle
import paper_1403_2136_amd as mx

pytestmark = pytest.mark.gpu
FIELDS = ("frag", "score", "offset", "strand")
M, X, GAP, QS = 5, -4, -26, 10


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def assert_same(got, ref, what=""):
    for f in FIELDS:
        bad = np.nonzero((got[f] != ref[f]).any(axis=1))[0]
        assert bad.size == 0, "%s: %s differs for %d reads, first %d: gpu %s oracle %s" % (
            what, f, bad.size, bad[0], got[bad[0]], ref[bad[0]])


def _case(seed=7):
    g = gen.with_n_runs(gen.uniform_genome(21_111, seed), seed + 1, 10, 1, 60)
    seq = g.seq.copy()
    seq[15000:15300] = seq[2000:2300]          # exact repeats
    r = gen.sample_reads(gen.Genome(seq, "q"), 40, seed + 2, [1, 2, 17, 64, 111, 250], 0.0, 0.3,
                         indel_max=2)
    q = gen.sample_qualities(r, seed + 3)
    q[::17] = ord("!")                         # some Q = 0 bases
    return seq, r, q


@pytest.mark.parametrize("F", [4096, 2048, 1024, 48])
def test_quality_scan_every_tile_shape(F):
    seq, r, q = _case()
    ref = oracle.scan(seq, F, r.seq, r.offsets, M, X, nthreads=8, quals=q, qscale=QS)
    ix = mx.Index(seq, F, 250, M, X, GAP, qual_scale=QS)
    for np_ in (8, 16, 32):
        if 128 * np_ > max(F, 1024):
            continue
        for R in (8, 32):
            mx.maxss_index_set_tiles(ix.handle, np_, R, 8)
            assert_same(ix.scan(r.seq, r.offsets, qual=q), ref, "F=%d NP=%d R=%d" % (F, np_, R))
    mx.maxss_index_set_tiles(ix.handle, 0, 0, 0)
    ix.close()


@pytest.mark.parametrize("mlen", [253, 300])
def test_quality_scan_score_bound_both_kernels(mlen):
    # match * qual_scale = 125: max_read_len 253 keeps the bound at 31625
    # (two-step kernels), 300 raises it to 37500 (per-step kernels)
    seq, r, q = _case(23)
    long_ = gen.sample_reads(gen.Genome(seq, "q"), 6, 29, [mlen], 0.0, 0.1)
    qs = gen.sample_qualities(long_, 31)
    reads = [r.read(i) for i in range(r.n)] + [long_.read(i) for i in range(long_.n)]
    quals = [q[int(r.offsets[i]):int(r.offsets[i + 1])] for i in range(r.n)] + \
        [qs[int(long_.offsets[i]):int(long_.offsets[i + 1])] for i in range(long_.n)]
    off = np.zeros(len(reads) + 1, np.uint64)
    off[1:] = np.cumsum([len(x) for x in reads])
    rs = np.frombuffer(b"".join(reads), np.uint8)
    qq = np.concatenate(quals)
    ref = oracle.scan(seq, 2048, rs, off, 5, -4, nthreads=8, quals=qq, qscale=25)
    ix = mx.Index(seq, 2048, mlen, 5, -4, GAP, qual_scale=25)
    assert_same(ix.scan(rs, off, qual=qq), ref, "max_read_len %d" % mlen)
    ix.close()


def test_quality_device_reads_and_invalid_quality():
    torch = _torch()
    seq, r, q = _case(17)
    q = q.copy()
    a = int(r.offsets[3])
    q[a + 1] = ord(" ")                        # read 3: a quality outside '!'..'~'
    ok = np.ones(r.n, bool)
    ok[3] = False
    keep = np.nonzero(ok)[0]
    sub = r.subset(keep)
    qs = np.concatenate([q[int(r.offsets[i]):int(r.offsets[i + 1])] for i in keep])
    ref = oracle.scan(seq, 2048, sub.seq, sub.offsets, M, X, nthreads=8, quals=qs, qscale=QS)
    ix = mx.Index(seq, 2048, 250, M, X, GAP, qual_scale=QS)
    s = torch.from_numpy(np.array(r.seq)).cuda()
    o = torch.from_numpy(r.offsets.astype(np.int64)).cuda()
    qd = torch.from_numpy(q).cuda()
    out = torch.zeros(r.n * 32, dtype=torch.uint8, device="cuda")
    ix.scan(s, o, out, qual=qd)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(mx.TOP2_DTYPE)
    assert got["frag"][3][0] == mx.MAXSS_READ_INVALID
    assert_same(got[keep], ref, "device reads")
    ix.close()


def test_quality_fast_and_one_strand():
    seq, r, q = _case(27)
    for flags, oflags in [(mx.MAXSS_FAST, oracle.FAST),
                          (mx.MAXSS_ONE_STRAND, oracle.ONE_STRAND),
                          (mx.MAXSS_FAST | mx.MAXSS_ONE_STRAND, oracle.FAST | oracle.ONE_STRAND)]:
        ref = oracle.scan(seq, 2048, r.seq, r.offsets, M, X, flags=oflags, nthreads=8, quals=q,
                          qscale=QS)
        ix = mx.Index(seq, 2048, 250, M, X, GAP, flags=flags, qual_scale=QS)
        assert_same(ix.scan(r.seq, r.offsets, qual=q), ref, "flags %d" % flags)
        ix.close()


@pytest.mark.parametrize("glob", [False, True])
def test_quality_nw_matches_oracle(glob):
    seq, r, q = _case(37)
    flags = mx.MAXSS_NW_GLOBAL if glob else 0
    ix = mx.Index(seq, 1024, 250, M, X, GAP, flags=flags, qual_scale=QS)
    top = ix.scan(r.seq, r.offsets, qual=q)
    ref = oracle.scan(seq, 1024, r.seq, r.offsets, M, X, nthreads=8, quals=q, qscale=QS)
    assert_same(top, ref, "scan")
    aln, cig = ix.align(r.seq, r.offsets, top, 60, 2048, qual=q)
    exp = oracle.align_top(seq, 1024, r.seq, r.offsets, ref, 60, M, X, GAP,
                           oracle.NW_GLOBAL if glob else oracle.NW_FIT, quals=q, qscale=QS)
    for i in range(r.n):
        assert (int(aln["score"][i]), int(aln["strand"][i]), int(aln["ref_begin"][i]),
                int(aln["ref_end"][i]), cig[i]) == \
            (exp[i]["score"], exp[i]["strand"], exp[i]["ref_begin"], exp[i]["ref_end"],
             exp[i]["cigar"]), i
    ix.close()


def test_quality_plan_graph():
    torch = _torch()
    seq, r, q = _case(47)
    ref = oracle.scan(seq, 2048, r.seq, r.offsets, M, X, nthreads=8, quals=q, qscale=QS)
    ix = mx.Index(seq, 2048, 250, M, X, GAP, qual_scale=QS)
    plan = mx.Plan(ix, capacity=r.n, pad=50, cigar_stride=512)
    s = torch.from_numpy(np.array(r.seq)).cuda()
    o = torch.from_numpy(r.offsets.astype(np.int64)).cuda()
    qd = torch.from_numpy(q).cuda()
    top = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda")
    aln = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda")
    cig = torch.zeros(r.n * 512, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(stream):
            plan.run(s, o, top, aln, cig, stream=stream, graph=True, qual=qd)
        stream.synchronize()
        assert_same(top.cpu().numpy().view(mx.TOP2_DTYPE), ref, "graph replay %d" % rep)
    exp = oracle.align_top(seq, 2048, r.seq, r.offsets, ref, 50, M, X, GAP, quals=q, qscale=QS)
    a = aln.cpu().numpy().view(mx.ALN_DTYPE)
    assert [int(x) for x in a["score"]] == [e["score"] for e in exp]
    # the same reads with qualities in another buffer: the graph is recorded
    # again for the new buffer, not replayed with the old one
    q2 = gen.sample_qualities(r, 4747)
    ref2 = oracle.scan(seq, 2048, r.seq, r.offsets, M, X, nthreads=8, quals=q2, qscale=QS)
    assert any((ref2[f] != ref[f]).any() for f in FIELDS)
    qd2 = torch.from_numpy(q2).cuda()
    for rep in range(2):
        with torch.cuda.stream(stream):
            plan.run(s, o, top, aln, cig, stream=stream, graph=True, qual=qd2)
        stream.synchronize()
        assert_same(top.cpu().numpy().view(mx.TOP2_DTYPE), ref2, "new qualities %d" % rep)
    plan.close()
    ix.close()


def test_quality_index_needs_qualities():
    seq, r, q = _case(57)
    ix = mx.Index(seq, 2048, 250, M, X, GAP, qual_scale=QS)
    with pytest.raises(mx.MaxssError) as e:
        ix.scan(r.seq, r.offsets)
    assert e.value.status == mx.MAXSS_EINVAL
    bad = q.copy()
    bad[5] = 0x7F
    with pytest.raises(mx.MaxssError) as e:
        ix.scan(r.seq, r.offsets, qual=bad)
    assert e.value.status == mx.MAXSS_EINVAL
    ix.close()
    # plain indexes ignore qualities
    ix = mx.Index(seq, 2048, 250, M, X, GAP)
    assert_same(ix.scan(r.seq, r.offsets, qual=q),
                oracle.scan(seq, 2048, r.seq, r.offsets, M, X, nthreads=8), "plain")
    ix.close()


def test_quality_longest_reads():
    # max_read_len 7168 with qual_scale 9: the window and one read's codes and
    # position scores take about 74 KB of LDS (NP = 32), and the score bound
    # 64512 > 31744 selects the per-step-max kernel
    g = gen.uniform_genome(16_000, 61)
    parts = [gen.sample_reads(g, 1, 62 + i, [m], 0.0, 0.1) for i, m in enumerate((7168, 7001))]
    reads = [p.read(0) for p in parts]
    quals = [gen.sample_qualities(p, 70 + i) for i, p in enumerate(parts)]
    off = np.zeros(len(reads) + 1, np.uint64)
    off[1:] = np.cumsum([len(x) for x in reads])
    rs = np.frombuffer(b"".join(reads), np.uint8)
    qq = np.concatenate(quals)
    ref = oracle.scan(g.seq, 4096, rs, off, 1, -1, nthreads=8, quals=qq, qscale=9)
    ix = mx.Index(g.seq, 4096, 7168, 1, -1, -2, qual_scale=9)
    assert ix.kernel_info()[1] == mx.MAXSS_KERNEL_STEP_MAX
    assert_same(ix.scan(rs, off, qual=qq), ref, "7168-base reads")
    ix.close()


def _split_case(seed=101):
    """Reads of both launches of the quality split side by side in the same
    tiles: bases at Phred >= 20 (one score pair at scale 10), reads with one
    Phred-2 base or several Phred-0 bases (several pairs), reads entirely at
    Phred 2 or entirely at 0 (one pair, another than the common one), reads
    with N, lengths 1..250, a genome with N runs."""
    g = gen.with_n_runs(gen.uniform_genome(41_000, seed), seed + 1, 12, 1, 80)
    r = gen.sample_reads(g, 150, seed + 2, [1, 2, 17, 64, 100, 111, 250], 0.0, 0.3, indel_max=2)
    q = np.maximum(gen.sample_qualities(r, seed + 3), ord("!") + 20)
    st = gen.Stream(seed, "q.split")
    kind = st.integers(0, 5, r.n)
    pos = st.uniform(r.n)
    seq = r.seq.copy()
    for i in range(r.n):
        a, b = int(r.offsets[i]), int(r.offsets[i + 1])
        if kind[i] == 1:
            q[a + int(pos[i] * (b - a))] = ord("#")
        elif kind[i] == 2:
            q[a:b:7] = ord("!")
        elif kind[i] == 3:
            q[a:b] = ord("#")
        elif kind[i] == 4:
            q[a:b] = ord("!")
        if i % 9 == 0 and b - a > 4:
            seq[a + 2] = ord("N")
    reads = gen.Reads(seq, r.offsets, r.start, r.span, r.strand, r.rate, r.n_indel)
    return g.seq, reads, q


def _one_pair(r, q):
    """Reads whose bases all map to one (match, mismatch) pair (match 5,
    mismatch -4, scale 10: Phred >= 20 gives (50, -13), 2 gives (18, -5), 0
    gives (0, 0); the case holds no other Phred values)."""
    cls = np.minimum(q.astype(np.int64) - 33, 20)
    out = np.zeros(r.n, bool)
    for i in range(r.n):
        c = cls[int(r.offsets[i]):int(r.offsets[i + 1])]
        out[i] = c.size == 0 or (c == c[0]).all()
    return out


@pytest.mark.parametrize("F", [2048, 3072, 4096])
def test_quality_split_both_launches_every_shape(F):
    """The quality split (register banks for reads with one score pair, the
    position-specific kernel for the others) against the oracle, with
    forced tiles (NP = 16 splits; 8 and 32 do not) and the built-in ones."""
    seq, r, q = _split_case()
    one = _one_pair(r, q)
    assert 0.3 < one.mean() < 0.8
    ref = oracle.scan(seq, F, r.seq, r.offsets, M, X, nthreads=8, quals=q, qscale=QS)
    ix = mx.Index(seq, F, 250, M, X, GAP, qual_scale=QS)
    if F % 2048 == 0:
        assert tuple(ix.kernel_info()) == (16, mx.MAXSS_KERNEL_REGISTER_BANK)
    for np_, R in ((16, 8), (16, 32), (16, 1), (8, 16), (32, 16), (0, 0)):
        if 128 * np_ > F:
            continue
        mx.maxss_index_set_tiles(ix.handle, np_, R, 8)
        assert_same(ix.scan(r.seq, r.offsets, qual=q), ref, "F=%d NP=%d R=%d" % (F, np_, R))
    mx.maxss_index_set_tiles(ix.handle, 0, 0, 0)
    ix.close()


def test_quality_split_flags_device_reads_and_graph():
    """The split with the fast scan, one strand and the neighbour exclusion;
    device reads through a plan replayed from its graph; second phase."""
    torch = _torch()
    seq, r, q = _split_case(131)
    for flags, oflags in [(mx.MAXSS_FAST, oracle.FAST), (mx.MAXSS_ONE_STRAND, oracle.ONE_STRAND),
                          (mx.MAXSS_EXCLUDE_ADJACENT, oracle.EXCL_ADJ)]:
        ref = oracle.scan(seq, 2048, r.seq, r.offsets, M, X, flags=oflags, nthreads=8, quals=q,
                          qscale=QS)
        ix = mx.Index(seq, 2048, 250, M, X, GAP, flags=flags, qual_scale=QS)
        assert_same(ix.scan(r.seq, r.offsets, qual=q), ref, "flags %d" % flags)
        ix.close()
    ref = oracle.scan(seq, 2048, r.seq, r.offsets, M, X, nthreads=8, quals=q, qscale=QS)
    ix = mx.Index(seq, 2048, 250, M, X, GAP, qual_scale=QS)
    plan = mx.Plan(ix, capacity=r.n, pad=50, cigar_stride=512)
    s = torch.from_numpy(np.array(r.seq)).cuda()
    o = torch.from_numpy(r.offsets.astype(np.int64)).cuda()
    qd = torch.from_numpy(q).cuda()
    top = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda")
    aln = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda")
    cig = torch.zeros(r.n * 512, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(stream):
            plan.run(s, o, top, aln, cig, stream=stream, graph=True, qual=qd)
        stream.synchronize()
        assert_same(top.cpu().numpy().view(mx.TOP2_DTYPE), ref, "graph replay %d" % rep)
    exp = oracle.align_top(seq, 2048, r.seq, r.offsets, ref, 50, M, X, GAP, quals=q, qscale=QS)
    a = aln.cpu().numpy().view(mx.ALN_DTYPE)
    assert [int(x) for x in a["score"]] == [e["score"] for e in exp]
    plan.close()
    ix.close()


def test_quality_split_candidate_scan():
    """The proposal's candidate scan on a quality index (both launches, one
    read per tile): a read that keeps its candidates carries the exact top-2
    among them, a read that falls back the full scan's record."""
    torch = _torch()
    from oracle import mlp
    seq, r, q = _split_case(151)
    ix = mx.Index(seq, 2048, 250, M, X, GAP, qual_scale=QS)
    m = mx.Model(gen.mlp_init(9))
    K = 4
    s = torch.from_numpy(np.array(r.seq)).cuda()
    o = torch.from_numpy(r.offsets.astype(np.int64)).cuda()
    qd = torch.from_numpy(q).cuda()
    out = torch.zeros(r.n * 32, dtype=torch.uint8, device="cuda")
    fb = torch.zeros(r.n, dtype=torch.uint8, device="cuda")
    cand = torch.zeros(r.n * K, dtype=torch.int32, device="cuda")
    mg = torch.zeros(r.n, dtype=torch.float32, device="cuda")
    fb2 = torch.zeros(r.n, dtype=torch.uint8, device="cuda")
    m.candidates(ix, s, o, K, 0.0, cand, mg, fb2)
    torch.cuda.synchronize()
    tau = float(np.median(mg.cpu().numpy()))
    m.scan(ix, s, o, K, tau, out, fb, qual=qd)
    m.candidates(ix, s, o, K, tau, cand, mg, fb2)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(mx.TOP2_DTYPE)
    fb, cand = fb.cpu().numpy(), cand.cpu().numpy().reshape(r.n, K)
    assert 0 < fb.sum() < r.n
    full, vals = oracle.scan(seq, 2048, r.seq, r.offsets, M, X, nthreads=8, want_values=True,
                             quals=q, qscale=QS)
    lens = np.diff(r.offsets.astype(np.int64))
    for i in range(r.n):
        if fb[i]:
            for f in FIELDS:
                assert (got[f][i] == full[f][i]).all(), i
            continue
        f1, s1, f2, s2 = mlp.top2_among(vals[i], cand[i])
        assert got["frag"][i].tolist() == [f1, f2] and got["score"][i].tolist() == [s1, s2], \
            (i, int(lens[i]))
    m.close()
    ix.close()


def test_quality_full_size_sampled():
    """The bench's quality leg at full size: the 100,000 bacterial reads with
    their synthetic qualities at qual_scale 10 (98% of them on the
    register-bank launch of the split), device reads in one call; 40 sampled
    reads against the oracle, including every sampled read whose bases carry
    more than one score pair."""
    torch = _torch()
    w = gen.workload("bacterial")
    q = gen.sample_qualities(w.reads, 91)
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap, qual_scale=10)
    s = torch.from_numpy(np.array(w.reads.seq)).cuda()
    o = torch.from_numpy(w.reads.offsets.astype(np.int64)).cuda()
    out = torch.zeros(w.reads.n * 32, dtype=torch.uint8, device="cuda")
    ix.scan(s, o, out, qual=torch.from_numpy(q).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(mx.TOP2_DTYPE)
    ix.close()
    # the sample: 30 drawn reads plus 10 reads whose bases carry more than one
    # (match, mismatch) pair (the score table's rule, halves rounded away
    # from zero; Phred >= 14 gives (10, -3))
    x = 1.0 - 10.0 ** (-(q.astype(np.float64) - 33) / 10.0)
    rnd = lambda v: np.sign(v) * np.floor(np.abs(v) + 0.5)
    pair = rnd(w.M * x * 10) * 256 + rnd(w.X * x * 10 / 3.0)
    starts = w.reads.offsets[:-1].astype(np.int64)
    first = np.repeat(pair[starts], w.reads.lengths().astype(np.int64))
    mixed = np.nonzero(np.add.reduceat((pair != first).astype(np.int64), starts) > 0)[0]
    assert mixed.size > 100
    st = gen.Stream(79, "qual.sample")
    idx = np.unique(np.concatenate([st.integers(0, w.reads.n, 30),
                                    mixed[st.integers(0, mixed.size, 10)]]))
    sub = w.reads.subset(idx)
    qs = np.concatenate([q[int(w.reads.offsets[i]):int(w.reads.offsets[i + 1])] for i in idx])
    ref = oracle.scan(w.genome.seq, w.F, sub.seq, sub.offsets, w.M, w.X, nthreads=16, quals=qs,
                      qscale=10)
    assert_same(got[idx], ref, "bacterial quality sample")
    assert (got["frag"][:, 0] != got["frag"][:, 1]).all()
