"""MaxSSmap_fast on the GPU (the first phase scores every other read base):
records bit-exact against the oracle's fast scan for every tile shape, both
strands and one, odd fragment lengths and the genome end, the plan and the
candidate scan, and NW on the fast winners."""
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
        assert bad.size == 0, "%s: %s differs for %d reads, first %d: gpu %s oracle %s" % (
            what, f, bad.size, bad[0], got[bad[0]], ref[bad[0]])


def _case(seed=11):
    g = gen.with_n_runs(gen.uniform_genome(23_457, seed), seed + 1, 12, 1, 80)
    seq = g.seq.copy()
    seq[15000:15300] = seq[2000:2300]          # exact repeats: ties
    seq[9000:9300] = seq[2000:2300]
    reads = [seq[2000:2000 + m].tobytes() for m in (1, 2, 3, 64, 129, 300)]
    reads.append(seq[23_457 - 40:].tobytes())   # the genome end
    r = gen.sample_reads(gen.Genome(seq, "fast"), 30, seed + 2, [17, 48, 111, 250, 300], 0.0,
                         0.3, indel_max=2)
    reads += [r.read(i) for i in range(r.n)]
    off = np.zeros(len(reads) + 1, np.uint64)
    off[1:] = np.cumsum([len(x) for x in reads])
    return seq, b"".join(reads), off


@pytest.mark.parametrize("F", [4096, 2048, 1024, 48])
def test_fast_scan_every_tile_shape(F):
    seq, reads, off = _case()
    ref = oracle.scan(seq, F, reads, off, flags=oracle.FAST, nthreads=8)
    ix = mx.Index(seq, F, 300, flags=mx.MAXSS_FAST)
    Fp = F // 2
    for np_ in (8, 16, 32):
        if 128 * np_ > max(Fp, 1024):
            continue
        for R in (8, 32):
            mx.maxss_index_set_tiles(ix.handle, np_, R, 8)
            assert_same(ix.scan(reads, off), ref, "F=%d NP=%d R=%d" % (F, np_, R))
    mx.maxss_index_set_tiles(ix.handle, 0, 0, 0)
    ix.close()


def test_fast_one_strand_and_paper_scores():
    seq, reads, off = _case(21)
    flags = oracle.FAST | oracle.ONE_STRAND
    ref = oracle.scan(seq, 2048, reads, off, 5, -4, flags=flags, nthreads=8)
    ix = mx.Index(seq, 2048, 300, 5, -4, -26, flags=mx.MAXSS_FAST | mx.MAXSS_ONE_STRAND)
    assert_same(ix.scan(reads, off), ref, "one strand, 5/-4")
    ix.close()


def test_fast_plan_and_nw():
    torch = _torch()
    seq, reads, off = _case(31)
    n = off.size - 1
    ref = oracle.scan(seq, 1024, reads, off, flags=oracle.FAST, nthreads=8)
    ix = mx.Index(seq, 1024, 300, flags=mx.MAXSS_FAST)
    plan = mx.Plan(ix, capacity=n, pad=60, cigar_stride=512)
    s = torch.from_numpy(np.frombuffer(reads, np.uint8).copy()).cuda()
    o = torch.from_numpy(off.astype(np.int64)).cuda()
    top = torch.empty(n * 32, dtype=torch.uint8, device="cuda")
    aln = torch.empty(n * 32, dtype=torch.uint8, device="cuda")
    cig = torch.zeros(n * 512, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.run(s, o, top, aln, cig, stream=stream, graph=True)
    stream.synchronize()
    assert_same(top.cpu().numpy().view(mx.TOP2_DTYPE), ref, "fast plan")
    exp = oracle.align_top(seq, 1024, reads, off, ref, 60)
    a = aln.cpu().numpy().view(mx.ALN_DTYPE)
    c = cig.cpu().numpy()
    for i in range(n):
        assert (int(a["score"][i]), int(a["strand"][i]), int(a["ref_begin"][i]),
                int(a["ref_end"][i]), mx.decode_cigar(c, i, 512)) == \
            (exp[i]["score"], exp[i]["strand"], exp[i]["ref_begin"], exp[i]["ref_end"],
             exp[i]["cigar"]), i
    plan.close()
    ix.close()


def test_fast_candidate_scan_exact_on_candidates():
    torch = _torch()
    from oracle import mlp
    seq, reads, off = _case(41)
    n = off.size - 1
    K = 4
    _, vals = oracle.scan(seq, 2048, reads, off, flags=oracle.FAST, nthreads=8,
                          want_values=True)
    ix = mx.Index(seq, 2048, 300, flags=mx.MAXSS_FAST)
    m = mx.Model(gen.mlp_init(3))
    s = torch.from_numpy(np.frombuffer(reads, np.uint8).copy()).cuda()
    o = torch.from_numpy(off.astype(np.int64)).cuda()
    cand = torch.zeros(n * K, dtype=torch.int32, device="cuda")
    mg = torch.zeros(n, dtype=torch.float32, device="cuda")
    fb = torch.zeros(n, dtype=torch.uint8, device="cuda")
    out = torch.zeros(n * 32, dtype=torch.uint8, device="cuda")
    m.candidates(ix, s, o, K, -1.0, cand, mg, fb)       # no read falls back
    m.scan(ix, s, o, K, -1.0, out, fb)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(mx.TOP2_DTYPE)
    cand = cand.cpu().numpy().reshape(n, K)
    assert not fb.cpu().numpy().any()
    for i in range(n):
        f1, s1, f2, s2 = mlp.top2_among(vals[i], cand[i])
        assert got["frag"][i].tolist() == [f1, f2] and got["score"][i].tolist() == [s1, s2], i
    m.close()
    ix.close()


def test_fast_full_size_sampled():
    """The bench's fast leg at full size: the 100,000 bacterial reads with
    MAXSS_FAST in one call; 40 sampled reads against the oracle's fast scan."""
    import torch
    assert torch.cuda.is_available()
    w = gen.workload("bacterial")
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap, flags=mx.MAXSS_FAST)
    s = torch.from_numpy(np.array(w.reads.seq)).cuda()
    o = torch.from_numpy(w.reads.offsets.astype(np.int64)).cuda()
    out = torch.zeros(w.reads.n * 32, dtype=torch.uint8, device="cuda")
    ix.scan(s, o, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(mx.TOP2_DTYPE)
    ix.close()
    idx = np.unique(gen.Stream(80, "fast.sample").integers(0, w.reads.n, 40))
    sub = w.reads.subset(idx)
    ref = oracle.scan(w.genome.seq, w.F, sub.seq, sub.offsets, w.M, w.X, flags=oracle.FAST,
                      nthreads=16)
    for f in ("frag", "score", "offset", "strand"):
        bad = np.nonzero((got[idx][f] != ref[f]).any(axis=1))[0]
        assert bad.size == 0, (f, idx[bad[:3]])
