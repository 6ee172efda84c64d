"""GPU parity of the second phase (NW on the best fragment) against the oracle:
score, strand, reference span and CIGAR string, exactly."""
import numpy as np
import pytest

import gen
import oracle
import paper_1403_2136_amd as mx

pytestmark = pytest.mark.gpu


def _check(ix, w_genome, F, seq, off, top, pad, M, X, gap, mode, stride=1024):
    aln, cig = ix.align(seq, off, top, pad, stride)
    sb = seq if isinstance(seq, bytes) else np.asarray(seq).tobytes()
    for i in range(len(off) - 1):
        r = sb[int(off[i]):int(off[i + 1])]
        o = oracle.align_one(w_genome, F, r, int(top["frag"][i][0]), int(top["strand"][i][0]),
                             pad, M, X, gap, mode)
        got = dict(score=int(aln["score"][i]), strand=int(aln["strand"][i]),
                   ref_begin=int(aln["ref_begin"][i]), ref_end=int(aln["ref_end"][i]),
                   cigar=cig[i])
        assert got == o, "read %d: gpu %s oracle %s" % (i, got, o)
        assert aln["flags"][i] == 0 and aln["cigar_len"][i] == len(cig[i])
    return aln, cig


def test_tiny_nw_fitting_all_reads():
    w = gen.workload("tiny")
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap)
    top = ix.scan(w.reads.seq, w.reads.offsets)
    _check(ix, w.genome.seq, w.F, w.reads.seq.tobytes(), w.reads.offsets, top, w.pad, w.M, w.X,
           w.gap, oracle.NW_FIT)
    ix.close()


def test_nw_with_indels_and_paper_scores():
    g = gen.uniform_genome(60_000, 41)
    r = gen.sample_reads(g, 60, 42, [36, 51, 100, 150], 0.1, 0.3, indel_max=2)
    ix = mx.Index(g.seq, 2048, 150, 5, -4, -26)
    top = ix.scan(r.seq, r.offsets)
    _check(ix, g.seq, 2048, r.seq.tobytes(), r.offsets, top, 100, 5, -4, -26, oracle.NW_FIT)
    ix.close()


def test_nw_global_mode():
    g = gen.uniform_genome(8000, 43)
    r = gen.sample_reads(g, 12, 44, [60], 0.1, 0.1, indel_max=1)
    ix = mx.Index(g.seq, 256, 60, 1, -1, -2, mx.MAXSS_NW_GLOBAL)
    top = ix.scan(r.seq, r.offsets)
    _check(ix, g.seq, 256, r.seq.tobytes(), r.offsets, top, 30, 1, -1, -2, oracle.NW_GLOBAL)
    ix.close()


def test_nw_region_clipped_at_both_ends_and_n():
    g = gen.with_n_runs(gen.uniform_genome(5000, 45), 46, 10, 1, 30)
    reads = [g.seq[0:70].tobytes(), g.seq[4930:5000].tobytes(), g.seq[2000:2070].tobytes(),
             b"N" * 20 + g.seq[3000:3050].tobytes()]
    off = np.zeros(5, np.uint64)
    off[1:] = np.cumsum([len(x) for x in reads])
    seq = b"".join(reads)
    ix = mx.Index(g.seq, 1024, 70)
    top = ix.scan(seq, off)
    _check(ix, g.seq, 1024, seq, off, top, 100, 1, -1, -2, oracle.NW_FIT)
    ix.close()


def test_nw_cigar_truncation_flag():
    g = gen.uniform_genome(8000, 47)
    r = gen.sample_reads(g, 4, 48, [100], 0.3, 0.3, indel_max=2)
    ix = mx.Index(g.seq, 512, 100)
    top = ix.scan(r.seq, r.offsets)
    aln, cig = ix.align(r.seq, r.offsets, top, 100, 8)
    ix.close()
    assert (aln["flags"] & mx.MAXSS_ALN_TRUNCATED).all()
    assert all(len(c) <= 7 for c in cig)


def _mixed_reads(g, n, seed, lengths, lo, hi, indels, random_reads=0, rseed=0):
    """Reads sampled from the genome plus reads of random bases (which align
    nowhere: low scores, the widest traceback windows)."""
    r = gen.sample_reads(g, n, seed, lengths, lo, hi, indel_max=indels)
    reads = [r.read(i) for i in range(r.n)]
    st = gen.Stream(rseed, "nw.random")
    for k in range(random_reads):
        m = int(lengths[k % len(lengths)])
        reads.append(gen.random_bases(st, m).tobytes())
    off = np.zeros(len(reads) + 1, np.uint64)
    off[1:] = np.cumsum([len(x) for x in reads])
    return b"".join(reads), off


@pytest.mark.parametrize("M,X,gap", [(1, -1, -2), (1, -1, -1), (2, -1, 0), (5, -4, -26)])
def test_nw_fitting_windows_of_every_width(M, X, gap):
    """Fitting mode through the two-pass kernel: 250 bp reads (traceback
    windows over one and several 256-column strips), reads of random bases,
    gap -1 (the window bound far from the end column) and gap 0 (no bound:
    the window is the whole region up to the end column)."""
    g = gen.with_n_runs(gen.uniform_genome(40_000, 51), 52, 6, 1, 40)
    seq, off = _mixed_reads(g, 24, 53, [36, 100, 250], 0.0, 0.3, 2, random_reads=9, rseed=54)
    ix = mx.Index(g.seq, 2048, 250, M, X, gap)
    top = ix.scan(seq, off)
    _check(ix, g.seq, 2048, seq, off, top, 100, M, X, gap, oracle.NW_FIT, stride=2048)
    ix.close()


def test_nw_fitting_ties_repeats_and_n():
    """Exact repeats inside one region (equal best end columns, the smallest
    wins), reads with N, reads at both genome ends."""
    g = gen.uniform_genome(12_000, 55)
    seq = g.seq.copy()
    seq[2300:2400] = seq[2000:2100]      # two copies in one NW region
    seq[2600:2700] = seq[2000:2100]
    reads = [seq[2000:2100].tobytes(), seq[2000:2050].tobytes() + b"NNNN" + seq[2054:2100].tobytes(),
             seq[0:80].tobytes(), seq[11_920:12_000].tobytes(), b"N" * 30,
             seq[5000:5100].tobytes()[::-1]]
    off = np.zeros(len(reads) + 1, np.uint64)
    off[1:] = np.cumsum([len(x) for x in reads])
    s = b"".join(reads)
    ix = mx.Index(seq, 1024, 100)
    top = ix.scan(s, off)
    _check(ix, seq, 1024, s, off, top, 100, 1, -1, -2, oracle.NW_FIT)
    ix.close()


def test_nw_fitting_quality_scores_two_pass():
    """Position-specific row scores at a small quality scale, which keeps the
    DP in 16 bits (the two-pass kernel): the window bound then sums each
    row's own match score."""
    g = gen.uniform_genome(30_000, 57)
    r = gen.sample_reads(g, 30, 58, [40, 100, 150], 0.05, 0.3, indel_max=2)
    q = gen.sample_qualities(r, 59)
    q[::13] = ord("!")
    ix = mx.Index(g.seq, 2048, 150, 5, -4, -26, qual_scale=2)
    top = ix.scan(r.seq, r.offsets, qual=q)
    aln, cig = ix.align(r.seq, r.offsets, top, 100, 1024, qual=q)
    sb = r.seq.tobytes()
    for i in range(r.n):
        a, b = int(r.offsets[i]), int(r.offsets[i + 1])
        o = oracle.align_one(g.seq, 2048, sb[a:b], int(top["frag"][i][0]), int(top["strand"][i][0]),
                             100, 5, -4, -26, oracle.NW_FIT, q[a:b].tobytes(), 2)
        got = dict(score=int(aln["score"][i]), strand=int(aln["strand"][i]),
                   ref_begin=int(aln["ref_begin"][i]), ref_end=int(aln["ref_end"][i]),
                   cigar=cig[i])
        assert got == o, "read %d: gpu %s oracle %s" % (i, got, o)
    ix.close()
