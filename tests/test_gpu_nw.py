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
