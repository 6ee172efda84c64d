"""The register-bank scan kernel (16 offset pairs per lane) on fragment
lengths that are not a multiple of its 2,048-offset segment, so that the
last segment of every fragment is partly masked (F = 3072, 2064) or every
segment is (F = 1024, 48).  The kernel is forced with maxss_index_set_tiles,
as the autotuner may pick it, and every record is compared with the oracle:
plain scores, MaxSSmap_fast, one strand and the neighbour exclusion, over
several tile shapes (Methods, "First phase of MaxSSmap"; Figure 1)."""
import numpy as np
import pytest

import gen
import oracle
import paper_1403_2136_amd as mx

pytestmark = pytest.mark.gpu
FIELDS = ("frag", "score", "offset", "strand")

# library flag -> oracle flag
FLAGS = {
    "plain": (0, 0),
    "fast": (mx.MAXSS_FAST, oracle.FAST),
    "one-strand": (mx.MAXSS_ONE_STRAND, oracle.ONE_STRAND),
    "exclude-adjacent": (mx.MAXSS_EXCLUDE_ADJACENT, oracle.EXCL_ADJ),
}


def assert_same(got, ref, what=""):
    for f in FIELDS:
        bad = np.nonzero((got[f] != ref[f]).any(axis=1))[0]
        assert bad.size == 0, "%s: %s differs for %d reads, first %d: gpu %s oracle %s" % (
            what, f, bad.size, bad[0], got[bad[0]], ref[bad[0]])


def _case(seed):
    """N runs, exact repeats (ties), reads of 1 to 300 bases, reads at the
    genome end and across fragment junctions."""
    g = gen.with_n_runs(gen.uniform_genome(31_111, seed), seed + 1, 12, 1, 80)
    seq = g.seq.copy()
    seq[20000:20300] = seq[2000:2300]
    seq[9000:9300] = seq[2000:2300]
    reads = [seq[2000:2000 + m].tobytes() for m in (1, 7, 64, 100, 129, 300)]
    reads.append(seq[31_111 - 50:].tobytes())
    for p in (3072 - 40, 2064 - 30, 6144 - 70):
        reads.append(seq[p:p + 100].tobytes())
    r = gen.sample_reads(gen.Genome(seq, "bank"), 30, seed + 2, [17, 48, 111, 250, 300], 0.0,
                         0.3, indel_max=2)
    reads += [r.read(i) for i in range(r.n)]
    off = np.zeros(len(reads) + 1, np.uint64)
    off[1:] = np.cumsum([len(x) for x in reads])
    return seq, b"".join(reads), off


@pytest.mark.parametrize("F", [3072, 2064, 1024, 48])
@pytest.mark.parametrize("mode", list(FLAGS))
def test_register_bank_partial_segments(F, mode):
    seq, reads, off = _case(101)
    lf, of = FLAGS[mode]
    ref = oracle.scan(seq, F, reads, off, flags=of, nthreads=8)
    ix = mx.Index(seq, F, 300, flags=lf)
    for R in (1, 8, 32):
        for rounds in (1, 8):
            ix.set_tiles(16, R, rounds)
            assert ix.kernel_info() == (16, mx.MAXSS_KERNEL_REGISTER_BANK)
            got = ix.scan(reads, off)
            assert_same(got, ref, "%s F=%d NP=16 R=%d rounds=%d" % (mode, F, R, rounds))
    ix.close()


def test_autotune_with_partial_segments_is_exact():
    """F = 3072: the autotuner times the register-bank shapes beside the
    built-in 8-pair kernel and keeps only byte-identical ones."""
    seq, reads, off = _case(111)
    ref = oracle.scan(seq, 3072, reads, off, nthreads=8)
    ix = mx.Index(seq, 3072, 300)
    res = ix.autotune(reads, off)
    assert res["rejected"] == 0, res
    assert_same(ix.scan(reads, off), ref, "after autotune %s" % res)
    ix.close()
