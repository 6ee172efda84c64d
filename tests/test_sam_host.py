"""The library's SAM formatting (host code) against the oracle's, on records
the oracle computed: the hand-derived toy records, and reads with ties,
reverse strands, unmapped and invalid reads, custom names, qualities and
the strict threshold.  The device MAPQ kernel is checked in the GPU tests."""
import json
import os

import numpy as np
import pytest

import gen
import oracle
from oracle import sam
import paper_1403_2136_amd as mx

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _records(genome, F, reads, pad, stride=256):
    """Oracle top-2 and NW results in the library's record layouts."""
    seq = b"".join(reads)
    off = np.cumsum([0] + [len(r) for r in reads]).astype(np.uint64)
    top = oracle.scan(genome, F, seq, off)
    alns = oracle.align_top(genome, F, seq, off, top, pad)
    aln = np.zeros(len(reads), dtype=mx.ALN_DTYPE)
    cig = np.zeros(len(reads) * stride, dtype=np.uint8)
    for i, a in enumerate(alns):
        aln[i]["score"], aln[i]["strand"] = a["score"], a["strand"]
        aln[i]["ref_begin"], aln[i]["ref_end"] = a["ref_begin"], a["ref_end"]
        c = a["cigar"].encode()
        if len(c) >= stride:
            aln[i]["flags"] = 1
        else:
            cig[i * stride:i * stride + len(c)] = np.frombuffer(c, dtype=np.uint8)
        aln[i]["cigar_len"] = len(c)
    return seq, off, top, alns, aln, cig


def _mapq(top, num=9, den=10, min_q=-1):
    s1 = top["score"][:, 0].astype(int)
    s2 = np.where(top["frag"][:, 1] >= 0, top["score"][:, 1], -1).astype(int)
    q = np.array([sam.mapq(a, b) if f >= 0 else 0 for a, b, f in zip(s1, s2, top["frag"][:, 0])],
                 dtype=np.uint8)
    m = np.array([sam.is_mapped(a, b, num, den, min_q) if f >= 0 else False
                  for a, b, f in zip(s1, s2, top["frag"][:, 0])], dtype=np.uint8)
    return q, m


def test_toy_records_equal_golden():
    g = json.load(open(os.path.join(GOLD, "sam_toy.json")))
    reads = [r.encode() for r in g["reads"]]
    seq, off, top, alns, aln, cig = _records(g["genome"].encode(), g["F"], reads, g["pad"])
    q, m = _mapq(top)
    txt = mx.maxss_sam_records(seq, off, top, aln, cig, 256, q, m, g["rname"], names=g["names"])
    assert txt == "".join(g["records"])


@pytest.mark.parametrize("min_q", [-1, 62])
def test_mixed_reads_equal_oracle_text(min_q):
    G = gen.uniform_genome(30_000, 21)
    s = G.seq.copy()
    s[20_000:21_000] = s[3_000:4_000]             # exact repeat: unmapped reads
    G = gen.Genome(s, "rep")
    r = gen.sample_reads(G, 60, 22, [30, 75, 120], 0.0, 0.25, indel_max=1)
    reads = [r.read(i) for i in range(r.n)] + [b"acgtnacgtacgtaacg"]
    seq, off, top, alns, aln, cig = _records(G.seq, 2048, reads, 50, stride=32)
    q, m = _mapq(top, min_q=min_q)
    names = ["read:%d/x" % i for i in range(len(reads))]
    txt = mx.maxss_sam_records(seq, off, top, aln, cig, 32, q, m, "chrT", names=names)
    exp = "".join(sam.record(names[i], reads[i], top[i], alns[i], "chrT", min_mapq=min_q,
                             truncated=bool(aln[i]["flags"] & 1)) for i in range(len(reads)))
    assert txt == exp
    assert m.sum() > 0 and (m == 0).sum() > 0 and (top["strand"][:, 0] == 1).any()


def test_invalid_read_and_default_names():
    top = np.zeros(2, dtype=mx.TOP2_DTYPE)
    top["frag"][0] = [-2, -1]
    top["frag"][1] = [3, -1]
    top["score"][1] = [5, -1]
    aln = np.zeros(2, dtype=mx.ALN_DTYPE)
    aln["ref_begin"][1] = 99
    cig = np.zeros(2 * 8, dtype=np.uint8)
    cig[8:11] = np.frombuffer(b"5=\x00", dtype=np.uint8)
    txt = mx.maxss_sam_records(b"AXGTTacgta", [0, 4, 10], top, aln, cig, 8,
                               np.array([0, 254], np.uint8), np.array([0, 1], np.uint8), "c")
    assert txt == ("r0\t4\t*\t0\t0\t*\t*\t0\t0\t*\t*\n"
                   "r1\t0\tc\t100\t254\t5=\t*\t0\t0\tTACGTA\t*\tAS:i:0\n")


def test_bad_names_rejected():
    top = np.zeros(1, dtype=mx.TOP2_DTYPE)
    aln = np.zeros(1, dtype=mx.ALN_DTYPE)
    cig = np.zeros(8, dtype=np.uint8)
    z = np.zeros(1, np.uint8)
    with pytest.raises(mx.MaxssError):
        mx.maxss_sam_records(b"ACGT", [0, 4], top, aln, cig, 8, z, z, "has space")
    with pytest.raises(mx.MaxssError):
        mx.maxss_sam_records(b"ACGT", [0, 4], top, aln, cig, 8, z, z, "c", names=["a\tb"])


def test_qualities_in_qual_column_equal_oracle():
    G = gen.uniform_genome(30_000, 31)
    s = G.seq.copy()
    s[20_000:21_000] = s[3_000:4_000]             # exact repeat: unmapped reads
    G = gen.Genome(s, "rep")
    r = gen.sample_reads(G, 50, 32, [30, 75, 120], 0.0, 0.4, indel_max=1)
    reads = [r.read(i) for i in range(r.n)]
    q = gen.sample_qualities(r, 33)
    seq, off, top, alns, aln, cig = _records(G.seq, 2048, reads, 50)
    mq, m = _mapq(top)
    txt = mx.maxss_sam_records(seq, off, top, aln, cig, 256, mq, m, "chrQ", qual=q)
    exp = "".join(sam.record("r%d" % i, reads[i], top[i], alns[i], "chrQ",
                             truncated=bool(aln[i]["flags"] & 1),
                             qual=q[int(off[i]):int(off[i + 1])].tobytes())
                  for i in range(len(reads)))
    assert txt == exp
    assert m.sum() > 0 and (m == 0).sum() > 0 and (top["strand"][:, 0] == 1).any()
    bad = q.copy()
    bad[7] = 0x20                                 # a space is no Phred+33 quality
    with pytest.raises(mx.MaxssError):
        mx.maxss_sam_records(seq, off, top, aln, cig, 256, mq, m, "chrQ", qual=bad)
