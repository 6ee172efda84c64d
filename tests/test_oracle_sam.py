"""Pins of the mapping-quality and SAM oracle: closed forms of the MAPQ
formula at powers of two, the paper's 0.9 ratio rule and its printed
threshold, the strict threshold of 62, invariants, and hand-derived SAM
records for the paper's toy genome."""
import json
import math
import os

import numpy as np

import gen
import oracle
from oracle import sam

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_mapq_closed_forms_at_powers_of_two():
    # -100 log2(2^-k) = 100 k exactly
    assert sam.mapq(8, 4) == 100
    assert sam.mapq(8, 2) == 200
    assert sam.mapq(64, 1) == 254          # 600, capped
    assert sam.mapq(7, 7) == 0
    assert sam.mapq(5, 0) == 254 and sam.mapq(5, -1) == 254
    assert sam.mapq(0, 0) == 0 and not sam.is_mapped(0, 0)


def test_ratio_rule_and_printed_threshold():
    g = json.load(open(os.path.join(GOLD, "closed_forms.json")))["mapq_threshold"]
    # the printed threshold is the MAPQ of the cutoff ratio to one decimal
    q = -100.0 * math.log(g["ratio"]) / math.log(2.0)
    assert round(q, g["printed_decimals"]) == g["printed"]
    # a read is mapped exactly when second/best < 0.9
    assert not sam.is_mapped(10, 9) and not sam.is_mapped(100, 90)
    assert sam.is_mapped(100, 89) and sam.is_mapped(1000, 899)
    assert sam.mapq(10, 9) == 15         # 15.2003..., integer part
    assert sam.mapq(100, 89) == 16       # 16.81...


def test_strict_threshold_boundary():
    t = json.load(open(os.path.join(GOLD, "closed_forms.json")))["strict_mapq"]["threshold"]
    # MAPQ > 62 as an integer means -100 log2(s2/s1) >= 63, i.e. s2/s1 <= 2^-0.63
    s1 = 1000
    cut = math.floor(s1 * math.exp(-0.63 * math.log(2.0)))
    assert sam.is_mapped(s1, cut, min_mapq=t)
    assert not sam.is_mapped(s1, cut + 1, min_mapq=t)


def test_mapq_nonincreasing_in_second_score():
    for s1 in (1, 7, 100, 250, 12160):
        q = [sam.mapq(s1, s2) for s2 in range(0, s1 + 1)]
        assert all(a >= b for a, b in zip(q, q[1:]))
        assert q[-1] == 0


def test_toy_genome_records_hand_derived():
    g = json.load(open(os.path.join(GOLD, "sam_toy.json")))
    genome = g["genome"].encode()
    reads = [r.encode() for r in g["reads"]]
    seq = b"".join(reads)
    off = np.cumsum([0] + [len(r) for r in reads]).astype(np.uint64)
    top = oracle.scan(genome, g["F"], seq, off)
    alns = oracle.align_top(genome, g["F"], seq, off, top, g["pad"])
    assert sam.header(g["rname"], len(genome)) == g["header"]
    for i, r in enumerate(reads):
        assert sam.record(g["names"][i], r, top[i], alns[i], g["rname"]) == g["records"][i]


def test_reverse_strand_record_shows_forward_sequence():
    G = gen.uniform_genome(20_000, 5)
    r = gen.sample_reads(G, 40, 6, [60], 0.0, 0.05)
    top = oracle.scan(G.seq, 2048, r.seq, r.offsets, nthreads=4)
    alns = oracle.align_top(G.seq, 2048, r.seq, r.offsets, top, 100)
    for i in range(r.n):
        line = sam.record("q", r.read(i), top[i], alns[i], "g").rstrip("\n").split("\t")
        if line[1] == "4":
            continue
        pos = int(line[3]) - 1
        seq = line[9]
        # an exact or near-exact read lies on the forward strand at POS
        ref = G.seq[pos:pos + len(seq)].tobytes().decode()
        same = sum(a == b for a, b in zip(seq, ref))
        assert same >= 0.9 * len(seq), (i, line)
        assert (line[1] == "16") == (int(alns[i]["strand"]) == 1)


def test_qual_column_follows_seq():
    """QUAL stays attached to its bases: on the reverse strand SEQ[j] is the
    complement of read base m-1-j, so QUAL[j] is that base's quality."""
    G = gen.uniform_genome(20_000, 15)
    r = gen.sample_reads(G, 40, 16, [45, 80], 0.0, 0.5)
    q = gen.sample_qualities(r, 17)
    top = oracle.scan(G.seq, 2048, r.seq, r.offsets, nthreads=4)
    alns = oracle.align_top(G.seq, 2048, r.seq, r.offsets, top, 100)
    comp = {"A": "T", "C": "G", "G": "C", "T": "A", "N": "N"}
    seen = set()
    for i in range(r.n):
        a, b = int(r.offsets[i]), int(r.offsets[i + 1])
        read, qi = r.read(i).decode().upper(), q[a:b].tobytes().decode()
        line = sam.record("q", r.read(i), top[i], alns[i], "g", qual=q[a:b].tobytes())
        f = line.rstrip("\n").split("\t")
        seq, qual = f[9], f[10]
        assert len(qual) == len(seq) == b - a
        seen.add(f[1])
        if f[1] == "16":
            m = len(read)
            for j in range(m):
                assert comp[seq[j]] == read[m - 1 - j] and qual[j] == qi[m - 1 - j], (i, j)
        else:
            assert seq == read and qual == qi, i
        # without qualities the column is "*"
        plain = sam.record("q", r.read(i), top[i], alns[i], "g")
        assert plain.rstrip("\n").split("\t")[10] == "*"
    assert {"0", "16"} <= seen
