"""The stored records of the full-size workloads' sampled reads.

tests/golden/make_fullsize_records.py writes them with the oracle on genome
slices (a fragment's value depends only on its extended window) and takes
each winner's representative from an oracle scan of that window alone.  Here
that method is checked against the plain whole-genome oracle on a smaller
genome of the same kind, and the stored file against its own invariants."""
import importlib.util
import json
import os

import numpy as np
import pytest

import gen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
FIELDS = ("frag", "score", "offset", "strand")


def _script():
    spec = importlib.util.spec_from_file_location(
        "make_fullsize_records", os.path.join(HERE, "golden", "make_fullsize_records.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_sliced_records_equal_whole_genome_oracle():
    S = _script()
    g = gen.chromosome_genome(33, G=2_000_000, families=12)
    r = gen.sample_reads(g, 10, 35, [36, 51, 100, 150, 250], 0.1, 0.3, indel_max=2)
    seq = g.seq.copy()
    # an exact copy across a fragment junction: ties between fragments
    seq[4096 * 200 - 120:4096 * 200 + 180] = seq[10_000:10_300]
    g2 = gen.Genome(seq, "tie", g.info)
    reads = [seq[10_000:10_250].tobytes(), seq[4096 * 200 - 120:4096 * 200 - 20].tobytes()]
    reads += [r.read(i) for i in range(r.n)]
    off = np.zeros(len(reads) + 1, np.uint64)
    off[1:] = np.cumsum([len(x) for x in reads])
    rr = gen.Reads(np.frombuffer(b"".join(reads), np.uint8).copy(), off,
                   np.zeros(len(reads), np.int64), np.zeros(len(reads), np.int64),
                   np.zeros(len(reads), np.int8), np.zeros(len(reads)), np.zeros(len(reads), np.int8))
    w = gen.Workload("small", g2, rr, F=4096, max_read_len=250)
    got = S.records(w, np.arange(rr.n), nslices=7)
    ref = oracle.scan(seq, 4096, rr.seq, rr.offsets, nthreads=8)
    for i in range(rr.n):
        for f in FIELDS:
            assert list(got[i][f]) == ref[f][i].tolist(), (i, f, got[i], ref[i])


def test_repeat_overlap_flags():
    S = _script()
    g = gen.chromosome_genome(41, G=400_000, families=3, repeat_frac=0.2)
    r = gen.sample_reads(g, 300, 42, [100], 0.1, 0.1)
    flag = S.in_repeat(g, r)
    placed = g.info["placed"]
    for i in range(r.n):
        a, b = int(r.start[i]), int(r.start[i] + r.span[i])
        want = any(p < b and p + L > a for p, L, _, _ in placed)
        assert bool(flag[i]) == want, i


@pytest.mark.parametrize("name,n_min", [("chromosome", 50), ("damaged", 24)])
def test_stored_records_invariants(name, n_min):
    d = json.load(open(os.path.join(HERE, "golden", "fullsize_records.json")))[name]
    recs = d["records"]
    assert len(recs) == len(d["index"]) >= n_min
    assert sum(d["from_repeat_copy"]) >= n_min // 4
    assert d["index"] == sorted(set(d["index"]))
    NF = (d["G"] + d["F"] - 1) // d["F"]
    for rec in recs:
        s1, s2 = rec["score"]
        f1, f2 = rec["frag"]
        assert s1 >= s2 >= 0 and 0 <= f1 < NF and 0 <= f2 < NF and f1 != f2
        assert s1 > s2 or f1 < f2
        assert all(0 <= o < d["F"] for o in rec["offset"]) and set(rec["strand"]) <= {0, 1}
