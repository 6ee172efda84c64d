"""Oracle pins of the adjacent-fragment exclusion of the second-best fragment
(the Introduction and the first phase keep the best and second-best
fragment; a read that also scores in a neighbour of its best fragment is at
the same locus, so that neighbour is an option to leave out): a hand-derived
genome whose fragment values are closed forms, and a numpy restatement of the
rule over the oracle's value matrix."""
import numpy as np

import gen
import oracle

F = 64


def _planted():
    """N genome with a random 40 bp read planted whole in fragment 5, its
    first 30 bases in fragment 6 and its first 20 in fragment 10: an exact
    run of k bases between N scores k (N mismatches everything)."""
    rng = np.random.default_rng(5)
    read = bytes(rng.choice(list(b"ACGT"), 40).astype(np.uint8))
    g = bytearray(b"N" * (16 * F))
    g[5 * F + 10:5 * F + 50] = read
    g[6 * F + 16:6 * F + 46] = read[:30]
    g[10 * F + 10:10 * F + 30] = read[:20]
    return bytes(g), read


def test_planted_values_and_exclusion():
    g, read = _planted()
    off = np.array([0, len(read)], np.uint64)
    plain, vals = oracle.scan(g, F, read, off, want_values=True)
    assert vals[0, 5] == 40 and vals[0, 6] == 30 and vals[0, 10] == 20
    assert (np.delete(vals[0], [5, 6, 10]) < 20).all()
    assert list(plain[0]["frag"]) == [5, 6] and list(plain[0]["score"]) == [40, 30]
    ex = oracle.scan(g, F, read, off, flags=oracle.EXCL_ADJ)[0]
    assert list(ex["frag"]) == [5, 10] and list(ex["score"]) == [40, 20]
    assert list(ex["offset"]) == [10, 10] and list(ex["strand"]) == [0, 0]


def test_best_at_either_end_of_the_genome():
    g, read = _planted()
    # best in fragment 0 (only fragment 1 is its neighbour) and in the last one
    for f_best in (0, 15):
        gg = bytearray(b"N" * (16 * F))
        gg[f_best * F + 5:f_best * F + 45] = read
        nb = 1 if f_best == 0 else 14
        gg[nb * F + 3:nb * F + 33] = read[:30]
        gg[8 * F + 3:8 * F + 23] = read[:20]
        off = np.array([0, len(read)], np.uint64)
        plain = oracle.scan(bytes(gg), F, read, off)[0]
        ex = oracle.scan(bytes(gg), F, read, off, flags=oracle.EXCL_ADJ)[0]
        assert list(plain["frag"]) == [f_best, nb]
        assert list(ex["frag"]) == [f_best, 8] and list(ex["score"]) == [40, 20]


def test_three_fragments_leave_no_second():
    g, read = _planted()
    gg = g[4 * F:7 * F]                      # fragments 4, 5, 6 become 0, 1, 2
    off = np.array([0, len(read)], np.uint64)
    ex = oracle.scan(gg, F, read, off, flags=oracle.EXCL_ADJ)[0]
    assert ex["frag"][0] == 1 and ex["score"][0] == 40
    assert (ex["frag"][1], ex["score"][1], ex["offset"][1], ex["strand"][1]) == (-1, -1, -1, -1)


def test_rule_restated_over_the_value_matrix():
    G = gen.uniform_genome(30_000, 61)
    s = G.seq.copy()
    s[12_000:13_000] = s[3_000:4_000]
    G = gen.Genome(s, "rep")
    r = gen.sample_reads(G, 80, 62, [40, 90, 150], 0.0, 0.3, indel_max=2)
    plain, vals = oracle.scan(G.seq, 512, r.seq, r.offsets, nthreads=4, want_values=True)
    ex = oracle.scan(G.seq, 512, r.seq, r.offsets, flags=oracle.EXCL_ADJ, nthreads=4)
    NF = vals.shape[1]
    adjacent = 0
    for i in range(r.n):
        v = vals[i].astype(np.int64)
        f1 = int(np.argmax(v))               # first maximum: smallest id on ties
        assert ex[i]["frag"][0] == f1 == plain[i]["frag"][0]
        keep = [f for f in range(NF) if abs(f - f1) > 1]
        f2 = keep[int(np.argmax(v[keep]))] if keep else -1
        assert ex[i]["frag"][1] == f2 and ex[i]["score"][1] == (v[f2] if keep else -1)
        if abs(int(plain[i]["frag"][1]) - f1) == 1:
            adjacent += 1
        else:                                # the rule changes nothing else
            assert ex[i].tobytes() == plain[i].tobytes()
    assert adjacent > 0
