"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each check uses a different
method (brute force over all subsequences or all alignments), a value the
paper prints for its worked example, a closed form, or an invariant that a
plausible slip in the oracle (dropped term, wrong sign, off-by-one offset,
swapped operands, wrong tie rule) would break.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def brute_maxss(x):
    """Maximum over all contiguous runs (and the empty run) by enumeration."""
    best = 0
    for i in range(len(x)):
        s = 0
        for j in range(i, len(x)):
            s += int(x[j])
            best = max(best, s)
    return best


def brute_window(read, genome, p, M, X):
    """Score of the window at p by enumerating every subsequence of the
    substitution scores (N or past-the-end is a mismatch)."""
    x = []
    for k, c in enumerate(read):
        g = genome[p + k] if p + k < len(genome) else "N"
        x.append(M if (c == g and c != "N") else X)
    return brute_maxss(x)


# ------------------------------------------------------------- Kadane pins

def test_maxss_seq_matches_bruteforce(oracle_lib):
    r = _rng(1)
    for n in list(range(0, 12)) + [31, 64]:
        for _ in range(40):
            x = r.integers(-5, 6, n)
            assert oracle_lib.maxss_seq(x) == brute_maxss(x)
    # +-1 sequences, the scoring of the workloads
    for _ in range(200):
        x = r.choice([-1, 1], size=int(r.integers(1, 64)))
        assert oracle_lib.maxss_seq(x) == brute_maxss(x)


def test_maxss_seq_special_cases(oracle_lib):
    assert oracle_lib.maxss_seq([]) == 0
    assert oracle_lib.maxss_seq([-3, -1, -7]) == 0          # empty run allowed
    assert oracle_lib.maxss_seq([4]) == 4
    assert oracle_lib.maxss_seq([2, -1, 2]) == 3            # bridge a dip
    assert oracle_lib.maxss_seq([2, -3, 2]) == 2            # do not bridge
    assert oracle_lib.maxss_seq([5, -4, 5, -4, 5]) == 7


def test_window_score_matches_bruteforce(oracle_lib):
    r = _rng(2)
    for _ in range(300):
        m = int(r.integers(1, 20))
        G = int(r.integers(1, 40))
        read = "".join(r.choice(list("ACGTN"), m, p=[.24, .24, .24, .24, .04]))
        genome = "".join(r.choice(list("ACGTN"), G, p=[.24, .24, .24, .24, .04]))
        p = int(r.integers(0, G + 3))
        M, X = int(r.integers(1, 6)), -int(r.integers(0, 6))
        assert oracle_lib.window_score(read, genome, p, M, X) == brute_window(read, genome, p, M, X)


def test_window_n_is_mismatch_everywhere(oracle_lib):
    assert oracle_lib.window_score("NNNN", "NNNN", 0, 1, -1) == 0
    assert oracle_lib.window_score("ACGT", "NNNN", 0, 5, -4) == 0
    assert oracle_lib.window_score("ACGT", "ACGT", 2, 1, -1) == 0   # "GT" then padding
    assert oracle_lib.window_score("GTAA", "ACGT", 2, 1, -1) == 2   # N padding past G
    assert oracle_lib.window_score("acgt", "ACGT", 0, 1, -1) == 4   # case-insensitive


# ------------------------------------------------- fragments (worked example)

def test_paper_toy_genome_fragments(oracle_lib):
    g = json.load(open(os.path.join(GOLD, "toy_genome_fig2.json")))
    genome, F = g["genome"], g["F"]
    assert oracle_lib.num_fragments(len(genome), F) == g["num_fragments"]
    # each fragment read as a query scores F*M exactly at its own offset 0
    for f, frag in enumerate(g["fragments"]):
        assert genome[f * F:(f + 1) * F] == frag
        reads = frag.encode()
        out = oracle_lib.scan(genome, F, reads, [0, F], M=1, X=-1, flags=oracle_lib.ONE_STRAND)
        assert out["score"][0][0] == F
        assert out["frag"][0][0] == f and out["offset"][0][0] == 0
    # the first base of each fragment (what threads 0..3 read first): a
    # one-base query equal to it reaches the full score in that fragment
    for f, b in enumerate(g["first_bases"]):
        assert genome[f * F] == b
        _, v = oracle_lib.scan(genome, F, b.encode(), [0, 1], flags=oracle_lib.ONE_STRAND,
                               want_values=True)
        assert v[0][f] == 1
        assert [int(x) for x in v[0]] == [int(b in fr) for fr in g["fragments"]]


def test_last_fragment_padded_with_n(oracle_lib):
    genome = "ACCGTAGGACCAT"   # 13 bases, F=3 -> 5 fragments, the last is "TNN"
    assert oracle_lib.num_fragments(len(genome), 3) == 5
    out, v = oracle_lib.scan(genome, 3, b"TNN", [0, 3], flags=oracle_lib.ONE_STRAND,
                             want_values=True)
    assert v.shape == (1, 5)
    assert v[0][4] == 1                 # T matches, the padding never does
    out, v = oracle_lib.scan(genome, 3, b"TAG", [0, 3], flags=oracle_lib.ONE_STRAND,
                             want_values=True)
    assert v[0][4] == 1                 # only T; "AG" would need bases past G


def test_windows_cross_fragment_junctions(oracle_lib):
    # the read spans the junction of fragments 0 and 1 and starts in fragment 0
    genome = "AAAACGTACCCC"
    out = oracle_lib.scan(genome, 4, b"ACGTAC", [0, 6], flags=oracle_lib.ONE_STRAND)
    assert out["score"][0][0] == 6
    assert out["frag"][0][0] == 0 and out["offset"][0][0] == 3


# ------------------------------------------------------------- scan invariants

def _small_case(seed, G=3000, F=256, n=12, m=40, rate=0.1):
    g = gen.uniform_genome(G, seed)
    r = gen.sample_reads(g, n, seed + 1, [m], rate, rate)
    return g, r, F


def test_scan_top2_matches_sort_of_fragment_values(oracle_lib):
    g, r, F = _small_case(5)
    out, vals = oracle_lib.scan(g.seq, F, r.seq, r.offsets, nthreads=4, want_values=True)
    NF = oracle_lib.num_fragments(g.G, F)
    for i in range(r.n):
        order = sorted(range(NF), key=lambda f: (-vals[i][f], f))
        assert out["frag"][i][0] == order[0] and out["score"][i][0] == vals[i][order[0]]
        assert out["frag"][i][1] == order[1] and out["score"][i][1] == vals[i][order[1]]


def test_scan_fragment_values_match_bruteforce_windows(oracle_lib):
    g, r, F = _small_case(6, G=700, F=96, n=4, m=12, rate=0.2)
    genome = g.seq.tobytes().decode()
    out, vals = oracle_lib.scan(g.seq, F, r.seq, r.offsets, want_values=True)
    NF = oracle_lib.num_fragments(g.G, F)
    comp = {"A": "T", "C": "G", "G": "C", "T": "A", "N": "N"}
    for i in range(r.n):
        q = r.read(i).decode()
        rc = "".join(comp[c] for c in reversed(q))
        for f in range(NF):
            best = max(brute_window(s, genome, f * F + o, 1, -1) for s in (q, rc) for o in range(F))
            assert vals[i][f] == best
        # representative: smallest strand then smallest offset among maxima
        f1 = out["frag"][i][0]
        cand = [(s, o) for s, qq in enumerate((q, rc)) for o in range(F)
                if brute_window(qq, genome, f1 * F + o, 1, -1) == vals[i][f1]]
        assert (out["strand"][i][0], out["offset"][i][0]) == min(cand)


def test_exact_copy_scores_m_at_true_offset(oracle_lib):
    g = gen.uniform_genome(20000, 9)
    F, m = 512, 60
    starts = [0, 511, 512, 7777, 19940]
    reads = b"".join(g.seq[s:s + m].tobytes() for s in starts)
    off = np.arange(len(starts) + 1) * m
    out = oracle_lib.scan(g.seq, F, reads, off, nthreads=4)
    for i, s in enumerate(starts):
        assert out["score"][i][0] == m
        assert out["frag"][i][0] == s // F and out["offset"][i][0] == s % F
        assert out["strand"][i][0] == 0
        assert 0 <= out["score"][i][1] <= m


def test_exact_repeat_tie_goes_to_smaller_fragment(oracle_lib):
    g = gen.uniform_genome(4096, 10).seq.copy()
    g[3000:3050] = g[100:150]           # exact repeat in fragment 5 (F=512)
    out = oracle_lib.scan(g, 512, g[3000:3050].tobytes(), [0, 50])
    assert out["score"][0].tolist() == [50, 50]
    assert out["frag"][0].tolist() == [0, 5]
    assert out["offset"][0].tolist() == [100, 3000 - 5 * 512]


def test_scores_bounded(oracle_lib):
    g, r, F = _small_case(7, rate=0.3)
    out, vals = oracle_lib.scan(g.seq, F, r.seq, r.offsets, M=5, X=-4, nthreads=4,
                                want_values=True)
    assert (vals >= 0).all() and (vals <= 5 * 40).all()


def test_right_n_padding_is_neutral(oracle_lib):
    g, r, F = _small_case(8)
    padded = b"".join(r.read(i) + b"N" * (i % 7) for i in range(r.n))
    off = np.zeros(r.n + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(r.read(i)) + (i % 7) for i in range(r.n)])
    a = oracle_lib.scan(g.seq, F, r.seq, r.offsets, flags=oracle_lib.ONE_STRAND)
    b = oracle_lib.scan(g.seq, F, padded, off, flags=oracle_lib.ONE_STRAND)
    assert (a == b).all()


def test_reverse_complement_swaps_strand_only(oracle_lib):
    g, r, F = _small_case(12)
    rc = b"".join(oracle_lib.revcomp(r.read(i)) for i in range(r.n))
    a, va = oracle_lib.scan(g.seq, F, r.seq, r.offsets, want_values=True)
    b, vb = oracle_lib.scan(g.seq, F, rc, r.offsets, want_values=True)
    assert (va == vb).all()
    assert (a["frag"] == b["frag"]).all() and (a["score"] == b["score"]).all()
    _, vf = oracle_lib.scan(g.seq, F, r.seq, r.offsets, flags=oracle_lib.ONE_STRAND,
                            want_values=True)
    _, vr = oracle_lib.scan(g.seq, F, rc, r.offsets, flags=oracle_lib.ONE_STRAND,
                            want_values=True)
    assert (np.maximum(vf, vr) == va).all()
    for i in range(r.n):
        f = a["frag"][i][0]
        if vf[i][f] == vr[i][f]:
            assert a["strand"][i][0] == 0 and b["strand"][i][0] == 0
        else:
            assert a["strand"][i][0] == int(vr[i][f] > vf[i][f])
            assert b["strand"][i][0] == 1 - a["strand"][i][0]
            assert a["offset"][i][0] == b["offset"][i][0]


def test_all_n_genome_scores_zero(oracle_lib):
    out = oracle_lib.scan(b"N" * 1000, 128, b"ACGTACGT" * 4, [0, 32])
    assert out["score"][0].tolist() == [0, 0]
    assert out["frag"][0].tolist() == [0, 1]
    assert out["offset"][0].tolist() == [0, 0] and out["strand"][0].tolist() == [0, 0]


def test_single_fragment_has_no_second(oracle_lib):
    out = oracle_lib.scan(b"ACGTACGTAC", 16, b"GTAC", [0, 4])
    assert out["frag"][0].tolist() == [0, -1]
    assert out["score"][0].tolist() == [4, -1]
    assert out["offset"][0][1] == -1 and out["strand"][0][1] == -1


def test_scan_rejects_bad_characters(oracle_lib):
    with pytest.raises(ValueError):
        oracle_lib.scan(b"ACGTX", 4, b"ACG", [0, 3])


# --------------------------------------------------------------------- NW pins

def _all_alignments(m, n):
    """Every global alignment path of lengths (m, n) as op strings."""
    if m == 0 and n == 0:
        yield ""
        return
    if m > 0 and n > 0:
        for rest in _all_alignments(m - 1, n - 1):
            yield "M" + rest
    if m > 0:
        for rest in _all_alignments(m - 1, n):
            yield "I" + rest
    if n > 0:
        for rest in _all_alignments(m, n - 1):
            yield "D" + rest


def _path_score(q, r, ops, M, X, gap):
    i = j = s = 0
    for op in ops:
        if op in "M=X":
            s += M if (q[i] == r[j] and q[i] != "N") else X
            i += 1; j += 1
        elif op == "I":
            s += gap; i += 1
        else:
            s += gap; j += 1
    return s, i, j


def brute_nw(q, r, M, X, gap, fitting):
    best = None
    spans = [(a, b) for a in range(len(r) + 1) for b in range(a, len(r) + 1)] if fitting \
        else [(0, len(r))]
    for a, b in spans:
        for ops in _all_alignments(len(q), b - a):
            s, _, _ = _path_score(q, r[a:b], ops, M, X, gap)
            best = s if best is None else max(best, s)
    return best


def _check_ops(q, r, jb, je, ops, score, M, X, gap):
    s, i, j = _path_score(q, r[jb:je], ops, M, X, gap)
    assert (s, i, j) == (score, len(q), je - jb)
    for k, op in enumerate(ops):
        assert op in "=XID"


@pytest.mark.parametrize("fitting", [False, True])
def test_nw_matches_enumeration_of_all_alignments(oracle_lib, fitting):
    r = _rng(3 + fitting)
    mode = oracle_lib.NW_FIT if fitting else oracle_lib.NW_GLOBAL
    for _ in range(60):
        m = int(r.integers(1, 5 if fitting else 6))
        n = int(r.integers(1, 6))
        q = "".join(r.choice(list("ACGT"), m))
        ref = "".join(r.choice(list("ACGTN"), n, p=[.23, .23, .23, .23, .08]))
        M, X, gap = int(r.integers(1, 6)), -int(r.integers(0, 5)), -int(r.integers(1, 8))
        sc, jb, je, ops = oracle_lib.nw(q, ref, M, X, gap, mode)
        assert sc == brute_nw(q, ref, M, X, gap, fitting)
        _check_ops(q, ref, jb, je, ops, sc, M, X, gap)
        if not fitting:
            assert (jb, je) == (0, n)


def test_nw_global_unit_costs_is_minus_edit_distance(oracle_lib):
    d = json.load(open(os.path.join(GOLD, "closed_forms.json")))["levenshtein_textbook"]
    for a, b, dist in d["pairs"]:
        if not a:
            continue
        sc, _, _, _ = oracle_lib.nw(a, b, 0, -1, -1, oracle_lib.NW_GLOBAL)
        assert sc == -dist, (a, b)


def test_nw_fitting_exact_occurrence(oracle_lib):
    g = gen.uniform_genome(500, 4).seq.tobytes().decode()
    q = g[200:260]
    sc, jb, je, ops = oracle_lib.nw(q, g, 1, -1, -2, oracle_lib.NW_FIT)
    assert sc == 60 and (jb, je) == (200, 260) and ops == "=" * 60


def test_nw_fitting_huge_gap_is_best_full_window(oracle_lib):
    r = _rng(11)
    for _ in range(50):
        m, n = int(r.integers(1, 9)), int(r.integers(1, 14))
        q = "".join(r.choice(list("ACGT"), m))
        ref = "".join(r.choice(list("ACGT"), n))
        sc, jb, je, ops = oracle_lib.nw(q, ref, 2, -3, -10 ** 6, oracle_lib.NW_FIT)
        if n >= m:
            best = max(sum(2 if q[k] == ref[p + k] else -3 for k in range(m))
                       for p in range(n - m + 1))
            assert sc == best and "I" not in ops and "D" not in ops
        else:   # the read is longer than the reference: gaps are forced
            assert sc <= -10 ** 6 + 2 * m and "I" in ops


def test_nw_traceback_priority_diag_first(oracle_lib):
    # read "A" against "AA": both columns give +1; the end is the smallest j
    sc, jb, je, ops = oracle_lib.nw("A", "AA", 1, -1, -2, oracle_lib.NW_FIT)
    assert (sc, jb, je, ops) == (1, 0, 1, "=")
    # global "AC" vs "A": diagonal at the first step is preferred over up
    sc, jb, je, ops = oracle_lib.nw("AA", "A", 1, -1, -1, oracle_lib.NW_GLOBAL)
    assert sc == 0 and ops in ("I=", "=I")
    assert ops == "I="   # traceback from (2,1): diagonal first, so the last pair is '='


def test_cigar_rle(oracle_lib):
    assert oracle_lib.cigar_rle("==X=") == "2=1X1="
    assert oracle_lib.cigar_rle("=" * 12 + "II" + "D") == "12=2I1D"
    assert oracle_lib.cigar_rle("") == ""


def test_align_one_region_and_strand(oracle_lib):
    g = gen.uniform_genome(10000, 21)
    F, m = 1024, 80
    s = 5000
    fwd = g.seq[s:s + m].tobytes()
    rc = oracle_lib.revcomp(fwd)
    a = oracle_lib.align_one(g.seq, F, fwd, s // F, 0)
    assert a["score"] == m and a["ref_begin"] == s and a["ref_end"] == s + m
    assert a["cigar"] == "%d=" % m
    b = oracle_lib.align_one(g.seq, F, rc, s // F, 1)
    assert b == dict(a, strand=1)
    # region clipped at the genome start
    c = oracle_lib.align_one(g.seq, F, g.seq[0:m].tobytes(), 0, 0)
    assert (c["ref_begin"], c["ref_end"], c["score"]) == (0, m, m)


# ------------------------------------------------------------- closed forms

def test_paper_closed_forms():
    d = json.load(open(os.path.join(GOLD, "closed_forms.json")))
    q = d["mapq_threshold"]
    assert round(-100 * math.log2(q["ratio"]), q["printed_decimals"]) == q["printed"]
    s = d["max_read_len_fermi"]
    cap = s["smem_bytes"] / s["bytes_per_base"] - s["lookahead"]
    assert int(cap) == s["cap_printed"]
    assert (int(cap) // 16) * 16 == s["limit"]
