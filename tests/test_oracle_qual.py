"""Pins of the base-quality scoring oracle (Methods, paragraph on base
qualities and the position specific scoring matrix): per-quality scores
probed through one-base alignments and checked against high-precision
decimal arithmetic; window scores and NW against brute force over explicit
per-position scores; the Q=93 / scale 3 reduction to the plain scoring; and
the strand symmetry with reversed qualities."""
from decimal import ROUND_HALF_UP, Decimal, getcontext

import numpy as np
import pytest

import gen
import oracle

getcontext().prec = 60
BIG_GAP = -10**5


def probe(Q, M, X, scale):
    """(match, mismatch) score of one base of quality Q, read off one-base
    global alignments (the gap is far too costly to use)."""
    q = chr(Q + 33)
    sm = oracle.nw("A", "A", M, X, BIG_GAP, oracle.NW_GLOBAL, qual=q, qscale=scale)[0]
    sx = oracle.nw("A", "C", M, X, BIG_GAP, oracle.NW_GLOBAL, qual=q, qscale=scale)[0]
    return sm, sx


def exact(Q, M, X, scale):
    """x = 1 - 10^(-Q/10) and the two scores to 50 digits."""
    x = Decimal(1) - Decimal(10) ** (Decimal(-Q) / Decimal(10))
    return Decimal(M) * x * scale, Decimal(X) * x * scale / Decimal(3)


def round_away(v: Decimal) -> int:
    return int(v.quantize(Decimal(1), rounding=ROUND_HALF_UP)) if v >= 0 else \
        -int((-v).quantize(Decimal(1), rounding=ROUND_HALF_UP))


@pytest.mark.parametrize("M,X,scale", [(1, -1, 10), (5, -4, 16), (2, -3, 7), (1, -1, 1)])
def test_per_quality_scores_match_high_precision(M, X, scale):
    for Q in range(0, 94):
        sm, sx = probe(Q, M, X, scale)
        for got, val in zip((sm, sx), exact(Q, M, X, scale)):
            frac = abs(val - val.to_integral_value(rounding="ROUND_FLOOR") - Decimal("0.5"))
            if frac > Decimal("1e-9"):
                assert got == round_away(val), (Q, got, val)
            else:                          # a half-integer: either neighbour
                assert got in (int(val - Decimal("0.5")), int(val + Decimal("0.5")))
    assert probe(0, M, X, scale) == (0, 0)       # x = 0: the base carries nothing


def _scores(qual, M, X, scale):
    return [probe(ord(c) - 33, M, X, scale) for c in qual]


def test_window_matches_brute_force_over_position_scores():
    r = np.random.default_rng(11)
    for _ in range(200):
        m = int(r.integers(1, 12))
        G = int(r.integers(1, 25))
        q = "".join(r.choice(list("ACGTN"), m, p=[.24, .24, .24, .24, .04]))
        g = "".join(r.choice(list("ACGTN"), G, p=[.24, .24, .24, .24, .04]))
        qual = "".join(chr(33 + int(v)) for v in r.integers(0, 42, m))
        p = int(r.integers(0, G + 2))
        step = int(r.choice([1, 2]))
        sc = _scores(qual, 5, -4, 10)
        vals = []
        for k in range(0, m, step):
            gb = g[p + k] if p + k < G else "N"
            vals.append(sc[k][0] if (q[k] == gb and q[k] != "N") else sc[k][1])
        # by enumeration of all runs (the empty run scores 0)
        best = max([0] + [sum(vals[i:j + 1]) for i in range(len(vals))
                          for j in range(i, len(vals))])
        assert oracle.window_score(q, g, p, 5, -4, step, qual, 10) == best


def test_top_quality_scale3_reduces_to_plain_scores():
    G = gen.uniform_genome(20_000, 3)
    r = gen.sample_reads(G, 12, 4, [20, 57, 100], 0.0, 0.3, indel_max=1)
    quals = np.full(r.seq.size, 33 + 93, np.uint8)
    # x = 1 - 1e-9.3: M x 3 rounds to 3M, X x 3 / 3 rounds to X
    a = oracle.scan(G.seq, 2048, r.seq, r.offsets, 1, -1, quals=quals, qscale=3, nthreads=4)
    b = oracle.scan(G.seq, 2048, r.seq, r.offsets, 3, -1, nthreads=4)
    for f in ("frag", "score", "offset", "strand"):
        assert (a[f] == b[f]).all()


def test_reverse_complement_with_reversed_qualities_swaps_strand():
    G = gen.uniform_genome(12_000, 5)
    r = gen.sample_reads(G, 8, 6, [30, 80], 0.0, 0.2)
    q = gen.sample_qualities(r, 7)
    seq2, q2 = [], []
    for i in range(r.n):
        a, b = int(r.offsets[i]), int(r.offsets[i + 1])
        seq2.append(oracle.revcomp(r.read(i)))
        q2.append(q[a:b][::-1].tobytes())
    s2 = b"".join(seq2)
    a1, v1 = oracle.scan(G.seq, 1024, r.seq, r.offsets, quals=q, qscale=10, want_values=True)
    a2, v2 = oracle.scan(G.seq, 1024, s2, r.offsets, quals=b"".join(q2), qscale=10,
                         want_values=True)
    assert (v1 == v2).all()
    assert (a1["frag"] == a2["frag"]).all() and (a1["score"] == a2["score"]).all()


def _all_paths(m, n):
    if m == 0 and n == 0:
        yield ""
        return
    if m and n:
        for t in _all_paths(m - 1, n - 1):
            yield "M" + t
    if m:
        for t in _all_paths(m - 1, n):
            yield "I" + t
    if n:
        for t in _all_paths(m, n - 1):
            yield "D" + t


@pytest.mark.parametrize("fitting", [False, True])
def test_nw_with_qualities_matches_enumeration(fitting):
    r = np.random.default_rng(21 + fitting)
    M, X, gap, scale = 5, -4, -3, 10
    for _ in range(60):
        m, n = int(r.integers(1, 5)), int(r.integers(1, 6))
        q = "".join(r.choice(list("ACGT"), m))
        ref = "".join(r.choice(list("ACGT"), n))
        qual = "".join(chr(33 + int(v)) for v in r.integers(0, 41, m))
        sc = _scores(qual, M, X, scale)
        spans = [(a, b) for a in range(n + 1) for b in range(a, n + 1)] if fitting else [(0, n)]
        best = None
        for a, b in spans:
            for ops in _all_paths(m, b - a):
                i = j = s = 0
                for op in ops:
                    if op == "M":
                        s += sc[i][0] if q[i] == ref[a + j] else sc[i][1]
                        i += 1; j += 1
                    elif op == "I":
                        s += gap * scale; i += 1
                    else:
                        s += gap * scale; j += 1
                best = s if best is None else max(best, s)
        mode = oracle.NW_FIT if fitting else oracle.NW_GLOBAL
        assert oracle.nw(q, ref, M, X, gap, mode, qual=qual, qscale=scale)[0] == best


def test_bad_quality_characters_rejected():
    with pytest.raises(ValueError):
        oracle.window_score("AC", "AC", 0, 1, -1, 1, " !", 10)
