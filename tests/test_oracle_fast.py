"""Pins of the MaxSSmap_fast oracle (Methods, MaxSSmap_fast paragraph: every
other read base is scored).  Checked by brute force over the subsampled
substitution scores, by the identity that splits the genome into its even
and odd positions (the fast scan of q is, per parity, the plain scan of
q[0::2] against that parity's positions with fragments of F/2), and by the
exact-copy closed form."""
import numpy as np

import gen
import oracle


def subst(a, b, M, X):
    return M if (a == b and a != "N") else X


def brute(vals):
    best = 0
    for i in range(len(vals)):
        s = 0
        for j in range(i, len(vals)):
            s += vals[j]
            best = max(best, s)
    return best


def test_fast_window_equals_brute_force_over_even_positions():
    r = np.random.default_rng(7)
    for _ in range(300):
        m = int(r.integers(1, 14))
        G = int(r.integers(1, 30))
        q = "".join(r.choice(list("ACGTN"), m, p=[.24, .24, .24, .24, .04]))
        g = "".join(r.choice(list("ACGTN"), G, p=[.24, .24, .24, .24, .04]))
        p = int(r.integers(0, G + 3))
        M, X = int(r.integers(1, 6)), -int(r.integers(1, 6))
        vals = [subst(q[k], g[p + k] if p + k < G else "N", M, X) for k in range(0, m, 2)]
        assert oracle.window_score(q, g, p, M, X, step=2) == brute(vals)


def test_fast_scan_splits_into_parity_scans():
    for seed in range(6):
        G = gen.uniform_genome(int(300 + 37 * seed), 40 + seed)
        F = 16 * (1 + seed % 3)
        r = gen.sample_reads(G, 5, 50 + seed, [7, 12, 21], 0.0, 0.3)
        fast = oracle.scan(G.seq, F, r.seq, r.offsets, flags=oracle.ONE_STRAND | oracle.FAST,
                           want_values=True)
        half = []
        for par in (0, 1):
            gp = G.seq[par::2].tobytes()
            gp = gp + b"N" * ((G.G + 1) // 2 - len(gp))      # same fragment count
            sub = [r.read(i)[0::2] for i in range(r.n)]
            seq = b"".join(sub)
            off = np.cumsum([0] + [len(x) for x in sub]).astype(np.uint64)
            half.append(oracle.scan(gp, F // 2, seq, off, flags=oracle.ONE_STRAND,
                                    want_values=True))
        v = np.maximum(half[0][1], half[1][1])
        assert (fast[1] == v).all()
        for i in range(r.n):
            f = int(fast[0]["frag"][i][0])
            assert fast[0]["score"][i][0] == v[i].max()
            # representative offset: the smallest original offset 2 o' + parity among maxima
            attain = [par for par in (0, 1) if half[par][1][i][f] == v[i][f]]
            reps = [2 * int(half[par][0]["offset"][i][0]) + par for par in attain
                    if int(half[par][0]["frag"][i][0]) == f]
            if len(reps) == len(attain):
                assert int(fast[0]["offset"][i][0]) == min(reps)
            elif reps:
                assert int(fast[0]["offset"][i][0]) <= min(reps)


def test_fast_exact_copy_scores_half_length():
    G = gen.uniform_genome(5000, 9)
    for m, p in [(1, 0), (2, 17), (9, 4000), (50, 123), (51, 4949)]:
        read = G.seq[p:p + m].tobytes()
        assert oracle.window_score(read, G.seq.tobytes(), p, 5, -4, step=2) == 5 * ((m + 1) // 2)
        top = oracle.scan(G.seq, 2048, read, np.array([0, m], np.uint64), 5, -4,
                          flags=oracle.FAST)
        assert top["score"][0][0] == 5 * ((m + 1) // 2)
