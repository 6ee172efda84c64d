"""Pins of the float64 proposal oracle: brute-force 4-mer counts, library
bfloat16 rounding, the decomposition identity, finite-difference gradients,
Adam's closed-form first step, its constant-gradient closed form and
torch.optim.Adam over several steps, a hand-computed forward with both
biases, a sort-based top-K and top-2 among candidates."""
import itertools

import numpy as np
import pytest

import gen
from oracle import mlp

KMERS = ["".join(p) for p in itertools.product("ACGT", repeat=4)]


def brute_counts(s: str) -> np.ndarray:
    s = s.upper()
    c = np.zeros(256, dtype=np.int64)
    for t in range(len(s) - 3):
        sub = s[t:t + 4]
        if "N" in sub:
            continue
        c[KMERS.index(sub)] += 1
    return c


def test_kmer_counts_match_substring_enumeration():
    r = np.random.default_rng(1)
    for L in [0, 1, 3, 4, 5, 17, 100]:
        s = "".join(r.choice(list("ACGTN"), L, p=[.23, .23, .23, .23, .08]))
        assert (mlp.kmer_counts(mlp.codes(s.encode())) == brute_counts(s)).all()


def test_profile_is_unit_or_zero():
    v = mlp.read_profiles(b"ACGTACGTTTGA")
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)
    z = mlp.read_profiles(b"ACGNNACN")
    assert (z == 0).all()


def test_reverse_strand_profile_is_profile_of_reverse_complement():
    import oracle
    r = gen.sample_reads(gen.uniform_genome(5000, 3), 5, 4, [60], 0.1, 0.1)
    for i in range(r.n):
        q = r.read(i)
        v = mlp.read_profiles(q)
        rc = oracle.revcomp(q)
        assert np.allclose(v[1], mlp.read_profiles(rc)[0])
        c = brute_counts(rc.decode())
        assert np.allclose(v[1], c / np.linalg.norm(c))


def test_fragment_profile_counts_kmers_starting_inside():
    g = gen.with_n_runs(gen.uniform_genome(1000, 5), 6, 5, 1, 10).seq.tobytes().decode()
    F = 64
    NF = (len(g) + F - 1) // F
    V = mlp.fragment_profiles(g.encode(), F)
    assert V.shape == (NF, 256)
    for f in [0, 3, NF - 1]:
        c = np.zeros(256, dtype=np.int64)
        for t in range(f * F, min(len(g), f * F + F)):
            sub = g[t:t + 4]
            if len(sub) == 4 and "N" not in sub:
                c[KMERS.index(sub)] += 1
        n = np.linalg.norm(c)
        assert np.allclose(V[f], c / n if n else 0)


def test_bf16_matches_torch_round_to_nearest_even():
    import torch
    r = np.random.default_rng(2)
    x = np.concatenate([r.normal(0, 1, 20000), r.uniform(-1e-3, 1e-3, 1000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -0.0, 0.0, 65504.0]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert (mlp.bf16(x) == ref).all()
    assert mlp.bf16(1 + 2 ** -8) == 1.0          # tie to even
    assert mlp.bf16(1 + 3 * 2 ** -9) == 1 + 2 ** -7


def _params(seed=0):
    return gen.mlp_init(seed).astype(np.float64)


def test_decomposed_forward_equals_plain():
    p = _params(1)
    r = np.random.default_rng(3)
    vr = r.random((3, 256))
    vf = r.random((5, 256))
    y = mlp.forward_decomposed(p, vr, vf)
    for i in range(3):
        for j in range(5):
            yp, _, _ = mlp.forward(p, np.concatenate([vr[i], vf[j]])[None, :])
            assert abs(yp[0] - y[i, j]) < 1e-12 * max(1.0, abs(y[i, j]))


def test_gradient_matches_central_differences():
    p = _params(2)
    r = np.random.default_rng(4)
    vr = np.abs(r.normal(size=(2, 256)))
    vr /= np.linalg.norm(vr, axis=1, keepdims=True)
    vc = np.abs(r.normal(size=(2, 64, 256)))
    vc /= np.linalg.norm(vc, axis=2, keepdims=True)
    loss, y, g = mlp.loss_and_grad(p, vr, vc)
    idx = np.concatenate([r.integers(0, 256 * 512, 40), np.arange(256 * 512, 256 * 512 + 256, 37),
                          np.arange(256 * 513, 256 * 514, 41), [mlp.N_PARAMS - 1]])
    h = 1e-6
    for i in idx:
        q = p.copy(); q[i] += h
        lp, _, _ = mlp.loss_and_grad(q, vr, vc)
        q[i] -= 2 * h
        lm, _, _ = mlp.loss_and_grad(q, vr, vc)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd), (i, fd, g[i])


def test_loss_of_uniform_scores_is_log64():
    p = np.zeros(mlp.N_PARAMS)
    vr = np.ones((3, 256)) / 16
    vc = np.ones((3, 64, 256)) / 16
    loss, y, g = mlp.loss_and_grad(p, vr, vc)
    assert abs(loss - np.log(64)) < 1e-12


def test_adam_first_step_is_lr_times_sign():
    a = mlp.Adam(4)
    th = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -1e-3, 5.0, 0.0])
    out = a.step(th, g, 0.01)
    expect = th - 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(out, expect)


def test_propose_matches_sort():
    r = np.random.default_rng(5)
    s = r.integers(0, 6, size=(4, 40)).astype(np.float64)    # many ties
    c, m = mlp.propose(s, 8)
    for i in range(4):
        order = np.lexsort((np.arange(40), -s[i]))
        assert sorted(order[:8]) == list(c[i])
        assert m[i] == s[i, order[0]] - s[i, order[1]]


def test_params_layout_size():
    assert mlp.N_PARAMS == 131_585
    p = gen.mlp_init(0)
    assert p.dtype == np.float32 and p.size == mlp.N_PARAMS
    W1, b1, w2, b2 = mlp.unpack(p)
    assert W1.shape == (256, 512) and b1.shape == (256,) and w2.shape == (256,)


# ---- pins of top2_among, Adam past its first step and the forward biases

def test_top2_among_matches_lexsort_on_tie_heavy_rows():
    """Top-2 among candidates by (value desc, id asc): against a lexsort of
    the candidate values.  Values in 0..3 make most rows tie at the top, so a
    reversed id rule or a max that keeps the last tie fails."""
    r = np.random.default_rng(11)
    for trial in range(300):
        NF = int(r.integers(2, 40))
        vals = r.integers(0, 4, NF)
        k = int(r.integers(1, NF + 1))
        cand = np.sort(r.choice(NF, k, replace=False))
        f1, s1, f2, s2 = mlp.top2_among(vals, cand)
        order = cand[np.lexsort((cand, -vals[cand]))]
        assert (f1, s1) == (int(order[0]), int(vals[order[0]]))
        if k == 1:
            assert (f2, s2) == (-1, -1)
        else:
            assert (f2, s2) == (int(order[1]), int(vals[order[1]]))
    # a hand-checked row: three fragments tie at 3; ids 4 and 7 are the two smallest
    assert mlp.top2_among(np.array([0, 2, 1, 0, 3, 2, 0, 3, 3]), [8, 7, 4, 1]) == (4, 3, 7, 3)


def test_top2_among_all_fragments_is_the_scan_top2():
    """Over every fragment, top2_among of the oracle's exact value row gives
    the scan's own top-2 (fragment and score); over a candidate set holding
    the scan's two winners it gives the same; over a set without the winner
    it gives the best remaining fragment of the value row."""
    import oracle
    g = gen.bacterial_genome(7, base_len=60_000)
    r = gen.sample_reads(g, 24, 8, [60], 0.0, 0.2, indel_max=1)
    F = 512
    top, vals = oracle.scan(g.seq, F, r.seq, r.offsets, want_values=True)
    NF = vals.shape[1]
    rng = np.random.default_rng(12)
    for i in range(r.n):
        f1, s1, f2, s2 = mlp.top2_among(vals[i], range(NF))
        assert (f1, s1, f2, s2) == (top["frag"][i][0], top["score"][i][0],
                                    top["frag"][i][1], top["score"][i][1])
        extra = rng.choice(NF, 10, replace=False)
        cand = np.unique(np.concatenate([extra, top["frag"][i]]))
        assert mlp.top2_among(vals[i], cand) == (f1, s1, f2, s2)
        rest = [f for f in range(NF) if f != f1]
        g1, t1, _, _ = mlp.top2_among(vals[i], rest)
        assert (g1, t1) == (f2, s2)


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient g, both bias-corrected moments equal g and g^2
    exactly at every step t (the EMA of a constant, divided by 1 - beta^t), so
    every step moves theta by lr * g / (|g| + eps).  A bias correction with a
    wrong power of beta (e.g. beta instead of beta^t) fails from step 2 on."""
    a = mlp.Adam(3)
    th = np.array([0.25, -1.0, 2.0])
    g = np.array([0.5, -3.0, 1e-4])
    lr = 0.01
    for t in range(1, 6):
        th_new = a.step(th, g, lr)
        assert np.allclose(th - th_new, lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0), t
        th = th_new


def test_adam_three_steps_match_torch_adam():
    """Three steps with changing gradients against torch.optim.Adam (float64,
    same betas and eps): the bias correction at t = 2 and 3 is pinned to an
    independent implementation of the same published update."""
    import torch
    r = np.random.default_rng(13)
    th0 = r.normal(size=50)
    grads = [r.normal(size=50) * s for s in (1.0, -2.5, 0.3)]
    lr = 3e-3
    a = mlp.Adam(50)
    th = th0.copy()
    p = torch.nn.Parameter(torch.from_numpy(th0.copy()))
    opt = torch.optim.Adam([p], lr=lr, betas=(0.9, 0.999), eps=1e-8)
    for g in grads:
        th = a.step(th, g, lr)
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        assert np.allclose(th, p.detach().numpy(), rtol=0, atol=1e-14)
    # by hand, element 0 of a scalar run g = (1, -2, 0.5), lr 0.1: after step 2
    # m = -0.11, v = 0.004999, m_hat = -0.11/0.19, v_hat = 0.004999/0.001999
    s = mlp.Adam(1)
    x = s.step(np.zeros(1), np.array([1.0]), 0.1)
    x = s.step(x, np.array([-2.0]), 0.1)
    step2 = (-0.11 / 0.19) / (np.sqrt(0.004999 / 0.001999) + 1e-8)
    assert abs(x[0] - (-0.1 / (1 + 1e-8) - 0.1 * step2)) < 1e-14


def test_forward_hand_computed_with_biases_and_negative_preactivation():
    """y = w2 . ReLU(W1 z + b1) + b2 on a hand-sized case: unit 0 is active
    (pre 1 + 2*0.5 + 0.5 = 2.5), unit 1 is negative (pre -1 + 0.25 = -0.75,
    contributes 0), unit 2 is active through its bias only (0.125); all other
    units have zero weights and a zero bias.  y = 2*2.5 + 0 + 4*0.125 - 0.75
    = 4.75.  Dropping b2 gives 5.5; dropping b1 gives 3.25; no ReLU gives
    0.95."""
    W1 = np.zeros((256, 512))
    b1 = np.zeros(256)
    w2 = np.zeros(256)
    W1[0, 3] = 1.0
    W1[0, 256 + 5] = 2.0
    b1[0] = 0.5
    W1[1, 3] = -1.0
    b1[1] = 0.25
    w2[1] = 5.0
    b1[2] = 0.125
    w2[0], w2[2] = 2.0, 4.0
    p = mlp.pack(W1, b1, w2, -0.75)
    vr = np.zeros(256)
    vr[3] = 1.0
    vf = np.zeros(256)
    vf[5] = 0.5
    y, pre, h = mlp.forward(p, np.concatenate([vr, vf])[None, :])
    assert y[0] == 4.75
    assert pre[0, 0] == 2.5 and pre[0, 1] == -0.75 and h[0, 1] == 0.0
    assert mlp.forward_decomposed(p, vr[None, :], vf[None, :])[0, 0] == 4.75
    # the training forward keeps b2 in every logit: with a zero fragment
    # profile unit 0's pre-activation is 1 + 0.5 = 1.5, so y = 3 + 0.5 - 0.75
    loss, yl, _ = mlp.loss_and_grad(p, vr[None, :], np.stack([vf, np.zeros(256)])[None, :, :])
    assert yl[0, 0] == 4.75 and yl[0, 1] == 2.75


# ------------------------------------------- training random numbers (oracle)

def test_splitmix64_published_values():
    # the generator's first outputs from state 0 and from state 1234567
    # (state += 0x9E3779B97F4A7C15, then the output function)
    assert [mlp.mix64(0 + (k + 1) * mlp.GAMMA) for k in range(3)] == \
        [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [mlp.mix64(1234567 + (k + 1) * mlp.GAMMA) for k in range(5)] == \
        [6457827717110365317, 3203168211198807973, 9817491932198370423,
         4593380528125082431, 16408922859458223821]
    key = mlp.sm_key(5, 2)
    assert mlp.sm_draw(key, 3) == mlp.mix64(key + 4 * mlp.GAMMA)


def test_init_params_glorot_statistics():
    p = mlp.init_params(9, 0)
    W1, b1, w2, b2 = mlp.unpack(p)
    a1, a2 = np.sqrt(6.0 / 768), np.sqrt(6.0 / 257)
    assert np.abs(W1).max() <= a1 and np.abs(w2).max() <= a2
    assert (b1 == 0).all() and b2 == 0
    # uniform on [-a, a]: mean 0 and variance a^2 / 3 within 5 standard errors
    n = W1.size
    assert abs(W1.mean()) < 5 * a1 / np.sqrt(3 * n)
    assert abs(W1.var() - a1 ** 2 / 3) < 5 * a1 ** 2 * np.sqrt(4 / 45 / n)
    assert not (mlp.init_params(10, 0) == p).all()
    q = mlp.init_params(9, 1)
    W1, b1, w2, b2 = mlp.unpack(q)
    assert (np.diag(W1[:, :256]) == 8).all() and (np.diag(W1[:, 256:]) == 1).all()
    assert np.count_nonzero(W1) == 512 and (b1 == -np.float32(0.2)).all() and (w2 == 1).all()


def test_batch_reads_visit_every_read_once_per_epoch():
    valid = list(range(0, 90, 3))                       # 30 labelled reads
    seen = [r for t in range(6) for r in mlp.batch_reads(4, t, 5, valid)]
    assert sorted(seen) == valid                        # 6 steps x 5 = one epoch
    nxt = [r for t in range(6, 12) for r in mlp.batch_reads(4, t, 5, valid)]
    assert sorted(nxt) == valid and nxt != seen
    assert mlp.batch_reads(4, 0, 5, valid) != mlp.batch_reads(5, 0, 5, valid)


def test_batch_candidates_rule():
    NF = 300
    rows = [mlp.batch_candidates(3, t, 8, b, (7 * t + b) % NF, -1 if b % 2 else (b + 1) % NF, NF)
            for t in range(40) for b in range(8)]
    counts = np.zeros(NF)
    for k, row in enumerate(rows):
        t, b = divmod(k, 8)
        lab = (7 * t + b) % NF
        assert len(row) == 64 and row[0] == lab and lab not in row[1:]
        assert len(set(row)) == 64 and all(0 <= f < NF for f in row)
        if b % 2 == 0 and (b + 1) % NF != lab:
            assert row[1] == (b + 1) % NF
        counts[row[2:]] += 1
    # the uniform draws cover the fragments evenly (chi-square, 299 dof)
    e = counts.sum() / NF
    assert ((counts - e) ** 2 / e).sum() < 299 + 6 * np.sqrt(2 * 299)
    # fewer fragments than candidates: every other fragment, then repeats
    small = mlp.batch_candidates(1, 0, 1, 0, 2, -1, 5)
    assert small[0] == 2 and sorted(set(small[1:])) == [0, 1, 3, 4]
    assert all(small[5 + j] == small[1 + j % 4] for j in range(59))
    assert mlp.batch_candidates(1, 0, 1, 0, 0, -1, 1) == [0] * 64
