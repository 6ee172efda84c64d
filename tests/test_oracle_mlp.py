"""Pins of the float64 proposal oracle: brute-force 4-mer counts, library
bfloat16 rounding, the decomposition identity, finite-difference gradients,
Adam's closed-form first step and a sort-based top-K."""
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
