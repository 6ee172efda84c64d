"""The seeded input generator: determinism and distribution checks."""
import numpy as np

import gen


def test_stream_is_counter_based_and_deterministic():
    a = gen.Stream(7, "x").u64(1000)
    s = gen.Stream(7, "x")
    b = np.concatenate([s.u64(10), s.u64(990)])
    assert (a == b).all()
    assert not (gen.Stream(8, "x").u64(1000) == a).all()
    assert not (gen.Stream(7, "y").u64(1000) == a).all()


def test_splitmix64_reference_values():
    # SplitMix64 with state 0: the first outputs of the published generator
    # (state += 0x9E3779B97F4A7C15; mix) are fixed by its definition.
    st = gen.Stream.__new__(gen.Stream)
    st.key = np.uint64(0)
    st.ctr = 0
    out = st.u64(3)
    assert [int(x) for x in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniform_range_and_moments():
    u = gen.Stream(1, "u").uniform(200_000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.005
    k = gen.Stream(1, "k").integers(3, 9, 100_000)
    assert k.min() == 3 and k.max() == 8


def test_genome_gc_content():
    g = gen.uniform_genome(200_000, 3, gc=0.41)
    s = g.seq
    gc = np.isin(s, np.frombuffer(b"GC", np.uint8)).mean()
    assert abs(gc - 0.41) < 0.005
    assert set(np.unique(s).tobytes()) <= set(b"ACGT")


def test_tiny_workload_deterministic():
    a = gen.workload("tiny")
    gen._GENOME_CACHE.clear()
    b = gen.workload("tiny")
    assert (a.genome.seq == b.genome.seq).all()
    assert (a.reads.seq == b.reads.seq).all() and (a.reads.offsets == b.reads.offsets).all()
    assert a.genome.G == 50_000 and a.reads.n == 200
    assert (a.reads.lengths() == 100).all()


def test_reads_substitution_rate_and_truth():
    g = gen.uniform_genome(100_000, 5)
    r = gen.sample_reads(g, 2000, 6, [100], 0.2, 0.2)
    comp = np.zeros(256, np.uint8)
    for x, y in zip(b"ACGT", b"TGCA"):
        comp[x] = y
    mism = 0
    for i in range(r.n):
        q = np.frombuffer(r.read(i), np.uint8)
        if r.strand[i]:
            q = comp[q[::-1]]
        t = g.seq[r.start[i]:r.start[i] + 100]
        mism += int((q != t).sum())
    rate = mism / (2000 * 100)
    # binomial: sd = sqrt(.2*.8/2e5) ~ 0.0009
    assert abs(rate - 0.2) < 0.005
    assert 0.45 < r.strand.mean() < 0.55


def test_reads_with_indels_have_exact_length():
    g = gen.uniform_genome(50_000, 8)
    r = gen.sample_reads(g, 500, 9, [36, 51, 100, 150, 250], 0.1, 0.3, indel_max=2)
    assert (np.isin(r.lengths(), [36, 51, 100, 150, 250])).all()
    assert set(np.unique(r.n_indel)) <= {0, 1, 2}
    assert (r.start >= 0).all() and (r.start + r.span <= g.G).all()


def test_damage_raises_ct_at_five_prime_end():
    g = gen.uniform_genome(50_000, 10)
    r = gen.sample_reads(g, 3000, 11, (36, 80), 0.0, 0.0, damage=True, length_mode="range")
    first = np.array([r.read(i)[0] for i in range(r.n)])
    last = np.array([r.read(i)[-1] for i in range(r.n)])
    # without damage each is ~25%; C->T at rate 0.3 at the first base
    assert (first == ord("C")).mean() < 0.21 and (first == ord("T")).mean() > 0.29
    assert (last == ord("G")).mean() < 0.21 and (last == ord("A")).mean() > 0.29


def test_negatives_distinct_unbiased_and_second_first():
    NF, B = 2269, 4096
    st = gen.Stream(5, "neg.test")
    labels = st.integers(0, NF, B)
    second = np.where(st.uniform(B) < 0.5, st.integers(0, NF, B), -1)
    neg = gen.sample_negatives(3, 0, labels, second, NF)
    assert neg.shape == (B, 63) and neg.dtype == np.int32
    assert ((neg >= 0) & (neg < NF)).all()
    assert (neg != labels[:, None]).all()
    for b in range(B):
        assert len(set(neg[b].tolist())) == 63
    has2 = (second >= 0) & (second != labels)
    assert (neg[has2, 0] == second[has2]).all()
    # the uniform draws cover the whole id range: mean and quartiles of a
    # uniform variable on [0, NF), within several standard errors
    u = neg[:, 1:].ravel().astype(np.float64)
    se = NF / np.sqrt(12 * u.size)
    assert abs(u.mean() - (NF - 1) / 2) < 6 * se
    assert abs((u < NF / 4).mean() - 0.25) < 0.01 and abs((u >= 3 * NF / 4).mean() - 0.25) < 0.01
    # tiny genomes: every other fragment appears, cycled
    small = gen.sample_negatives(3, 1, np.array([2]), np.array([-1]), 5)
    assert sorted(set(small[0].tolist())) == [0, 1, 3, 4]
