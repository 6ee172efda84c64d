"""Batching: plans (no allocation per call), HIP graph replay, mixed read
lengths in one launch, every tile shape, and the autotuner's parity gate."""
import os

import numpy as np
import pytest

import gen
import oracle
import paper_1403_2136_amd as mx

pytestmark = pytest.mark.gpu

FIELDS = ("frag", "score", "offset", "strand")


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def assert_same(got, ref, what=""):
    for f in FIELDS:
        bad = np.nonzero((got[f] != ref[f]).any(axis=1))[0]
        assert bad.size == 0, "%s: %s differs for %d reads, first %d: gpu %s oracle %s" % (
            what, f, bad.size, bad[0], got[bad[0]], ref[bad[0]])


def _dev(torch, a, dtype=None):
    t = torch.from_numpy(np.array(a, copy=True))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def mixed_case(seed=3, G=60_000, n=96, lens=(36, 51, 100, 150, 250), repeats=40):
    g = gen.uniform_genome(G, seed)
    seq = g.seq.copy()
    st = gen.Stream(seed, "batch.repeats")
    for _ in range(repeats):
        L = int(st.integers(40, 400, 1)[0])
        a = int(st.integers(0, G - L, 1)[0])
        b = int(st.integers(0, G - L, 1)[0])
        seq[b:b + L] = seq[a:a + L]
    g = gen.Genome(seq, "mixed")
    r = gen.sample_reads(g, n, seed + 1, list(lens), 0.05, 0.3, indel_max=2)
    return g, r


def test_plan_step_matches_calls_and_oracle():
    torch = _torch()
    g, r = mixed_case()
    ix = mx.Index(g.seq, 1024, 250)
    ref = oracle.scan(g.seq, 1024, r.seq, r.offsets, nthreads=8)
    plan = mx.Plan(ix, capacity=200, pad=60, cigar_stride=512)
    s, o = _dev(torch, r.seq), _dev(torch, r.offsets.astype(np.int64))
    top = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda")
    aln = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda")
    cig = torch.zeros(r.n * 512, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    plan.run(s, o, top, aln, cig, stream=stream)
    torch.cuda.synchronize()
    got = top.cpu().numpy().view(mx.TOP2_DTYPE)
    assert_same(got, ref, "plan")
    a2, c2 = ix.align(r.seq, r.offsets, ref, 60, 512)
    assert (aln.cpu().numpy().view(mx.ALN_DTYPE) == a2).all()
    cg = cig.cpu().numpy()
    assert [mx.decode_cigar(cg, i, 512) for i in range(r.n)] == c2
    plan.close()
    ix.close()


def test_mixed_lengths_one_launch_equals_per_length_launches():
    g, r = mixed_case(seed=5)
    ix = mx.Index(g.seq, 1024, 250)
    whole = ix.scan(r.seq, r.offsets)
    lens = r.lengths()
    for L in np.unique(lens):
        idx = np.nonzero(lens == L)[0]
        sub = r.subset(idx)
        part = ix.scan(sub.seq, sub.offsets)
        assert (part == whole[idx]).all()
    ref = oracle.scan(g.seq, 1024, r.seq, r.offsets, nthreads=8)
    assert_same(whole, ref, "mixed")
    ix.close()


def test_graph_replays_with_new_contents():
    torch = _torch()
    g = gen.uniform_genome(40_000, 7)
    ra = gen.sample_reads(g, 64, 8, [36, 100, 150], 0.1, 0.2, indel_max=1)
    # a second batch with the same read lengths (so the same CSR offsets) but
    # other sequences: every base re-drawn with probability 0.3
    rb_seq = gen.substitute(gen.Stream(9, "replay.b"), ra.seq, 0.3)
    ix = mx.Index(g.seq, 512, 150)
    ref_a = ix.scan(ra.seq, ra.offsets)
    ref_b = ix.scan(rb_seq, ra.offsets)
    assert_same(ref_a, oracle.scan(g.seq, 512, ra.seq, ra.offsets, nthreads=8), "eager a")
    plan = mx.Plan(ix, capacity=64, pad=50, cigar_stride=256)
    s = _dev(torch, ra.seq)
    o = _dev(torch, ra.offsets.astype(np.int64))
    top = torch.empty(64 * 32, dtype=torch.uint8, device="cuda")
    aln = torch.empty(64 * 32, dtype=torch.uint8, device="cuda")
    cig = torch.zeros(64 * 256, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    src = {0: ra.seq, 1: rb_seq}
    refs = {0: ref_a, 1: ref_b}
    for rep, which in enumerate([0, 1, 0, 1, 1, 0]):
        s.copy_(torch.from_numpy(np.array(src[which])).cuda())
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            plan.run(s, o, top, aln, cig, stream=stream, graph=True)
        stream.synchronize()
        got = top.cpu().numpy().view(mx.TOP2_DTYPE)
        assert_same(got, refs[which], "replay %d" % rep)
        # the program's own eager work between replays
        eager = ix.scan(ra.seq[:300].copy(), [0, 100, 200, 300])
        assert eager.shape == (3,)
        torch.cuda.synchronize()
    plan.close()
    ix.close()


def _adversarial():
    g = gen.with_n_runs(gen.uniform_genome(20_000, 11), 12, 15, 1, 80)
    seq = g.seq.copy()
    seq[15000:15300] = seq[2000:2300]          # exact repeat: ties
    seq[9000:9300] = seq[2000:2300]
    reads = [seq[2000:2000 + m].tobytes() for m in (1, 7, 64, 100, 129, 300)]
    r = gen.sample_reads(gen.Genome(seq, "adv"), 24, 13, [17, 48, 111, 250, 300], 0.1, 0.3,
                         indel_max=2)
    reads += [r.read(i) for i in range(r.n)]
    off = np.zeros(len(reads) + 1, np.uint64)
    off[1:] = np.cumsum([len(x) for x in reads])
    return seq, b"".join(reads), off


@pytest.mark.parametrize("F", [4096, 2048, 1024, 8192])
def test_every_tile_shape_is_exact(F):
    seq, reads, off = _adversarial()
    ref = oracle.scan(seq, F, reads, off, nthreads=8)
    ix = mx.Index(seq, F, 300)
    for np_ in (8, 16, 32):
        if 128 * np_ > max(F, 1024):
            continue
        for R in (1, 3, 8, 32):
            for rounds in (1, 8, 64):
                ix.set_tiles(np_, R, rounds)
                got = ix.scan(reads, off)
                assert_same(got, ref, "F=%d NP=%d R=%d rounds=%d" % (F, np_, R, rounds))
    ix.close()


def test_autotune_parity_gate_and_cache(tmp_path):
    g, r = mixed_case(seed=17, G=80_000, n=256)
    ix = mx.Index(g.seq, 2048, 250)
    cache = str(tmp_path / "tune.txt")
    res = ix.autotune(r.seq, r.offsets, cache)
    assert res["tried"] > 0 and res["rejected"] == 0 and res["from_cache"] == 0
    assert res["best_ms"] <= res["default_ms"] + 1e-6
    ref = oracle.scan(g.seq, 2048, r.seq, r.offsets, nthreads=8)
    assert_same(ix.scan(r.seq, r.offsets), ref, "after autotune")
    res2 = ix.autotune(r.seq, r.offsets, cache)
    assert res2["from_cache"] == 1 and res2["np"] == res["np"]
    assert os.path.getsize(cache) > 0
    # an entry with the same key but a shape outside the accepted range is
    # skipped: the shapes are timed again
    key = open(cache).readline().split("|")[0]
    bad = str(tmp_path / "bad.txt")
    with open(bad, "w") as f:
        f.write(key + "| np=7 R=500 rounds=3 best_ms=1.0 default_ms=2.0\n")
    res3 = ix.autotune(r.seq, r.offsets, bad)
    assert res3["from_cache"] == 0 and res3["tried"] > 0 and res3["np"] in (0, 8, 16, 32)
    assert_same(ix.scan(r.seq, r.offsets), ref, "after a skipped cache entry")
    ix.close()
