"""The chromosome-scale and damaged-read workloads.

Scaled-down genomes of the same kind (41% GC, interspersed repeat families,
F = 4096) are checked in full against the oracle, through the plan and its
captured graph, NW included, and through the learned proposal.  The
full-size workloads run in the launch configuration of the benchmark (one
plan, graph replay) and are checked on sampled reads against records the
oracle wrote (tests/golden/make_fullsize_records.py: a fragment's value
depends only on the bases of its extended window, so the oracle runs on
genome slices at once and the per-fragment values are stitched back
together).  Every read is also checked against properties that hold at any
size.
"""
import hashlib
import json
import os
import time

import numpy as np
import pytest

import gen
import oracle
import paper_1403_2136_amd as mx
from oracle import mlp

pytestmark = pytest.mark.gpu

FIELDS = ("frag", "score", "offset", "strand")
GOLDEN_FULLSIZE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                               "fullsize_records.json")


def reads_sha256(r) -> str:
    """Digest of a read set (offsets, then bases), as the golden script takes it."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(r.offsets, dtype=np.uint64).tobytes())
    h.update(np.ascontiguousarray(r.seq, dtype=np.uint8).tobytes())
    return h.hexdigest()


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def assert_same(got, ref, what=""):
    for f in FIELDS:
        bad = np.nonzero((got[f] != ref[f]).any(axis=1))[0]
        assert bad.size == 0, "%s: %s differs for %d reads, first %d: gpu %s oracle %s" % (
            what, f, bad.size, bad[0], got[bad[0]], ref[bad[0]])


def plan_step(ix, r, pad, stride=512, graph=True):
    """One plan step on its own stream (graph replay when `graph`)."""
    torch = _torch()
    s = torch.from_numpy(np.array(r.seq)).cuda()
    o = torch.from_numpy(r.offsets.astype(np.int64)).cuda()
    top = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda")
    aln = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda")
    cig = torch.zeros(r.n * stride, dtype=torch.uint8, device="cuda")
    plan = mx.Plan(ix, capacity=r.n, pad=pad, cigar_stride=stride)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.run(s, o, top, aln, cig, stream=stream, graph=graph)
    stream.synchronize()
    plan.close()
    return (top.cpu().numpy().view(mx.TOP2_DTYPE).copy(),
            aln.cpu().numpy().view(mx.ALN_DTYPE).copy(), cig.cpu().numpy())


def check_properties(w, got, aln):
    """Invariants over every read of a workload."""
    lens = w.reads.lengths().astype(np.int64)
    sc = got["score"].astype(np.int64)
    assert (sc[:, 1] >= 0).all() and (sc[:, 0] >= sc[:, 1]).all()
    assert (sc[:, 0] <= lens * w.M).all()
    assert (got["frag"][:, 0] != got["frag"][:, 1]).all()
    NF = (w.genome.G + w.F - 1) // w.F
    assert ((got["frag"] >= 0) & (got["frag"] < NF)).all()
    assert ((got["offset"] >= 0) & (got["offset"] < w.F)).all()
    tie = sc[:, 0] == sc[:, 1]
    assert (got["frag"][tie, 0] < got["frag"][tie, 1]).all()
    assert (aln["strand"] == got["strand"][:, 0]).all()
    assert (aln["ref_begin"] <= aln["ref_end"]).all()


# ------------------------------------------------------------ scaled down

@pytest.fixture(scope="module")
def chrom_small():
    return gen.chromosome_genome(33, G=3_000_000, families=12)


def test_chromosome_like_mixed_lengths_plan_graph_and_nw(chrom_small):
    g = chrom_small
    r = gen.sample_reads(g, 120, 34, [36, 51, 100, 150, 250], 0.1, 0.3, indel_max=2)
    F = 4096
    ix = mx.Index(g.seq, F, 250)
    ref = oracle.scan(g.seq, F, r.seq, r.offsets, nthreads=16)
    got, aln, cig = plan_step(ix, r, 100)
    assert_same(got, ref, "chromosome-like, graph")
    exp = oracle.align_top(g.seq, F, r.seq, r.offsets, ref, 100)
    for i in range(r.n):
        e = exp[i]
        assert (int(aln["score"][i]), int(aln["strand"][i]), int(aln["ref_begin"][i]),
                int(aln["ref_end"][i]), mx.decode_cigar(cig, i, 512)) == \
            (e["score"], e["strand"], e["ref_begin"], e["ref_end"], e["cigar"]), i
    ix.close()


def test_damaged_reads_plan_and_proposal(chrom_small):
    """Damaged short reads (36-80 bp, 15-30% substitutions, C->T / G->A end
    damage, 0-1 indels): plan records equal the oracle's; the proposed path
    (untrained network, K = 16, about half the reads falling back) reports
    the full scan's record for fallen-back reads and the exact top-2 among
    its candidates for the others."""
    torch = _torch()
    g = chrom_small
    r = gen.sample_reads(g, 128, 53, (36, 80), 0.15, 0.30, indel_max=1, damage=True,
                         length_mode="range")
    F, K = 4096, 16
    ix = mx.Index(g.seq, F, 80)
    ref, vals = oracle.scan(g.seq, F, r.seq, r.offsets, nthreads=16, want_values=True)
    got, aln, cig = plan_step(ix, r, 100, graph=False)
    assert_same(got, ref, "damaged, plan")
    m = mx.Model(gen.mlp_init(54))
    s = torch.from_numpy(np.array(r.seq)).cuda()
    o = torch.from_numpy(r.offsets.astype(np.int64)).cuda()
    cand = torch.zeros(r.n * K, dtype=torch.int32, device="cuda")
    mg = torch.zeros(r.n, dtype=torch.float32, device="cuda")
    fb = torch.zeros(r.n, dtype=torch.uint8, device="cuda")
    m.candidates(ix, s, o, K, 0.0, cand, mg, fb)
    torch.cuda.synchronize()
    tau = float(np.median(mg.cpu().numpy()))
    out = torch.zeros(r.n * 32, dtype=torch.uint8, device="cuda")
    m.scan(ix, s, o, K, tau, out, fb)
    m.candidates(ix, s, o, K, tau, cand, mg, torch.zeros_like(fb))
    torch.cuda.synchronize()
    pr = out.cpu().numpy().view(mx.TOP2_DTYPE)
    fb = fb.cpu().numpy()
    cand = cand.cpu().numpy().reshape(r.n, K)
    assert 0 < fb.sum() < r.n
    for i in range(r.n):
        if fb[i]:
            assert all((pr[f][i] == ref[f][i]).all() for f in FIELDS), i
            continue
        f1, s1, f2, s2 = mlp.top2_among(vals[i], cand[i])
        assert pr["frag"][i].tolist() == [f1, f2] and pr["score"][i].tolist() == [s1, s2], i
    m.close()
    ix.close()


# ------------------------------------------------------------- full size

@pytest.mark.slow
@pytest.mark.parametrize("name", ["chromosome", "damaged"])
def test_full_size_workload_sampled(name):
    """The whole workload in one plan step (graph replay); sampled reads
    (chromosome: 10 per length class, damaged: 24; about a third of them from
    repeat-family copies) against the oracle's records stored by
    tests/golden/make_fullsize_records.py; invariants over every read."""
    t0 = time.time()
    gold = json.load(open(GOLDEN_FULLSIZE))[name]
    w = gen.workload(name)
    assert w.reads.n == gold["n_reads"] and w.genome.G == gold["G"]
    assert reads_sha256(w.reads) == gold["reads_sha256"], "generator output changed"
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap)
    print("%s: genome and index %.1fs" % (name, time.time() - t0), flush=True)
    got, aln, _ = plan_step(ix, w.reads, w.pad, stride=256)
    ix.close()
    print("%s: plan step %.1fs" % (name, time.time() - t0), flush=True)
    check_properties(w, got, aln)
    idx = np.array(gold["index"], dtype=np.int64)
    ref = np.zeros(idx.size, dtype=mx.TOP2_DTYPE)
    for i, rec in enumerate(gold["records"]):
        for f in FIELDS:
            ref[f][i] = rec[f]
    assert_same(got[idx], ref, name + " sample")
