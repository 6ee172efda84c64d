"""Out-of-memory paths, forced from the host: maxss_fail_alloc_after(n) makes
the n-th device allocation fail as an exhausted device would.  For every entry
point that allocates, each of its allocations in turn is made to fail: the
call must return MAXSS_ENOMEM with a message, release what it allocated, and
the same call must then succeed with the records of an unhindered run.  The
no-allocation scan must succeed with the hook armed for its first
allocation."""
import numpy as np
import pytest

import gen
import paper_1403_2136_amd as mx

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def case():
    g = gen.uniform_genome(30_000, 91)
    r = gen.sample_reads(g, 40, 92, [36, 100, 150], 0.0, 0.3, indel_max=2)
    return g, r


def _walk(call, check, limit=120):
    """Fail allocation 1, 2, ... of `call` until it needs none that fails;
    returns how many allocations it makes."""
    for n in range(1, limit + 1):
        mx.maxss_fail_alloc_after(n)
        try:
            res = call()
        except mx.MaxssError as e:
            mx.maxss_fail_alloc_after(0)
            assert e.status == mx.MAXSS_ENOMEM, e
            assert "out of memory" in str(e).lower() or "memory" in str(e).lower(), e
            check(call())          # the same call, unhindered
            continue
        mx.maxss_fail_alloc_after(0)
        check(res)
        return n - 1
    mx.maxss_fail_alloc_after(0)
    raise AssertionError("more than %d allocations" % limit)


def test_index_scan_align_host(case):
    g, r = case
    ix = mx.Index(g.seq, 2048, 150)
    ref = ix.scan(r.seq, r.offsets)
    ref_aln, ref_cig = ix.align(r.seq, r.offsets, ref, 100, 512)

    def same_index(h):
        G, NF, F = mx.maxss_index_info(h)
        assert (G, F) == (g.G, 2048)
        got = mx.maxss_scan_reads(h, r.seq, r.offsets)
        assert got.tobytes() == ref.tobytes()
        mx.maxss_index_free(h)

    na = _walk(lambda: mx.maxss_index_genome(g.seq, 2048, 150), same_index)
    assert na >= 3
    ns = _walk(lambda: ix.scan(r.seq, r.offsets), lambda got: np.testing.assert_array_equal(
        got.view(np.uint8), ref.view(np.uint8)))
    assert ns >= 8

    def same_aln(res):
        aln, cig = res
        assert aln.tobytes() == ref_aln.tobytes() and cig == ref_cig

    _walk(lambda: ix.align(r.seq, r.offsets, ref, 100, 512), same_aln)
    ix.close()


def test_device_scan_plan_and_noalloc(case):
    torch = _torch()
    g, r = case
    ix = mx.Index(g.seq, 2048, 150, flags=mx.MAXSS_EXCLUDE_ADJACENT)
    s = torch.from_numpy(np.array(r.seq)).cuda()
    o = torch.from_numpy(r.offsets.astype(np.int64)).cuda()
    out = torch.zeros(r.n * 32, dtype=torch.uint8, device="cuda")
    ix.scan(s, o, out)
    torch.cuda.synchronize()
    ref = out.cpu().numpy().copy()

    def scan_dev():
        out.zero_()
        ix.scan(s, o, out)
        torch.cuda.synchronize()
        return out.cpu().numpy().copy()

    _walk(scan_dev, lambda got: np.testing.assert_array_equal(got, ref))
    # the no-allocation scan makes none: armed for the first allocation, it
    # still runs, and the hook is still armed afterwards
    mx.maxss_fail_alloc_after(1)
    out.zero_()
    mx.maxss_scan_reads_noalloc(ix.handle, s, o, out)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == ref).all()
    with pytest.raises(mx.MaxssError) as e:
        ix.scan(r.seq, r.offsets)
    assert e.value.status == mx.MAXSS_ENOMEM
    mx.maxss_fail_alloc_after(0)

    def plan_step():
        plan = mx.Plan(ix, capacity=r.n, pad=100, cigar_stride=512)
        top = torch.zeros(r.n * 32, dtype=torch.uint8, device="cuda")
        aln = torch.zeros(r.n * 32, dtype=torch.uint8, device="cuda")
        cig = torch.zeros(r.n * 512, dtype=torch.uint8, device="cuda")
        plan.run(s, o, top, aln, cig)
        torch.cuda.synchronize()
        plan.close()
        return top.cpu().numpy().copy()

    _walk(plan_step, lambda got: np.testing.assert_array_equal(got, ref))
    ix.close()


def test_proposal_training_and_guarded_scan(case):
    torch = _torch()
    g, _ = case
    r = gen.sample_reads(g, 300, 93, [100], 0.0, 0.1)
    ix = mx.Index(g.seq, 1024, 100)
    s = torch.from_numpy(np.array(r.seq)).cuda()
    o = torch.from_numpy(r.offsets.astype(np.int64)).cuda()
    lab = torch.zeros(r.n * 32, dtype=torch.uint8, device="cuda")
    ix.scan(s, o, lab)
    torch.cuda.synchronize()

    def train():
        m = mx.Model(seed=1, init=mx.MAXSS_INIT_PROFILE_MATCH)
        try:
            st = m.train(ix, s, o, lab, 3, batch=32, lr=1e-3, seed=2, hard_negatives=4,
                         eval_every=2, K=8, val_fraction=0.2)
            return m.params(), st
        finally:
            m.close()

    ref_p, ref_st = train()
    _walk(train, lambda res: (np.testing.assert_array_equal(res[0], ref_p),
                              None if res[1] == ref_st else pytest.fail("%s != %s" % (res[1], ref_st))))
    m = mx.Model(seed=1, init=mx.MAXSS_INIT_PROFILE_MATCH)
    out = torch.zeros(r.n * 32, dtype=torch.uint8, device="cuda")
    fb = torch.zeros(r.n, dtype=torch.uint8, device="cuda")
    m.scan(ix, s, o, 8, 0.5, out, fb, min_score=60)
    torch.cuda.synchronize()
    ref = out.cpu().numpy().copy()

    def guarded():
        out.zero_()
        m.scan(ix, s, o, 8, 0.5, out, fb, min_score=60)
        torch.cuda.synchronize()
        return out.cpu().numpy().copy()

    _walk(guarded, lambda got: np.testing.assert_array_equal(got, ref))
    m.close()
    ix.close()
