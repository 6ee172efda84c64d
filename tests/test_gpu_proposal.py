"""GPU parity of the learned proposal against the float64 oracle.

Profiles are bit-exact (both sides normalise in float64 with correctly
rounded sqrt and divide, then round to float32 and bf16).  Network outputs
are compared with a bound derived from float32 accumulation: with u = 2^-24
and gamma_n = n u / (1 - n u), the GPU's pre-activations differ from the
oracle's by at most gamma_257 (sum_j |W1_kj z_j| + |b1_k|) per half, and y by
at most sum_k |w2_k| |dh_k| + gamma_257 (sum_k |w2_k h_k| + |b2|); the test
uses twice that bound.  Top-K membership at float ties is not pinned: a
candidate set is accepted when it differs from the oracle's only among
fragments whose scores lie within the bound of the K-th score.
"""
import numpy as np
import pytest

import gen
import oracle
from oracle import mlp
import paper_1403_2136_amd as mx

pytestmark = pytest.mark.gpu
U = 2.0 ** -24


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def gamma(n):
    return n * U / (1 - n * U)


@pytest.fixture(scope="module")
def small():
    """200 kbp genome with repeats, F = 2048 (98 fragments), 96 reads."""
    g = gen.uniform_genome(200_000, 61)
    seq = g.seq.copy()
    seq[150_000:152_000] = seq[20_000:22_000]
    g = gen.Genome(seq, "small")
    r = gen.sample_reads(g, 96, 62, [36, 51, 100, 150], 0.1, 0.3, indel_max=2)
    ix = mx.Index(g.seq, 2048, 150)
    yield g, r, ix
    ix.close()


def _dev_reads(torch, r):
    return (torch.from_numpy(np.array(r.seq)).cuda(),
            torch.from_numpy(r.offsets.astype(np.int64)).cuda())


def test_profiles_bit_exact(small):
    torch = _torch()
    g, r, ix = small
    s, o = _dev_reads(torch, r)
    rp = torch.zeros(r.n * 2 * 256, dtype=torch.float32, device="cuda")
    fp = torch.zeros(ix.NF * 256, dtype=torch.float32, device="cuda")
    mx.maxss_profiles(ix, s, o, rp, fp)
    torch.cuda.synchronize()
    rp = rp.cpu().numpy().reshape(r.n, 2, 256)
    fp = fp.cpu().numpy().reshape(ix.NF, 256)
    for i in range(r.n):
        ref = mlp.read_profiles(r.read(i)).astype(np.float32)
        assert (rp[i] == ref).all(), i
    ref_f = mlp.fragment_profiles(g.seq.tobytes(), 2048).astype(np.float32)
    assert (fp == ref_f).all()


def _oracle_scores(params, g, r, F):
    sh = mlp.shadow(params)
    vf = mlp.bf16(mlp.fragment_profiles(g.seq.tobytes(), F))
    W1, b1, w2, b2 = mlp.unpack(sh)
    ys, bounds = [], []
    for i in range(r.n):
        vr = mlp.bf16(mlp.read_profiles(r.read(i)))
        y = mlp.forward_decomposed(sh, vr, vf)                 # (2, NF)
        # error bound of the fp32 computation (see module docstring)
        ma = np.abs(vr) @ np.abs(W1[:, :256]).T + np.abs(b1)    # (2, H)
        mb = np.abs(vf) @ np.abs(W1[:, 256:]).T                 # (NF, H)
        pre = (vr @ W1[:, :256].T + b1)[:, None, :] + (vf @ W1[:, 256:].T)[None, :, :]
        h = np.maximum(pre, 0)
        dh = gamma(257) * (ma[:, None, :] + mb[None, :, :]) + U * np.abs(pre)
        by = dh @ np.abs(w2) + gamma(257) * (h @ np.abs(w2) + abs(b2))
        k = np.argmax(y, axis=0)
        ys.append(y.max(axis=0))
        bounds.append(2 * by.max(axis=0))
    return np.array(ys), np.array(bounds)


def test_scores_within_fp32_bound(small):
    torch = _torch()
    g, r, ix = small
    params = gen.mlp_init(5)
    m = mx.Model(params)
    s, o = _dev_reads(torch, r)
    out = torch.zeros(r.n * ix.NF, dtype=torch.float32, device="cuda")
    m.scores(ix, s, o, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(r.n, ix.NF).astype(np.float64)
    ref, bound = _oracle_scores(params, g, r, 2048)
    err = np.abs(got - ref)
    assert (err <= bound).all(), (err.max(), bound[err > bound][:3])
    m.close()


def test_candidates_and_margin(small):
    torch = _torch()
    g, r, ix = small
    params = gen.mlp_init(6)
    m = mx.Model(params)
    K, tau = 16, 0.05
    s, o = _dev_reads(torch, r)
    cand = torch.zeros(r.n * K, dtype=torch.int32, device="cuda")
    mg = torch.zeros(r.n, dtype=torch.float32, device="cuda")
    fb = torch.zeros(r.n, dtype=torch.uint8, device="cuda")
    m.candidates(ix, s, o, K, tau, cand, mg, fb)
    torch.cuda.synchronize()
    cand = cand.cpu().numpy().reshape(r.n, K)
    mg = mg.cpu().numpy()
    fb = fb.cpu().numpy()
    ref, bound = _oracle_scores(params, g, r, 2048)
    rc, rm = mlp.propose(ref, K)
    for i in range(r.n):
        assert (np.diff(cand[i]) > 0).all()
        kth = np.sort(ref[i])[::-1][K - 1]
        tol = 2 * bound[i].max()
        for f in set(cand[i]) ^ set(rc[i]):       # only near-ties may differ
            assert abs(ref[i, f] - kth) <= tol, (i, f)
        assert abs(mg[i] - rm[i]) <= 2 * tol
        if abs(rm[i] - tau) > 2 * tol:
            assert fb[i] == (rm[i] < tau)
    m.close()


def test_proposed_scan_exact_on_scanned_fragments(small):
    """Every read: a fallen-back read carries the full scan's record; any
    other read carries the exact top-2 among the candidate set the library
    proposed (which is itself checked against the oracle's scores in
    test_candidates_and_margin), with the full scan's representatives for
    the fragments the full scan also reports."""
    torch = _torch()
    g, r, ix = small
    params = gen.mlp_init(7)
    m = mx.Model(params)
    K = 8
    s, o = _dev_reads(torch, r)
    out = torch.zeros(r.n * 32, dtype=torch.uint8, device="cuda")
    fb = torch.zeros(r.n, dtype=torch.uint8, device="cuda")
    cand = torch.zeros(r.n * K, dtype=torch.int32, device="cuda")
    mg = torch.zeros(r.n, dtype=torch.float32, device="cuda")
    fb2 = torch.zeros(r.n, dtype=torch.uint8, device="cuda")
    ref, bound = _oracle_scores(params, g, r, 2048)
    rc, rm = mlp.propose(ref, K)
    tau = float(np.median(rm))                        # about half the reads fall back
    m.scan(ix, s, o, K, tau, out, fb)
    m.candidates(ix, s, o, K, tau, cand, mg, fb2)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(mx.TOP2_DTYPE)
    fb, fb2 = fb.cpu().numpy(), fb2.cpu().numpy()
    cand = cand.cpu().numpy().reshape(r.n, K)
    assert (fb == fb2).all()
    assert 0 < fb.sum() < r.n
    full, vals = oracle.scan(g.seq, 2048, r.seq, r.offsets, nthreads=8, want_values=True)
    for i in range(r.n):
        if fb[i]:
            for f in ("frag", "score", "offset", "strand"):
                assert (got[f][i] == full[f][i]).all(), i
            continue
        f1, s1, f2, s2 = mlp.top2_among(vals[i], cand[i])
        assert got["frag"][i].tolist() == [f1, f2] and got["score"][i].tolist() == [s1, s2], i
        for e in (0, 1):
            for k in (0, 1):
                if got["frag"][i][e] == full["frag"][i][k]:
                    assert got["score"][i][e] == full["score"][i][k]
                    assert got["offset"][i][e] == full["offset"][i][k], (i, e, k)
                    assert got["strand"][i][e] == full["strand"][i][k], (i, e, k)
    m.close()


def _train_batch(g, r, ix, seed, B=32):
    torch = _torch()
    labels = gen.Stream(seed, "t.lab").integers(0, ix.NF, B)
    second = -np.ones(B, dtype=np.int64)
    negs = gen.sample_negatives(seed, 0, labels, second, ix.NF)
    cand = np.concatenate([labels[:, None].astype(np.int32), negs], axis=1)
    strand = (gen.Stream(seed, "t.str").uniform(B) < 0.5).astype(np.int8)
    sub = r.subset(np.arange(B) % r.n)
    return sub, cand, strand


def _grad_bound(sh, t, B):
    """Per-parameter bound on |GPU gradient - oracle gradient|.

    The GPU rounds the per-read pre-activation gradient dA[b,k] = sum_c dh
    and the per-pair dh to bf16 (8 significant bits, round to nearest:
    relative error at most 2^-8) before the weight-gradient
    GEMMs, and accumulates in float32.  Upstream, y carries the forward
    float32 error, which reaches p = softmax(y) and hence dy and dh with
    relative error eps_up = 2 max|dy_err| + a few float32 units.  A ReLU
    unit whose pre-activation lies within the forward error of zero may flip,
    contributing |dy w2| to dh.
    """
    W1, b1, w2, b2 = mlp.unpack(sh)
    z, pre, h, dy, dh = t["z"], t["pre"], t["h"], t["dy"], t["dh"]
    n = z.shape[0]
    pre_err = gamma(257) * (np.abs(z) @ np.abs(W1).T + np.abs(b1))
    y_err = np.abs(w2) @ pre_err.T + gamma(257) * (np.abs(h) @ np.abs(w2) + abs(b2))
    eps_up = 2 * y_err.max() + 8 * U
    dh_abs = (np.abs(dh) + (np.abs(pre) <= pre_err) * np.abs(np.outer(dy, w2))) * (1 + eps_up)
    ub = 2.0 ** -8
    dA_abs = dh_abs.reshape(B, -1, 256).sum(axis=1)
    vr = np.abs(z.reshape(B, -1, 512)[:, 0, :256])
    bw1a = (ub + gamma(64) + gamma(B) + eps_up) * (dA_abs.T @ vr)
    bw1b = (ub + gamma(n) + eps_up) * (dh_abs.T @ np.abs(z[:, 256:]))
    bdb1 = (gamma(n) + eps_up) * dh_abs.sum(axis=0)
    bdw2 = (gamma(n) + eps_up + gamma(257)) * (np.abs(h).T @ np.abs(dy)) + np.abs(dy) @ (pre_err * (np.abs(pre) <= pre_err))
    bdb2 = (gamma(n) + eps_up) * np.abs(dy).sum()
    return np.concatenate([np.concatenate([bw1a, bw1b], axis=1).ravel(), bdb1, bdw2, [bdb2]]) + 1e-12


def test_train_step_gradient_matches_oracle(small):
    torch = _torch()
    g, r, ix = small
    params = gen.mlp_init(8)
    m = mx.Model(params)
    sub, cand, strand = _train_batch(g, r, ix, 9)
    s, o = _dev_reads(torch, sub)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(mx.MLP_PARAMS, dtype=torch.float32, device="cuda")
    m.train_step(ix, s, o, torch.from_numpy(cand.ravel()).cuda(),
                 torch.from_numpy(strand).cuda(), 0.0, loss, grad)
    torch.cuda.synchronize()
    vf = mlp.bf16(mlp.fragment_profiles(g.seq.tobytes(), 2048))
    vr = np.stack([mlp.bf16(mlp.read_profiles(sub.read(b)))[strand[b]] for b in range(sub.n)])
    sh = mlp.shadow(params)
    ref_loss, _, ref_g, t = mlp.loss_and_grad(sh, vr, vf[cand], parts=True)
    got_g = grad.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - ref_loss) <= 1e-4 * max(1.0, ref_loss)
    bound = _grad_bound(sh, t, sub.n)
    err = np.abs(got_g - ref_g)
    assert (err <= 2 * bound).all(), (np.argmax(err / (2 * bound)), (err / (2 * bound)).max())
    # lr = 0: parameters unchanged
    assert (m.params() == params).all()
    m.close()


def test_adam_steps_follow_oracle_trajectory(small, tmp_path):
    """One Adam step matches the oracle's update; 30 more steps on the same
    batch follow the oracle's loss trajectory (float64 Adam on the same
    bf16-shadowed forward) and lower the loss; save/load round-trips."""
    torch = _torch()
    g, r, ix = small
    params = gen.mlp_init(10)
    m = mx.Model(params)
    sub, cand, strand = _train_batch(g, r, ix, 11)
    s, o = _dev_reads(torch, sub)
    c = torch.from_numpy(cand.ravel()).cuda()
    st = torch.from_numpy(strand).cuda()
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(mx.MLP_PARAMS, dtype=torch.float32, device="cuda")
    lr = 3e-3
    m.train_step(ix, s, o, c, st, lr, loss, grad)
    torch.cuda.synchronize()
    g0 = grad.cpu().numpy().astype(np.float64)
    expect = mlp.Adam(mx.MLP_PARAMS).step(params.astype(np.float64), g0, lr)
    assert np.allclose(m.params(), expect, rtol=1e-5, atol=1e-7)
    # oracle trajectory
    vf = mlp.bf16(mlp.fragment_profiles(g.seq.tobytes(), 2048))
    vr = np.stack([mlp.bf16(mlp.read_profiles(sub.read(b)))[strand[b]] for b in range(sub.n)])
    p, opt, ref = params.astype(np.float64), mlp.Adam(mx.MLP_PARAMS), []
    for _ in range(31):
        lo, _, gr = mlp.loss_and_grad(mlp.shadow(p), vr, vf[cand])
        ref.append(lo)
        p = opt.step(p, gr, lr)
    got = [loss.item()]
    for k in range(1, 31):
        m.train_step(ix, s, o, c, st, lr, loss, None)
        if k % 10 == 0:
            torch.cuda.synchronize()
            got.append(loss.item())
    for k, gl in zip((0, 10, 20, 30), got):
        assert abs(gl - ref[k]) <= 0.03 * ref[k], (k, gl, ref[k])
    assert got[-1] < 0.75 * got[0]
    path = str(tmp_path / "m.bin")
    m.save(path)
    m2 = mx.Model(path=path)
    assert (m2.params() == m.params()).all()
    m.close()
    m2.close()


def _gain(g, F, K, length, rate_lo, rate_hi, indels, steps, lr):
    """Train on plain-scan labels of 12,288 reads; measure on 2,048 held-out
    reads against the same network untrained and against the cosine of the
    4-mer profiles; pick tau on 2,048 validation reads and run the proposed
    path on the held-out reads."""
    torch = _torch()
    from paper_1403_2136_amd import proposal as P
    ix = mx.Index(g.seq, F, length)
    mk = lambda n, seed: gen.sample_reads(g, n, seed, [length], rate_lo, rate_hi, indel_max=indels)
    tr, te, va = mk(12288, 72), mk(2048, 73), mk(2048, 74)
    dtr, dte, dva = (P.DeviceReads(x.seq, x.offsets) for x in (tr, te, va))
    ltr, lte, lva = (P.scan_labels(ix, d) for d in (dtr, dte, dva))
    params = gen.mlp_init(75)
    untrained, model = mx.Model(params), mx.Model(params)
    losses = P.train(ix, model, dtr, ltr, steps=steps, batch=256, lr=lr, seed=76)
    res = {"train_loss": (round(losses[0][1], 3), round(losses[-1][1], 3))}
    for name, m in (("trained", model), ("untrained", untrained)):
        c, _, _ = P.candidates(ix, m, dte, K)
        res["recall_" + name] = float(P.recall(c, lte).mean())
        res["ce_" + name] = P.heldout_loss(P.scores(ix, m, dte), lte, 77)
    vr = torch.zeros(te.n * 512, dtype=torch.float32, device="cuda")
    vf = torch.zeros(ix.NF * 256, dtype=torch.float32, device="cuda")
    s, o = dte.view()
    mx.maxss_profiles(ix, s, o, vr, vf)
    torch.cuda.synchronize()
    vr = vr.cpu().numpy().reshape(te.n, 2, 256)
    vf = vf.cpu().numpy().reshape(ix.NF, 256)
    cc, _ = mlp.propose(np.maximum(vr[:, 0] @ vf.T, vr[:, 1] @ vf.T), K)
    res["recall_cosine"] = float(P.recall(cc, lte).mean())
    c, mg, _ = P.candidates(ix, model, dva, K)
    tau = P.choose_margin(c, mg, lva, 0.995)
    out = torch.zeros(te.n * 32, dtype=torch.uint8, device="cuda")
    fbt = torch.zeros(te.n, dtype=torch.uint8, device="cuda")
    model.scan(ix, s, o, K, tau, out, fbt)
    torch.cuda.synchronize()
    res["tau"] = tau
    res["agreement"] = P.top1_agreement(out.cpu().numpy().view(mx.TOP2_DTYPE), lte)
    res["fallback"] = float(fbt.cpu().numpy().mean())
    for m in (model, untrained):
        m.close()
    ix.close()
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in res.items()}


def test_trained_proposal_gains_over_untrained(capsys):
    """What training on plain-scan labels buys, on a 600 kbp genome
    (293 fragments, K = 8).  On 250 bp reads with 0-5% substitutions the
    profiles carry the fragment's signal and the trained network must rank
    the best fragment into the top K far more often than the untrained one
    and lower the held-out loss; on 100 bp reads with 10-30% substitutions
    and indels (the bacterial read mix) the numbers are reported only.  In
    both, the proposed path with tau chosen on validation reads must agree
    with the full scan on at least 99% of held-out reads."""
    g = gen.bacterial_genome(71, base_len=600_000)
    strong = _gain(g, 2048, 8, 250, 0.0, 0.05, 0, 400, 2e-3)
    weak = _gain(g, 2048, 8, 100, 0.1, 0.3, 2, 400, 2e-3)
    with capsys.disabled():
        print("\nproposal gain, 250 bp 0-5%%: %s\nproposal gain, 100 bp 10-30%%: %s" % (strong, weak))
    assert strong["recall_trained"] > strong["recall_untrained"] + 0.1
    assert strong["ce_trained"] < strong["ce_untrained"] - 0.2
    assert strong["train_loss"][1] < strong["train_loss"][0]
    for r in (strong, weak):
        assert r["agreement"] >= 0.99


def test_train_step_rejects_bad_candidate_ids(small):
    torch = _torch()
    g, r, ix = small
    m = mx.Model(gen.mlp_init(12))
    sub, cand, strand = _train_batch(g, r, ix, 13, B=4)
    cand[2, 5] = ix.NF          # out of range
    s, o = _dev_reads(torch, sub)
    with pytest.raises(mx.MaxssError) as e:
        m.train_step(ix, s, o, torch.from_numpy(cand.ravel()).cuda(),
                     torch.from_numpy(strand).cuda(), 1e-3)
    assert e.value.status == mx.MAXSS_EINVAL
    assert (m.params() == gen.mlp_init(12)).all()
    m.close()
