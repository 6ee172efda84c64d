"""Mapping quality on the device and SAM records from the device pipeline,
against the oracle: every (best, second) score pair up to 1,023 plus random
pairs up to the int16 score range, both thresholds; then scan + NW + MAPQ on
the GPU formatted as SAM, byte for byte against the oracle's text."""
import numpy as np
import pytest

import gen
import oracle
from oracle import sam
import paper_1403_2136_amd as mx

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _pairs():
    s1, s2 = [], []
    for a in range(0, 1024):
        s1.extend([a] * (a + 2))
        s2.extend(range(-1, a + 1))
    st = gen.Stream(5, "mapq.pairs")
    a = st.integers(1, 65536, 100_000)
    b = (st.uniform(100_000) * (a + 1)).astype(np.int64)
    s1.extend(a.tolist())
    s2.extend(b.tolist())
    return np.array(s1, np.int64), np.array(s2, np.int64)


@pytest.mark.parametrize("num,den,min_q", [(9, 10, -1), (1, 1, 62), (3, 4, 20)])
def test_mapq_kernel_every_pair(num, den, min_q):
    torch = _torch()
    s1, s2 = _pairs()
    n = s1.size + 1
    top = np.zeros(n, dtype=mx.TOP2_DTYPE)
    top["frag"][:-1, 0] = 0
    top["frag"][:-1, 1] = np.where(s2 >= 0, 1, -1)
    top["score"][:-1, 0] = s1
    top["score"][:-1, 1] = s2
    top["frag"][-1, 0] = -2                       # an invalid read
    d = torch.from_numpy(top.view(np.uint8).copy()).cuda()
    q = torch.zeros(n, dtype=torch.uint8, device="cuda")
    m = torch.zeros(n, dtype=torch.uint8, device="cuda")
    mx.maxss_mapq(d, n, q, m, num, den, min_q)
    torch.cuda.synchronize()
    q, m = q.cpu().numpy(), m.cpu().numpy()
    ref_q = np.array([sam.mapq(a, b) for a, b in zip(s1, s2)] + [0], np.uint8)
    ref_m = np.array([sam.is_mapped(a, b, num, den, min_q) for a, b in zip(s1, s2)] + [False],
                     np.uint8)
    bad = np.nonzero(q != ref_q)[0]
    assert bad.size == 0, (bad[:5], s1[bad[:5]], s2[bad[:5]], q[bad[:5]], ref_q[bad[:5]])
    assert (m == ref_m).all()


def test_device_pipeline_sam_equals_oracle():
    torch = _torch()
    G = gen.uniform_genome(150_000, 31)
    s = G.seq.copy()
    s[100_000:102_000] = s[10_000:12_000]
    G = gen.Genome(s, "rep")
    r = gen.sample_reads(G, 150, 32, [36, 100, 150], 0.0, 0.3, indel_max=2)
    F, pad, stride = 2048, 100, 64
    ix = mx.Index(G.seq, F, 150)
    sd = torch.from_numpy(np.array(r.seq)).cuda()
    od = torch.from_numpy(r.offsets.astype(np.int64)).cuda()
    top = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda")
    aln = torch.empty(r.n * 32, dtype=torch.uint8, device="cuda")
    cig = torch.zeros(r.n * stride, dtype=torch.uint8, device="cuda")
    q = torch.empty(r.n, dtype=torch.uint8, device="cuda")
    m = torch.empty(r.n, dtype=torch.uint8, device="cuda")
    ix.scan(sd, od, top)
    ix.align(sd, od, top, pad, stride, aln, cig)
    mx.maxss_mapq(top, r.n, q, m)
    torch.cuda.synchronize()
    topn = top.cpu().numpy().view(mx.TOP2_DTYPE)
    alnn = aln.cpu().numpy().view(mx.ALN_DTYPE)
    txt = mx.maxss_sam_header(ix.handle, "chrS") + mx.maxss_sam_records(
        r.seq, r.offsets, topn, alnn, cig.cpu().numpy(), stride, q.cpu().numpy(),
        m.cpu().numpy(), "chrS")
    ix.close()
    otop = oracle.scan(G.seq, F, r.seq, r.offsets, nthreads=16)
    oal = oracle.align_top(G.seq, F, r.seq, r.offsets, otop, pad)
    exp = sam.header("chrS", G.G) + "".join(
        sam.record("r%d" % i, r.read(i), otop[i], oal[i], "chrS",
                   truncated=len(oal[i]["cigar"]) >= stride) for i in range(r.n))
    assert txt == exp
    lines = txt.splitlines()[3:]
    flags = [int(x.split("\t")[1]) for x in lines]
    assert 4 in flags and 0 in flags and 16 in flags
