"""The scan's time does not depend on how divergent the reads are.

The paper's runs take the same minutes whatever the divergence of the reads
(Results, Table 3(b): MaxSSmap at divergence .1, .2 and .3): the first phase
scores every cell of every (read, strand, fragment, offset), with no early
exit.  The same must hold here: on the bacterial genome, 50,000 reads of
100 bp with no substitution and 50,000 with 30% substitutions (same lengths,
no indels, no N) take the same scan kernel time within 2%.
"""
import numpy as np
import pytest

import gen
import paper_1403_2136_amd as mx

pytestmark = pytest.mark.gpu


def _scan_ms(ix, s, o, out, torch):
    mx.maxss_profile_enable(True)
    ix.scan(s, o, out, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    ms, k = mx.maxss_profile_read("scan")
    mx.maxss_profile_enable(False)
    assert k == 1
    return ms


def test_scan_time_independent_of_divergence():
    import torch
    assert torch.cuda.is_available()
    w = gen.workload("bacterial", n_reads=1)
    g = w.genome
    sets = {}
    for rate in (0.0, 0.3):
        r = gen.sample_reads(g, 50_000, 123, [100], rate, rate)
        assert (r.lengths() == 100).all()
        assert not (np.frombuffer(r.seq.tobytes(), np.uint8) == ord("N")).any()
        sets[rate] = (torch.from_numpy(np.array(r.seq)).cuda(),
                      torch.from_numpy(r.offsets.astype(np.int64)).cuda())
    ix = mx.Index(g.seq, w.F, 100)
    out = torch.empty(50_000 * 32, dtype=torch.uint8, device="cuda")
    for rate in sets:                       # warm-up
        _scan_ms(ix, *sets[rate], out, torch)
    times = {0.0: [], 0.3: []}
    for _ in range(3):
        for rate in (0.0, 0.3):
            times[rate].append(_scan_ms(ix, *sets[rate], out, torch))
    a, b = np.median(times[0.0]), np.median(times[0.3])
    print("scan ms at divergence 0: %s, at 0.3: %s" % (times[0.0], times[0.3]), flush=True)
    assert abs(a - b) / min(a, b) <= 0.02, (a, b)
    ix.close()
