"""Training and use of the learned fragment proposal.

Labels come from the plain scan itself (the best fragment and strand of
every training read).  Each step takes a batch of reads, the label fragment
and 63 negatives per read (the second-best fragment when there is one, the
rest uniform; drawn by the caller's seeded generator and passed in), and runs
the library's forward, backward and Adam kernels.  The margin threshold is
chosen on held-out reads so that the proposal agrees with the full scan's
best fragment on a target fraction of them.
"""
from __future__ import annotations

import numpy as np

from . import TOP2_DTYPE, Index, Model


def _torch():
    import torch
    return torch


class DeviceReads:
    """Reads uploaded once; `view(a, b)` gives the CSR slice of reads [a, b)
    without a copy (offsets stay absolute)."""

    def __init__(self, seq: np.ndarray, offsets: np.ndarray):
        torch = _torch()
        self.n = offsets.size - 1
        self.seq = torch.from_numpy(np.ascontiguousarray(seq)).cuda()
        self.off = torch.from_numpy(np.ascontiguousarray(offsets).astype(np.int64)).cuda()

    def view(self, a: int = 0, b: int | None = None):
        b = self.n if b is None else b
        return self.seq, self.off[a:b + 1]


def scan_labels(index: Index, reads: DeviceReads, stream=None) -> np.ndarray:
    """Top-2 records of the plain scan (host copy)."""
    torch = _torch()
    out = torch.empty(max(reads.n, 1) * 32, dtype=torch.uint8, device="cuda")
    s, o = reads.view()
    index.scan(s, o, out, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:reads.n * 32].view(TOP2_DTYPE).copy()


def train(index: Index, model: Model, reads: DeviceReads, labels: np.ndarray, steps: int,
          batch: int = 256, lr: float = 1e-3, seed: int = 0, stream=None, log=None):
    """`steps` Adam steps over consecutive batches of the (already shuffled)
    uploaded reads; returns the per-step mean losses."""
    import gen
    torch = _torch()
    nb = max(1, reads.n // batch)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    NF = index.NF
    for step in range(steps):
        b = step % nb
        a, e = b * batch, min(reads.n, (b + 1) * batch)
        lab = labels["frag"][a:e, 0].astype(np.int64)
        sec = labels["frag"][a:e, 1].astype(np.int64)
        neg = gen.sample_negatives(seed, step, lab, sec, NF)
        cand = np.concatenate([lab[:, None].astype(np.int32), neg], axis=1)
        strand = labels["strand"][a:e, 0].astype(np.int8)
        s, o = reads.view(a, e)
        model.train_step(index, s, o, torch.from_numpy(cand.ravel()).cuda(),
                         torch.from_numpy(strand).cuda(), lr, loss, None, stream)
        if step % 50 == 0 or step == steps - 1:
            torch.cuda.synchronize()
            losses.append((step, float(loss.item())))
            if log:
                log("step %d loss %.4f" % losses[-1])
    return losses


def candidates(index: Index, model: Model, reads: DeviceReads, K: int, tau: float = 0.0):
    """(candidates (n, K), margins (n,), fell_back (n,)) on host."""
    torch = _torch()
    n = reads.n
    cand = torch.zeros(n * K, dtype=torch.int32, device="cuda")
    mg = torch.zeros(n, dtype=torch.float32, device="cuda")
    fb = torch.zeros(n, dtype=torch.uint8, device="cuda")
    s, o = reads.view()
    model.candidates(index, s, o, K, tau, cand, mg, fb)
    torch.cuda.synchronize()
    return cand.cpu().numpy().reshape(n, K), mg.cpu().numpy(), fb.cpu().numpy()


def scores(index: Index, model: Model, reads: DeviceReads) -> np.ndarray:
    """Network score of every (read, fragment), max over strands (host,
    float32, n x NF)."""
    torch = _torch()
    out = torch.zeros(max(reads.n, 1) * index.NF, dtype=torch.float32, device="cuda")
    s, o = reads.view()
    model.scores(index, s, o, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:reads.n * index.NF].reshape(reads.n, index.NF)


def heldout_loss(score: np.ndarray, labels: np.ndarray, seed: int) -> float:
    """Mean softmax cross-entropy of the label fragment against 63 negatives
    drawn as in training, on strand-maxed scores of held-out reads."""
    import gen
    n, NF = score.shape
    lab = labels["frag"][:, 0].astype(np.int64)
    neg = gen.sample_negatives(seed, 0, lab, labels["frag"][:, 1].astype(np.int64), NF)
    s = np.take_along_axis(score.astype(np.float64),
                           np.concatenate([lab[:, None], neg.astype(np.int64)], axis=1), axis=1)
    top = s.max(axis=1, keepdims=True)
    lse = np.log(np.exp(s - top).sum(axis=1)) + top[:, 0]
    return float((lse - s[:, 0]).mean())


def recall(cand: np.ndarray, labels: np.ndarray) -> np.ndarray:
    """Per read: is the full scan's best fragment among the candidates."""
    return (cand == labels["frag"][:, :1]).any(axis=1)


def choose_margin(cand: np.ndarray, margins: np.ndarray, labels: np.ndarray,
                  target: float = 0.995) -> float:
    """Smallest threshold tau such that the reads either fall back
    (margin < tau) or hold their best fragment among the candidates for at
    least `target` of the held-out reads."""
    hit = recall(cand, labels)
    order = np.argsort(margins)
    m = margins[order]
    miss = (~hit[order]).astype(np.int64)
    n = m.size
    # after falling back the first k reads (smallest margins), misses left:
    left = miss.sum() - np.concatenate([[0], np.cumsum(miss)])
    ok = (n - left) / n >= target
    k = int(np.argmax(ok)) if ok.any() else n
    if k == 0:
        return float(m[0]) if n else 0.0          # nothing needs to fall back
    if k >= n:
        return float("inf")
    return float(np.nextafter(np.float32(m[k - 1]), np.float32(np.inf)))


def top1_agreement(got: np.ndarray, ref: np.ndarray) -> float:
    return float((got["frag"][:, 0] == ref["frag"][:, 0]).mean())


def score_agreement(got: np.ndarray, ref: np.ndarray) -> float:
    return float((got["score"][:, 0] == ref["score"][:, 0]).mean())
