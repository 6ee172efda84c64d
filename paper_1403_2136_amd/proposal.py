"""Marshalling for the learned fragment proposal.

Device reads live in torch tensors; labels are the plain scan's records
(maxss_scan_reads); training, its read order and negative draws, the
held-out evaluation and the choice of the acceptance thresholds all run in
the library (maxss_model_train).  These helpers only move buffers.
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


def scan_labels(index: Index, reads: DeviceReads, stream=None):
    """Top-2 records of the plain scan: (host copy, device tensor)."""
    torch = _torch()
    out = torch.empty(max(reads.n, 1) * 32, dtype=torch.uint8, device="cuda")
    s, o = reads.view()
    index.scan(s, o, out, stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:reads.n * 32].view(TOP2_DTYPE).copy(), out


def train(index: Index, model: Model, reads: DeviceReads, labels_dev, steps: int, **opts) -> dict:
    """maxss_model_train over all of `reads` (the last val_fraction held out)."""
    s, o = reads.view()
    return model.train(index, s, o, labels_dev, steps, **opts)


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


def scan_proposed(index: Index, model: Model, reads: DeviceReads, K: int, tau: float,
                  min_score: int = -1):
    """maxss_scan_reads_proposed: (records, fell_back) on host."""
    torch = _torch()
    n = reads.n
    out = torch.zeros(max(n, 1) * 32, dtype=torch.uint8, device="cuda")
    fb = torch.zeros(max(n, 1), dtype=torch.uint8, device="cuda")
    s, o = reads.view()
    model.scan(index, s, o, K, tau, out, fb, min_score=min_score)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:n * 32].view(TOP2_DTYPE).copy(), fb.cpu().numpy()[:n].copy()
