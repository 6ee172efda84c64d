"""Benchmark of the MaxSS hot path on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic reads
already resident in HBM: maxss_scan_reads (read encoding, the MaxSS scan of
every read against every fragment on both strands, top-2 merge, exact re-scan
of the two winners) followed by maxss_align_top (NW of every read on its best
fragment).  The metric is MaxSS GCUPS = (sum over reads of 2 * G * m) / step
time / 1e9 (both strands, every genome start position).

The roofline object prices the scan kernel at a fixed algorithmic unit, one
16-bit lane operation per cell (the Kadane step's saturating add), against
the packed 16-bit VALU peak derived from 256 CUs x 64 lanes x 2.4 GHz x 2;
beside it are the peak measured on the GPU by maxss_roof_int16 and the
launched kernel's own instructions per cell.

Beside the step, on the same reads: the scan of host buffers (PCIe
included), MaxSSmap_fast, base-quality scoring, the neighbour exclusion of
the second-best fragment and the learned proposal against the full scan;
then the batched path on the 248 Mbp chromosome-scale workload (persistent
scan, captured graph, autotuned tiles; one eager and one timed graph step),
the damaged short reads on that genome (one eager plan step) and the CPU
oracle on samples (each leg can be switched off).

Prints one JSON line.  `--gpus N` with N > 1 is refused: the benchmark
measures one GPU (the scan shards by reads across GPUs with no collective).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used for the roofline objects
HBM_PEAK_GBS = 8000.0
CU, SIMD_LANES, CLOCK = 256, 64, 2.4e9          # 256 CUs x 4 SIMD16 = 64 lanes/clk/CU
INT16_PACKED_OPS = CU * SIMD_LANES * CLOCK * 2   # 16-bit lane ops/s with packed math
# The scan's algorithmic unit, fixed whatever kernel runs: one 16-bit lane
# operation per cell, the Kadane step's saturating add H = max(0, H + sigma)
# (the add and the clamp at zero are one saturating add).  The running
# maximum and the score selection are not counted: the kernel shares them
# between cells (one three-input minimum per two steps, the per-base score
# pairs once per window word).
UNIT_OPS_PER_CELL = 1.0
# Context from the paper (Table 3(b) and its CPU comparison; rates derived
# from the printed minutes, one strand): Tesla M2050 and 12-core Xeon X5650.
PAPER_CONTEXT = {"gpu_gcups_derived": 69.0, "gpu": "Tesla M2050 (Fermi), MaxSSmap 28 min for "
                 "100,000 x 251 bp reads on E. coli",
                 "cpu_gcups_derived": 8.6, "cpu": "12-core Xeon X5650, OpenMP, 224 min"}


def recorded_traffic(workload: str):
    """HBM bytes per scan launch from the committed counter summary of this
    workload, or None when there is none or the scan kernel's sources have
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "scan_kernel_%s.md" % workload)
    if not os.path.exists(path):
        return None
    want, traffic = None, None
    for line in open(path):
        if line.startswith("scan sources sha256:"):
            want = line.split(":", 1)[1].split()
        elif line.startswith("traffic bytes per launch:"):
            traffic = int(line.split(":", 1)[1])
    have = [hashlib.sha256(open(os.path.join(ROOT, "paper_1403_2136_amd", "csrc", f), "rb")
                           .read()).hexdigest() for f in ("scan.hip", "internal.h")]
    return traffic if want == have else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_info() -> dict:
    """The host's CPU model, its logical CPU count, the CPUs this process may
    run on and the cgroup CPU quota (None when unlimited)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = float(q) / float(per)
    except (OSError, ValueError):
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)), "cgroup_quota_cpus": quota}


def cpu_threads(info: dict) -> int:
    """Threads for the all-cores leg: the CPUs this process may run on,
    bounded by the cgroup quota and by OMP_NUM_THREADS when the host sets it
    (the CPU share a one-GPU job is given)."""
    n = info["affinity"]
    if info["cgroup_quota_cpus"]:
        n = min(n, max(1, int(info["cgroup_quota_cpus"])))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_baseline(w, budget_s: float = 6.0):
    """The oracle as it stands on this host (scan + top-2 + NW), median of
    three runs on each of two legs: all cores (see cpu_threads) on a sample of
    the workload's reads sized to about budget_s, and one thread on a sample
    sized to about max(budget_s / 2, 3.5 s) per run (at least 10 s over its
    three runs).  The tiny workload (50 kbp, 200 reads) is timed in full; the
    full-workload time is an extrapolation from the all-cores rate."""
    import numpy as np

    import gen
    import oracle
    info = cpu_info()
    threads = cpu_threads(info)
    G = w.genome.G

    def run(sub, nt, ww=w):
        t0 = time.perf_counter()
        top = oracle.scan(ww.genome.seq, ww.F, sub.seq, sub.offsets, ww.M, ww.X, nthreads=nt)
        oracle.align_top(ww.genome.seq, ww.F, sub.seq, sub.offsets, top, ww.pad, ww.M, ww.X,
                         ww.gap)
        return time.perf_counter() - t0

    # calibration: one read per thread
    k0 = min(threads, w.reads.n)
    dt0 = run(w.reads.subset(np.arange(k0)), threads)
    per_read_mt = dt0 / k0 * threads          # seconds per read on one of `threads` threads
    k = int(min(w.reads.n, max(threads, budget_s / max(per_read_mt, 1e-6) * threads)))
    k = max(threads, (k // threads) * threads)
    rates = []
    for rep in range(3):
        sub = w.reads.subset((np.arange(k) + k0 + rep * k) % w.reads.n)
        dt = run(sub, threads)
        rates.append(2.0 * G * float(sub.lengths().sum()) / dt / 1e9)
    # one thread: at least 3.5 s per run, so that the three runs take >= 10 s
    k1 = max(1, int(math.ceil(max(0.5 * budget_s, 3.5) / max(per_read_mt, 1e-6))))
    rates1, t1 = [], 0.0
    for rep in range(3):
        one = w.reads.subset((np.arange(k1) + rep * k1) % w.reads.n)
        dt = run(one, 1)
        t1 += dt
        rates1.append(2.0 * G * float(one.lengths().sum()) / dt / 1e9)
    tiny = gen.workload("tiny")
    tiny_rates = []
    for _ in range(3):
        dt = run(tiny.reads, threads, tiny)
        tiny_rates.append(2.0 * tiny.genome.G * float(tiny.reads.lengths().sum()) / dt / 1e9)
    value = float(np.median(rates))
    full_cells = 2.0 * G * float(w.reads.lengths().sum())
    return {"value": round(value, 3), "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": "3 runs of %d of the %d reads (scan both strands + top-2 + NW), median; "
                      "GCUPS of the runs %s" % (k, w.reads.n, [round(x, 3) for x in rates]),
            "host": info,
            # an extrapolation from the sample's rate, not a measurement
            "full_workload_s_extrapolated": round(full_cells / (value * 1e9), 1),
            "single_thread": {"value": round(float(np.median(rates1)), 3), "cores": 1,
                              "sample": "3 runs of %d reads, %.1f s in all, median" % (k1, t1)},
            "tiny_workload_in_full": {"value": round(float(np.median(tiny_rates)), 3),
                                      "cores": threads, "reads": tiny.reads.n,
                                      "sample": "all 200 reads of the 50 kbp workload, median "
                                                "of 3"},
            "paper_context": PAPER_CONTEXT}


def _cosine_recall(ix, dreads, labels, K):
    """Recall@K of the non-learned ranking (cosine of the 4-mer profiles, max
    over strands, ties to the smaller id) on device reads: evaluation only."""
    import numpy as np
    import torch

    import paper_1403_2136_amd as mx
    s, o = dreads.view()
    vr = torch.zeros(dreads.n * 512, dtype=torch.float32, device="cuda")
    vf = torch.zeros(ix.NF * 256, dtype=torch.float32, device="cuda")
    mx.maxss_profiles(ix, s, o, vr, vf)
    torch.cuda.synchronize()
    vr = vr.view(dreads.n, 2, 256).double()
    vf = vf.view(ix.NF, 256).double()
    sc = torch.maximum(vr[:, 0] @ vf.T, vr[:, 1] @ vf.T).cpu().numpy()
    ids = np.broadcast_to(np.arange(ix.NF), sc.shape)
    top = np.lexsort((ids, -sc), axis=1)[:, :K]
    return float((top == labels["frag"][:, :1]).any(axis=1).mean())


def proposal_leg(ix, w, seq, off, top_full, stream, args, tw=None, name=None):
    """Learned proposal on the workload's genome.  Training reads are drawn
    like the workload's with their own seed (bacterial: `train_reads`;
    damaged: `damaged_train_reads`) or given (`tw`), labelled by the plain
    scan, and trained in the library (maxss_model_train: profile-matching
    start, hard negatives, early stopping on held-out recall@K, margin and
    exact-score thresholds for 99.5% held-out agreement).  Then the proposal
    path and the full scan are timed over the same number of passes on the
    workload's reads (already in HBM), with top-1 agreement and fallback."""
    import numpy as np
    import torch

    import gen
    import paper_1403_2136_amd as mx
    from paper_1403_2136_amd import proposal as P
    t0 = time.time()
    if tw is None:
        if w.name == "bacterial":
            tw = gen.workload("proposal_train", n_reads=args.train_reads)
        else:
            tw = gen.workload(w.name, n_reads=args.damaged_train_reads, read_seed=53)
    dtr = P.DeviceReads(tw.reads.seq, tw.reads.offsets)
    _, lab = P.scan_labels(ix, dtr)
    t_label = time.time() - t0
    model = mx.Model(seed=43, init=mx.MAXSS_INIT_PROFILE_MATCH)
    t1 = time.time()
    st = P.train(ix, model, dtr, lab, args.train_steps, batch=256, lr=args.train_lr, seed=44,
                 hard_negatives=args.hard_negatives, eval_every=200, K=args.K, val_fraction=0.1,
                 target_agreement=0.995)
    t_train = time.time() - t1
    del dtr, lab
    log("proposal%s: labels %.1fs, training %.1fs: %s" % (
        " " + name if name else "", t_label, t_train, st))
    n = w.reads.n
    out = torch.empty(n * 32, dtype=torch.uint8, device="cuda")
    fbt = torch.empty(n, dtype=torch.uint8, device="cuda")
    tau, ms = st["tau"], st["min_score"]
    model.scan(ix, seq, off, args.K, tau, out, fbt, stream=stream, min_score=ms)   # warm-up
    torch.cuda.synchronize()
    reps = 3 if w.name == "bacterial" else 1     # a damaged-workload pass takes about a minute
    t_prop = t_full = 0.0
    for rep in range(reps):
        t2 = time.perf_counter()
        model.scan(ix, seq, off, args.K, tau, out, fbt, stream=stream, min_score=ms)
        torch.cuda.synchronize()
        t_prop += time.perf_counter() - t2
        t3 = time.perf_counter()
        ix.scan(seq, off, top_full, stream=stream)
        torch.cuda.synchronize()
        t_full += time.perf_counter() - t3
        log("proposal: timed pass %d done" % rep)
    t_prop /= reps
    t_full /= reps
    got = out.cpu().numpy().view(mx.TOP2_DTYPE)
    ref = top_full.cpu().numpy().view(mx.TOP2_DTYPE)
    # recall@K of the trained network and of the cosine ranking on a sample
    # of the workload's reads
    k = min(n, 4096)
    sub = w.reads.subset(np.arange(k))
    dsub = P.DeviceReads(sub.seq, sub.offsets)
    c, _, _ = P.candidates(ix, model, dsub, args.K)
    rec = float((c == ref[:k]["frag"][:, :1]).any(axis=1).mean())
    cos = _cosine_recall(ix, dsub, ref[:k], args.K)
    res = {"reads_per_s": round(n / t_prop, 1), "full_scan_reads_per_s": round(n / t_full, 1),
           "speedup": round(t_full / t_prop, 3),
           "top1_agreement": round(float((got["frag"][:, 0] == ref["frag"][:, 0]).mean()), 5),
           "score_agreement": round(float((got["score"][:, 0] == ref["score"][:, 0]).mean()), 5),
           "fallback_rate": round(float(fbt.cpu().numpy().mean()), 4), "K": args.K,
           "tau": tau, "min_score": ms, "passes_timed": reps,
           "recall_at_K": {"trained": round(rec, 4), "cosine": round(cos, 4),
                           "sample_reads": k},
           "training": {kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in st.items()},
           "train_reads": tw.reads.n, "train_steps": args.train_steps,
           "train_s": round(t_train, 2), "label_s": round(t_label, 2)}
    log("proposal: %s" % res)
    model.close()
    return res


def proposal_regime_leg(args, dev, stream):
    """The learned proposal where 4-mer profiles carry the fragment's signal:
    the bacterial genome with 100,000 reads of 100 bp at 0-5% substitutions
    and no indels (training: 200,000 other such reads)."""
    import numpy as np
    import torch

    import gen
    import paper_1403_2136_amd as mx
    w = gen.workload("bacterial", n_reads=1)
    g = w.genome
    test = gen.sample_reads(g, args.regime_reads, 81, [100], 0.0, 0.05)
    train = gen.sample_reads(g, 2 * args.regime_reads, 82, [100], 0.0, 0.05)
    wt = gen.Workload("bacterial-low-divergence", g, test, F=w.F, max_read_len=100)
    tw = gen.Workload("bacterial-low-divergence-train", g, train, F=w.F, max_read_len=100)
    ix = mx.Index(g.seq, w.F, 100, w.M, w.X, w.gap)
    seq = torch.from_numpy(test.seq).to(dev)
    off = torch.from_numpy(test.offsets.astype(np.int64)).to(dev)
    top = torch.empty(test.n * 32, dtype=torch.uint8, device=dev)
    res = proposal_leg(ix, wt, seq, off, top, stream, args, tw=tw, name="low divergence")
    res["workload"] = ("bacterial genome, %d reads of 100 bp, 0-5%% substitutions, no indels, "
                       "both strands" % test.n)
    ix.close()
    return res


def fast_leg(w, seq, off, top_full, full_scan_ms, stream):
    """MaxSSmap_fast (every other read base scored): scan time against the
    full scan's on the same reads, and top-1 agreement with the full scan."""
    import numpy as np
    import torch

    import paper_1403_2136_amd as mx
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap, flags=mx.MAXSS_FAST)
    n = w.reads.n
    out = torch.empty(n * 32, dtype=torch.uint8, device="cuda")
    ix.scan(seq, off, out, stream=stream)
    torch.cuda.synchronize()
    mx.maxss_profile_enable(True)
    ix.scan(seq, off, out, stream=stream)
    torch.cuda.synchronize()
    ms, k = mx.maxss_profile_read("scan")
    mx.maxss_profile_enable(False)
    got = out.cpu().numpy().view(mx.TOP2_DTYPE)
    ref = top_full.cpu().numpy().view(mx.TOP2_DTYPE)
    half = (w.reads.lengths().astype(np.int64) + 1) // 2
    cells = 2.0 * w.genome.G * float(half.sum())
    ix.close()
    res = {"scan_ms_per_launch": round(ms / max(k, 1), 3),
           "full_scan_ms_per_launch": round(full_scan_ms, 3),
           "speedup": round(full_scan_ms / (ms / max(k, 1)), 3),
           "fast_gcups_kernel": round(cells / (ms / max(k, 1) / 1e3) / 1e9, 1),
           "top1_agreement": round(float((got["frag"][:, 0] == ref["frag"][:, 0]).mean()), 5)}
    log("fast: %s" % res)
    return res


def qual_leg(w, seq, off, full_scan_ms, stream, scale: int = 10):
    """Base-quality scoring (position-specific scores from synthetic Phred
    qualities at 1/scale resolution): scan time against the plain scan's on
    the same reads, and the share of reads whose bases all map to one
    (match, mismatch) pair (the register-bank launch of the quality split;
    the others take the position-specific kernel)."""
    import numpy as np
    import torch

    import gen
    import paper_1403_2136_amd as mx
    qh = gen.sample_qualities(w.reads, 91)
    q = torch.from_numpy(qh).cuda()
    # the score table's rule: x = 1 - 10^(-Q/10), pair = (round(M x scale),
    # round(X x scale / 3)), halves away from zero
    x = 1.0 - 10.0 ** (-(qh.astype(np.float64) - 33) / 10.0)
    rnd = lambda v: np.sign(v) * np.floor(np.abs(v) + 0.5)
    pair = rnd(w.M * x * scale) * 256 + rnd(w.X * x * scale / 3.0)
    starts = w.reads.offsets[:-1].astype(np.int64)
    first = np.repeat(pair[starts], w.reads.lengths().astype(np.int64))
    diff = np.add.reduceat((pair != first).astype(np.int64), starts)
    one_pair = float((diff == 0).mean())
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap, qual_scale=scale)
    n = w.reads.n
    out = torch.empty(n * 32, dtype=torch.uint8, device="cuda")
    ix.scan(seq, off, out, stream=stream, qual=q)
    torch.cuda.synchronize()
    mx.maxss_profile_enable(True)
    ix.scan(seq, off, out, stream=stream, qual=q)
    torch.cuda.synchronize()
    ms, k = mx.maxss_profile_read("scan")
    mx.maxss_profile_enable(False)
    ix.close()
    cells = 2.0 * w.genome.G * float(w.reads.lengths().astype(np.int64).sum())
    res = {"qual_scale": scale, "scan_ms_per_launch": round(ms / max(k, 1), 3),
           "plain_scan_ms_per_launch": round(full_scan_ms, 3),
           "gcups_kernel": round(cells / (ms / max(k, 1) / 1e3) / 1e9, 1),
           "slowdown": round((ms / max(k, 1)) / full_scan_ms, 3),
           "reads_with_one_score_pair": round(one_pair, 4)}
    log("qual: %s" % res)
    return res


def excl_leg(w, seq, off, top_full, full_scan_ms, stream):
    """Second-best fragment with the best one's neighbours left out: the
    reads whose plain second is a neighbour are scanned again.  Reports the
    scan kernel time of both passes against the plain scan and how many
    reads took the second pass."""
    import numpy as np
    import torch

    import paper_1403_2136_amd as mx
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap,
                  flags=mx.MAXSS_EXCLUDE_ADJACENT)
    n = w.reads.n
    out = torch.empty(n * 32, dtype=torch.uint8, device="cuda")
    ix.scan(seq, off, out, stream=stream)
    torch.cuda.synchronize()
    mx.maxss_profile_enable(True)
    ix.scan(seq, off, out, stream=stream)
    torch.cuda.synchronize()
    ms, k = mx.maxss_profile_read("scan")
    mx.maxss_profile_enable(False)
    ix.close()
    ref = top_full.cpu().numpy().view(mx.TOP2_DTYPE)
    got = out.cpu().numpy().view(mx.TOP2_DTYPE)
    f1, f2 = ref["frag"][:, 0].astype(np.int64), ref["frag"][:, 1].astype(np.int64)
    again = int(((f1 >= 0) & (f2 >= 0) & (np.abs(f2 - f1) == 1)).sum())
    res = {"scan_ms_both_passes": round(ms, 3), "scan_launches": k,
           "plain_scan_ms_per_launch": round(full_scan_ms, 3),
           "overhead": round(ms / full_scan_ms, 4), "reads_scanned_again": again,
           "reads": n, "second_changed": int((got["frag"][:, 1] != ref["frag"][:, 1]).sum())}
    log("exclude adjacent: %s" % res)
    return res


def scan_roofline(cells: float, scan_s: float, kind: int, knp: int, workload: str,
                  measured_peak):
    """Roofline object of the scan kernel: the fixed algorithmic unit (one
    16-bit lane operation per cell) against the packed 16-bit VALU peak
    derived from the chip's unit counts and clock; the kernel's own
    instruction count per cell is reported beside it."""
    import paper_1403_2136_amd as mx
    achieved = UNIT_OPS_PER_CELL * cells / scan_s / 1e12
    peak = INT16_PACKED_OPS / 1e12
    kops = mx.KERNEL_OPS_PER_CELL[kind]
    r = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2),
         "unit": "Tops/s", "frac": round(achieved / peak, 4),
         "traffic": recorded_traffic(workload),
         "unit_ops_per_cell": UNIT_OPS_PER_CELL,
         "cells_per_launch": cells,
         "kernel": {"np": knp, "variant": ["step-max", "two-step", "register-bank"][kind],
                    "ops_per_cell": kops,
                    "issue_frac": round(kops * cells / scan_s / 1e12 / peak, 4)}}
    if measured_peak:
        r["measured_peak"] = round(measured_peak / 1e12, 2)
        r["frac_of_measured_peak"] = round(achieved / (measured_peak / 1e12), 4)
    return r


def batched_run(name: str, args, steps: int, dev, measured_peak, budget_s: float,
                tune_tiles: bool = True):
    """The batched path on a chromosome-scale workload: one persistent scan
    launch per mixed-length batch, replayed from a captured HIP graph, tiles
    from the autotuner (parity-gated) unless tune_tiles is False.  One eager
    step with kernel events (also the warm-up), then up to `steps` graph
    steps, fewer when they would take more than budget_s; the first graph
    step includes the capture.  With steps = 0 the eager step is the timed
    one."""
    import numpy as np
    import torch

    import gen
    import paper_1403_2136_amd as mx
    t0 = time.time()
    w = gen.workload(name)
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap)
    n = w.reads.n
    log("%s: genome and index %.1fs" % (name, time.time() - t0))
    seq = torch.from_numpy(w.reads.seq).to(dev)
    off = torch.from_numpy(w.reads.offsets.astype(np.int64)).to(dev)
    top = torch.empty(n * 32, dtype=torch.uint8, device=dev)
    aln = torch.empty(n * 32, dtype=torch.uint8, device=dev)
    stride = 256
    cig = torch.empty(n * stride, dtype=torch.uint8, device=dev)
    cells = 2.0 * w.genome.G * float(w.reads.lengths().sum())
    t1 = time.time()
    tune = None
    if tune_tiles and args.tune_sample > 0:
        sample = w.reads.subset(np.arange(0, n, max(1, n // args.tune_sample))[:args.tune_sample])
        tune = ix.autotune(sample.seq, sample.offsets)
        log("%s: autotune %.1fs %s" % (name, time.time() - t1, tune))
    plan = mx.Plan(ix, capacity=n, pad=w.pad, cigar_stride=stride)
    stream = torch.cuda.Stream()

    def step(graph):
        with torch.cuda.stream(stream):
            plan.run(seq, off, top, aln, cig, stream=stream, graph=graph)

    mx.maxss_profile_enable(True)
    t2 = time.perf_counter()
    step(False)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t2
    scan_ms, scan_k = mx.maxss_profile_read("scan")
    nw_ms, nw_k = mx.maxss_profile_read("nw")
    other = {k: mx.maxss_profile_read(k) for k in ("encode", "merge", "rescan")}
    mx.maxss_profile_enable(False)
    log("%s: eager step %.1fs, scan kernel %.1f ms" % (name, t_eager, scan_ms))
    k = max(1, min(steps, int(budget_s / max(t_eager, 1e-3)))) if steps > 0 else 0
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for i in range(k):
        step(True)
        torch.cuda.synchronize()
        log("%s: timed graph step %d done" % (name, i))
    dt = time.perf_counter() - t3
    if k == 0:
        k, dt = 1, t_eager
    knp, kind = ix.kernel_info()
    scan_s = scan_ms / max(scan_k, 1) / 1e3
    res = {"workload": "%s: %d bp genome, F=%d (%d fragments), %d reads, lengths %d-%d, both "
                       "strands, match %d mismatch %d gap %d; step = scan + top-2 + NW" % (
                           name, w.genome.G, w.F, ix.NF, n, int(w.reads.lengths().min()),
                           int(w.reads.lengths().max()), w.M, w.X, w.gap),
           "gcups": round(cells / (dt / k) / 1e9, 2), "ms_per_step": round(dt / k * 1e3, 3),
           "steps": k, "eager_step_s": round(t_eager, 3),
           "reads_per_s": round(n / (dt / k), 1),
           "scan_gcups_kernel": round(cells / scan_s / 1e9, 1),
           "scan_ms_per_launch": round(scan_s * 1e3, 3),
           "nw_ms_per_launch": round(nw_ms / max(nw_k, 1), 3),
           "other_ms": {kk: round(v[0] / max(v[1], 1), 3) for kk, v in other.items()},
           "step_path": ("plan + hipGraph replay (capture in the first timed step)" if steps > 0
                         else "plan, one eager step with kernel events")
                        + (", autotuned tiles" if tune is not None else ", built-in tiles"),
           "autotune": tune,
           "roofline": scan_roofline(cells, scan_s, kind, knp, name, measured_peak)}
    plan.close()
    ix.close()
    return res, w


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bacterial",
                    choices=["tiny", "bacterial", "chromosome", "damaged"])
    ap.add_argument("--reads", type=int, default=None, help="override the read count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=6.0,
                    help="seconds per all-cores run of the oracle (three runs; the one-thread "
                         "runs take half as long each)")
    ap.add_argument("--no-proposal", action="store_true",
                    help="skip the learned-proposal leg (training + reads/s vs the full scan)")
    ap.add_argument("--no-qual", action="store_true",
                    help="skip the base-quality scoring leg")
    ap.add_argument("--no-fast", action="store_true",
                    help="skip the MaxSSmap_fast leg (every other read base scored)")
    ap.add_argument("--no-excl", action="store_true",
                    help="skip the leg that leaves the best fragment's neighbours out of the "
                         "second-best")
    ap.add_argument("--no-chromosome", action="store_true",
                    help="skip the chromosome-scale batched leg of the default run")
    ap.add_argument("--no-damaged", action="store_true",
                    help="skip the damaged-read leg (one eager step) of the default run")
    ap.add_argument("--batched-budget", type=float, default=60.0,
                    help="seconds of timed graph steps on a chromosome-scale workload (the "
                         "step count is lowered to fit)")
    ap.add_argument("--tune-sample", type=int, default=256,
                    help="reads the autotuner times each tile shape on")
    ap.add_argument("--train-reads", type=int, default=200_000)
    ap.add_argument("--damaged-train-reads", type=int, default=22_000,
                    help="training + validation reads of the damaged workload's proposal leg "
                         "(labels cost a full scan of the 248 Mbp genome each)")
    ap.add_argument("--train-steps", type=int, default=10_000)
    ap.add_argument("--train-lr", type=float, default=3e-3)
    ap.add_argument("--hard-negatives", type=int, default=32)
    ap.add_argument("--regime-reads", type=int, default=100_000,
                    help="reads of the low-divergence proposal leg (0: skip it)")
    ap.add_argument("--K", type=int, default=64)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (the "
                         "known-size kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the MaxSS scan shards by reads with no "
              "collective, and the benchmark reports the single-GPU rate (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_1403_2136_amd as mx

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 3}))
        return
    measured_peak = mx.maxss_roof_int16()
    log("measured packed 16-bit add rate: %.2f T lane-ops/s" % (measured_peak / 1e12))
    base = {
        "metric": "MaxSS GCUPS; reads/s, learned-proposal vs full scan at >=99% top-1 agreement",
        "unit": "GCUPS", "n_gpus": 1, "warmup": args.warmup, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int16", "data": "synthetic"}

    if args.workload in ("chromosome", "damaged"):
        # a chromosome-scale step takes tens of seconds: the timed steps are
        # capped to the batched budget
        bres, w = batched_run(args.workload, args, args.steps, dev, measured_peak,
                              args.batched_budget)
        res = dict(base, value=bres["gcups"], steps=bres["steps"], ms_per_step=bres["ms_per_step"],
                   config={k: v for k, v in bres.items() if k not in ("gcups", "roofline")},
                   roofline=bres["roofline"])
        res["config"]["steps_requested"] = args.steps
        if not args.no_proposal and w.name == "damaged":
            ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap)
            seq = torch.from_numpy(w.reads.seq).to(dev)
            off = torch.from_numpy(w.reads.offsets.astype(np.int64)).to(dev)
            top = torch.empty(w.reads.n * 32, dtype=torch.uint8, device=dev)
            res["proposal"] = proposal_leg(ix, w, seq, off, top, torch.cuda.current_stream(),
                                           args)
            ix.close()
        if not args.no_cpu_baseline:
            log("cpu baseline (oracle) ...")
            res["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
        print(json.dumps(res), flush=True)
        return

    t0 = time.time()
    w = gen.workload(args.workload, n_reads=args.reads)
    log("workload %s: G=%d reads=%d (%.1fs)" % (w.name, w.genome.G, w.reads.n, time.time() - t0))
    ix = mx.Index(w.genome.seq, w.F, w.max_read_len, w.M, w.X, w.gap)
    n = w.reads.n
    seq = torch.from_numpy(w.reads.seq).to(dev)
    off = torch.from_numpy(w.reads.offsets.astype(np.int64)).to(dev)
    top = torch.empty(n * 32, dtype=torch.uint8, device=dev)
    aln = torch.empty(n * 32, dtype=torch.uint8, device=dev)
    stride = 256
    cig = torch.empty(n * stride, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    G = w.genome.G
    cells = 2.0 * G * float(w.reads.lengths().sum())

    def step():
        ix.scan(seq, off, top, stream=stream)
        ix.align(seq, off, top, w.pad, stride, aln, cig, stream=stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup %d done" % i)
    mx.maxss_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    scan_ms, scan_k = mx.maxss_profile_read("scan")
    nw_ms, nw_k = mx.maxss_profile_read("nw")
    other = {k: mx.maxss_profile_read(k) for k in ("encode", "merge", "rescan")}
    mx.maxss_profile_enable(False)
    log("timed %d steps in %.3fs; scan kernel %.3f ms/launch, nw %.3f ms/launch, %s" % (
        args.steps, dt, scan_ms / max(scan_k, 1), nw_ms / max(nw_k, 1),
        {k: round(v[0] / max(v[1], 1), 3) for k, v in other.items()}))
    ms_step = dt / args.steps * 1e3
    gcups = cells / (dt / args.steps) / 1e9
    scan_s = scan_ms / max(scan_k, 1) / 1e3
    knp, kind = ix.kernel_info()
    res = dict(base, value=round(gcups, 2), steps=args.steps, ms_per_step=round(ms_step, 3))
    res["config"] = {
        "workload": "%s: %d bp genome, F=%d (%d fragments), %d reads, lengths %d-%d, both "
                    "strands, match %d mismatch %d gap %d; step = scan + top-2 + NW" % (
                        w.name, G, w.F, ix.NF, n, int(w.reads.lengths().min()),
                        int(w.reads.lengths().max()), w.M, w.X, w.gap),
        "reads_per_s": round(n / (dt / args.steps), 1),
        "scan_gcups_kernel": round(cells / scan_s / 1e9, 1),
        "scan_ms_per_launch": round(scan_s * 1e3, 3),
        "nw_ms_per_launch": round(nw_ms / max(nw_k, 1), 3),
        "other_ms": {k: round(v[0] / max(v[1], 1), 3) for k, v in other.items()},
        "step_path": "maxss_scan_reads + maxss_align_top",
    }
    res["roofline"] = scan_roofline(cells, scan_s, kind, knp, w.name, measured_peak)
    # PCIe-inclusive: one scan of host buffers (reads copied in, records
    # copied out inside the call); reported beside, never as, the value
    t0 = time.perf_counter()
    ix.scan(w.reads.seq, w.reads.offsets)
    t_e2e = time.perf_counter() - t0
    res["config"]["scan_host_buffers_s"] = round(t_e2e, 3)
    res["config"]["scan_host_buffers_gcups"] = round(cells / t_e2e / 1e9, 1)
    if not args.no_fast:
        res["fast"] = fast_leg(w, seq, off, top, scan_s * 1e3, stream)
    if not args.no_qual:
        res["qual"] = qual_leg(w, seq, off, scan_s * 1e3, stream)
    if not args.no_excl:
        res["exclude_adjacent"] = excl_leg(w, seq, off, top, scan_s * 1e3, stream)
    if not args.no_proposal and w.name == "bacterial":
        res["proposal"] = proposal_leg(ix, w, seq, off, top, stream, args)
    ix.close()
    if not args.no_proposal and w.name == "bacterial" and args.regime_reads:
        res["proposal_low_divergence"] = proposal_regime_leg(args, dev, stream)
    del seq, off, top, aln, cig
    if not args.no_chromosome and w.name == "bacterial":
        # the batched path at chromosome scale: one eager and one graph step
        bres, _ = batched_run("chromosome", args, 1, dev, measured_peak, args.batched_budget)
        res["chromosome"] = bres
    if not args.no_damaged and w.name == "bacterial":
        # the damaged short reads on the same genome: one eager plan step,
        # built-in tiles
        dres, _ = batched_run("damaged", args, 0, dev, measured_peak, args.batched_budget,
                              tune_tiles=False)
        res["damaged"] = dres
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
