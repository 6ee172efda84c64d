"""Expected top-2 records for sampled reads of the two full-size 248 Mbp
workloads (chromosome: lengths 36/51/100/150/250; damaged: 36-80 bp), written
by the oracle alone into fullsize_records.json.

Run from the repository root:  python tests/golden/make_fullsize_records.py

Sample: per workload, reads drawn uniformly plus reads whose sampled span
overlaps a repeat-family copy (the generator records every copy it places).
Chromosome: 10 per length class, 3 of them from repeat copies; damaged: 24,
8 of them from repeat copies.

Oracle use: a fragment's value depends only on the bases of its extended
window [f*F, f*F + F + E - 1), E = max_read_len, so the oracle scans genome
slices of whole fragments (plus that extension) in parallel threads and the
per-fragment values are stitched together.  The top-2 comes from the oracle's
top-2 rule over those values (value desc, id asc), and each winner's
representative strand and offset from an oracle scan of that fragment's
extended window alone, whose fragment 0 is the winner.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402
from oracle import mlp  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_records.json")


def reads_sha256(r) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(r.offsets, dtype=np.uint64).tobytes())
    h.update(np.ascontiguousarray(r.seq, dtype=np.uint8).tobytes())
    return h.hexdigest()


def in_repeat(genome, r):
    """Per read: does its sampled span overlap a placed repeat copy?"""
    placed = np.array([(p, L) for p, L, _, _ in genome.info["placed"]], dtype=np.int64)
    order = np.argsort(placed[:, 0])
    starts, ends = placed[order, 0], placed[order, 0] + placed[order, 1]
    run_end = np.maximum.accumulate(ends)
    a, b = r.start, r.start + r.span
    k = np.searchsorted(starts, b, side="left") - 1        # last copy starting before b
    ok = k >= 0
    return ok & (run_end[np.maximum(k, 0)] > a)


def choose(w, seed):
    st = gen.Stream(seed, "fullsize.sample")
    lens = w.reads.lengths()
    rep = in_repeat(w.genome, w.reads)
    if w.name == "chromosome":
        classes = [[c] for c in np.unique(lens)]
        n_uni, n_rep = 7, 3
    else:
        classes = [np.unique(lens)]
        n_uni, n_rep = 16, 8
    idx = []
    for c in classes:
        inc = np.isin(lens, c)
        for pool, k in ((np.nonzero(inc & ~rep)[0], n_uni), (np.nonzero(inc & rep)[0], n_rep)):
            pick = []
            while len(pick) < k:
                j = int(pool[st.integers(0, pool.size, 1)[0]])
                if j not in pick and j not in idx:
                    pick.append(j)
            idx.extend(pick)
    return np.array(sorted(idx), dtype=np.int64), rep


def sliced_values(genome, F, E, sub, M, X, nslices):
    G = genome.size
    NF = (G + F - 1) // F
    bounds = np.linspace(0, NF, nslices + 1).astype(np.int64)
    vals = np.zeros((sub.n, NF), dtype=np.int32)
    errors = []

    def work(k):
        try:
            a, b = int(bounds[k]), int(bounds[k + 1])
            if a == b:
                return
            lo, hi = a * F, min(G, b * F + E - 1)
            _, v = oracle.scan(genome[lo:hi], F, sub.seq, sub.offsets, M, X, nthreads=1,
                               want_values=True)
            vals[:, a:b] = v[:, :b - a]
        except Exception as e:  # re-raised below
            errors.append(e)

    th = [threading.Thread(target=work, args=(k,)) for k in range(nslices)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    if errors:
        raise errors[0]
    return vals


def representative(genome, F, E, read, f, M, X):
    """(value, strand, offset) of fragment f from an oracle scan of its
    extended window alone (fragment 0 of that slice)."""
    G = genome.size
    lo, hi = f * F, min(G, f * F + F + E - 1)
    off = np.array([0, len(read)], dtype=np.uint64)
    rec, v = oracle.scan(genome[lo:hi], F, read, off, M, X, nthreads=1, want_values=True)
    slot = [k for k in range(2) if int(rec["frag"][0][k]) == 0]
    assert slot, (f, rec)
    k = slot[0]
    return int(v[0, 0]), int(rec["strand"][0][k]), int(rec["offset"][0][k])


def records(w, idx, nslices):
    sub = w.reads.subset(idx)
    E = w.max_read_len
    vals = sliced_values(w.genome.seq, w.F, E, sub, w.M, w.X, nslices)
    NF = vals.shape[1]
    out = []
    allf = np.arange(NF)
    for i in range(sub.n):
        f1, s1, f2, s2 = mlp.top2_among(vals[i], allf)
        row = {"frag": [f1, f2], "score": [s1, s2], "offset": [], "strand": []}
        for f, s in ((f1, s1), (f2, s2)):
            v, st, o = representative(w.genome.seq, w.F, E, sub.read(i), f, w.M, w.X)
            assert v == s, (i, f, v, s)
            row["strand"].append(st)
            row["offset"].append(o)
        out.append(row)
    return out


def main():
    nslices = max(1, os.cpu_count() or 1)
    res = {"description": "oracle top-2 records of sampled reads of the full-size workloads "
                          "(written by make_fullsize_records.py)"}
    for name, seed in (("chromosome", 901), ("damaged", 902)):
        t0 = time.time()
        w = gen.workload(name)
        idx, rep = choose(w, seed)
        print("%s: %d reads sampled (%d from repeat copies); oracle on %d slices" % (
            name, idx.size, int(rep[idx].sum()), nslices), flush=True)
        recs = records(w, idx, nslices)
        res[name] = {"G": int(w.genome.G), "F": w.F, "n_reads": w.reads.n,
                     "reads_sha256": reads_sha256(w.reads),
                     "index": idx.tolist(), "from_repeat_copy": rep[idx].astype(int).tolist(),
                     "records": recs}
        print("%s: done in %.0f s" % (name, time.time() - t0), flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
