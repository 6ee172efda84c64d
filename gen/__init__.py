"""Seeded synthetic genomes and reads for the MaxSS scan workloads.

This module is shared by the tests, the benchmark and the smoke check as the
one source of inputs.  It holds none of the method's arithmetic (no scoring,
no scan, no alignment): it only draws bases, reads, substitutions, indels and
damage from a counter-based generator, so that the oracle and the GPU path see
byte-identical inputs.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used in counter mode: draw i of
stream (seed, name) is mix64(key(seed, name) + (i+1) * 0x9E3779B97F4A7C15),
where mix64 is SplitMix64's output function.  Streams are independent of the
order in which they are consumed, so every array is reproducible on its own.

The workloads stand in for the paper's data (simulated E. coli K-12 and human
chromosome 1 reads, ancient horse reads), which are not available; the shapes,
sizes and distributions follow the five workload descriptions:

  tiny        50,000 bp uniform genome, F=2,048, 200 x 100 bp reads, 10%
              substitutions, no gaps.
  bacterial   4.6 Mbp genome at 50% GC plus 1% of its length as inserted exact
              1-5 kbp repeats, F=2,048, 100,000 x 100 bp reads, 10-30%
              substitutions, 0-2 indels of length 1-30 (read or genome side).
  chromosome  248 Mbp at 41% GC with 5% of bases from 50 repeat families
              (300-6,000 bp consensus, 0-15% copy divergence), F=4,096, 20,000
              reads of lengths {36,51,100,150,250} in equal proportion.
  proposal    bacterial genome; 200,000 training reads (own seed); the
              bacterial reads are the test set.
  damaged     chromosome genome; 50,000 reads of length 36-80, 15-30%
              substitutions, C->T at the 5' end and G->A at the 3' end at rate
              0.3 decaying linearly over 10 bases, 0-1 indels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

_GOLD = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)


def _mix64(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _fnv1a(s: str) -> int:
    h = 0xCBF29CE484222325
    for ch in s.encode():
        h = ((h ^ ch) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


class Stream:
    """Counter-mode SplitMix64 stream keyed by (seed, name)."""

    def __init__(self, seed: int, name: str):
        k = np.array([(seed * 0x9E3779B97F4A7C15 + _fnv1a(name)) & 0xFFFFFFFFFFFFFFFF],
                     dtype=np.uint64)
        self.key = _mix64(k)[0]
        self.ctr = 0

    def u64(self, n: int) -> np.ndarray:
        idx = np.arange(self.ctr + 1, self.ctr + 1 + n, dtype=np.uint64)
        self.ctr += n
        with np.errstate(over="ignore"):
            return _mix64(self.key + idx * _GOLD)

    def uniform(self, n: int) -> np.ndarray:
        """Doubles in [0, 1) from the top 53 bits."""
        return (self.u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def integers(self, lo: int, hi: int, n: int) -> np.ndarray:
        """Integers in [lo, hi) (hi - lo << 2^53, so the bias is negligible)."""
        return lo + np.floor(self.uniform(n) * (hi - lo)).astype(np.int64)


def random_bases(st: Stream, n: int, gc: float = 0.5, chunk: int = 1 << 24) -> np.ndarray:
    """n i.i.d. bases (ASCII) with P(C)=P(G)=gc/2, P(A)=P(T)=(1-gc)/2."""
    out = np.empty(n, dtype=np.uint8)
    a = (1.0 - gc) / 2.0
    cut = np.array([a, 0.5, 0.5 + gc / 2.0])  # A | C | G | T
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        u = st.uniform(e - s)
        out[s:e] = ACGT[np.searchsorted(cut, u, side="right")]
    return out


_COMP = np.zeros(256, dtype=np.uint8)
for _a, _b in zip(b"ACGTN", b"TGCAN"):
    _COMP[_a] = _b


def _revcomp(a: np.ndarray) -> np.ndarray:
    return _COMP[a[::-1]]


def substitute(st: Stream, seq: np.ndarray, rate) -> np.ndarray:
    """Each base independently, with probability `rate` (scalar or per-base
    array), replaced by one of the three other bases uniformly."""
    seq = seq.copy()
    u = st.uniform(seq.size)
    hit = u < rate
    code = np.full(256, 0, dtype=np.int64)
    code[ACGT] = np.arange(4)
    shift = st.integers(1, 4, seq.size)
    newc = (code[seq] + shift) % 4
    seq[hit] = ACGT[newc[hit]]
    return seq


@dataclass
class Genome:
    seq: np.ndarray          # uint8 ASCII
    name: str
    info: dict = field(default_factory=dict)

    @property
    def G(self) -> int:
        return int(self.seq.size)


@dataclass
class Reads:
    seq: np.ndarray          # uint8 ASCII, CSR-concatenated
    offsets: np.ndarray      # uint64, n+1 entries
    start: np.ndarray        # int64 true genome start of the sampled span
    span: np.ndarray         # int64 genome bases covered
    strand: np.ndarray       # int8 0 = forward, 1 = reverse complement
    rate: np.ndarray         # float64 substitution rate
    n_indel: np.ndarray      # int8

    @property
    def n(self) -> int:
        return int(self.offsets.size - 1)

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def read(self, i: int) -> bytes:
        return self.seq[int(self.offsets[i]):int(self.offsets[i + 1])].tobytes()

    def subset(self, idx) -> "Reads":
        idx = np.asarray(idx, dtype=np.int64)
        parts = [self.seq[int(self.offsets[i]):int(self.offsets[i + 1])] for i in idx]
        lens = np.array([p.size for p in parts], dtype=np.uint64)
        off = np.zeros(idx.size + 1, dtype=np.uint64)
        off[1:] = np.cumsum(lens)
        seq = np.concatenate(parts) if parts else np.zeros(0, dtype=np.uint8)
        return Reads(seq, off, self.start[idx], self.span[idx], self.strand[idx],
                     self.rate[idx], self.n_indel[idx])


# ------------------------------------------------------------------ genomes

def uniform_genome(G: int, seed: int, gc: float = 0.5) -> Genome:
    st = Stream(seed, "genome.bases")
    return Genome(random_bases(st, G, gc), "uniform", dict(gc=gc, seed=seed))


def bacterial_genome(seed: int, base_len: int = 4_600_000, gc: float = 0.5,
                     repeat_frac: float = 0.01, rep_lo: int = 1000,
                     rep_hi: int = 5000) -> Genome:
    """i.i.d. sequence, then exact copies of random existing segments of length
    U[rep_lo, rep_hi] inserted at random positions until >= repeat_frac of the
    base length has been inserted."""
    base = random_bases(Stream(seed, "genome.bases"), base_len, gc)
    st = Stream(seed, "genome.repeats")
    target = int(repeat_frac * base_len)
    ev = []
    tot = 0
    while tot < target:
        L = int(st.integers(rep_lo, rep_hi + 1, 1)[0])
        src = int(st.integers(0, base_len - L + 1, 1)[0])
        dst = int(st.integers(0, base_len + 1, 1)[0])
        ev.append((dst, src, L))
        tot += L
    ev.sort()
    parts, cur = [], 0
    for dst, src, L in ev:
        parts.append(base[cur:dst])
        parts.append(base[src:src + L])
        cur = dst
    parts.append(base[cur:])
    seq = np.concatenate(parts)
    return Genome(seq, "bacterial", dict(seed=seed, inserted=tot, n_repeats=len(ev),
                                         repeats=ev, gc=gc))


def chromosome_genome(seed: int, G: int = 248_000_000, gc: float = 0.41, families: int = 50,
                      cons_lo: int = 300, cons_hi: int = 6000, div_hi: float = 0.15,
                      repeat_frac: float = 0.05) -> Genome:
    """i.i.d. sequence; `families` consensus sequences of length U[cons_lo,
    cons_hi]; copies with substitution divergence U[0, div_hi] overwrite random
    positions until >= repeat_frac of the bases are repeat-derived."""
    seq = random_bases(Stream(seed, "genome.bases"), G, gc)
    stf = Stream(seed, "genome.families")
    cons = []
    for _ in range(families):
        L = int(stf.integers(cons_lo, cons_hi + 1, 1)[0])
        cons.append(random_bases(stf, L, gc))
    st = Stream(seed, "genome.copies")
    target = int(repeat_frac * G)
    tot = n = 0
    placed = []     # (position, length, family, divergence) of every copy
    while tot < target:
        fam = int(st.integers(0, families, 1)[0])
        d = float(st.uniform(1)[0]) * div_hi
        c = substitute(st, cons[fam], d)
        pos = int(st.integers(0, G - c.size + 1, 1)[0])
        seq[pos:pos + c.size] = c
        placed.append((pos, int(c.size), fam, d))
        tot += c.size
        n += 1
    return Genome(seq, "chromosome", dict(seed=seed, gc=gc, repeat_bases=tot, copies=n,
                                          placed=placed))


def with_n_runs(g: Genome, seed: int, runs: int, run_lo: int = 1, run_hi: int = 200) -> Genome:
    """Copy of g with `runs` runs of N of length U[run_lo, run_hi] (edge cases)."""
    seq = g.seq.copy()
    st = Stream(seed, "genome.nruns")
    for _ in range(runs):
        L = int(st.integers(run_lo, run_hi + 1, 1)[0])
        p = int(st.integers(0, max(1, g.G - L + 1), 1)[0])
        seq[p:p + L] = ord("N")
    return Genome(seq, g.name + "+N", dict(g.info, n_runs=runs))


# -------------------------------------------------------------------- reads

def sample_reads(genome: Genome, n: int, seed: int, lengths, rate_lo: float, rate_hi: float,
                 indel_max: int = 0, indel_len_hi: int = 30, damage: bool = False,
                 length_mode: str = "choice") -> Reads:
    """Reads from random positions and strands.

    Per read, in this order: a genome span, indels (count U{0..indel_max},
    length U{1..indel_len_hi}, 50/50 read-side insertion of random bases or
    genome-side deletion, at uniform interior read positions), substitutions
    at a per-read rate U[rate_lo, rate_hi] (each base to one of the three others
    uniformly), reverse complement for strand 1, then optional ancient-DNA
    damage (C->T at distance d < 10 from the 5' end, G->A at distance d < 10
    from the 3' end, each with probability 0.3 * (1 - d/10)).
    `lengths`: a list to choose from uniformly (length_mode "choice") or an
    inclusive (lo, hi) range (length_mode "range")."""
    G = genome.G
    st = Stream(seed, "reads.meta")
    if length_mode == "choice":
        lens_c = np.asarray(lengths, dtype=np.int64)
        m = lens_c[st.integers(0, lens_c.size, n)]
    else:
        m = st.integers(int(lengths[0]), int(lengths[1]) + 1, n)
    strand = (st.uniform(n) < 0.5).astype(np.int8)
    rate = rate_lo + st.uniform(n) * (rate_hi - rate_lo)
    n_ind = st.integers(0, indel_max + 1, n).astype(np.int8) if indel_max > 0 else np.zeros(n, np.int8)
    sti = Stream(seed, "reads.indels")
    stp = Stream(seed, "reads.start")
    stb = Stream(seed, "reads.insert_bases")
    pieces = []
    start = np.zeros(n, dtype=np.int64)
    span = np.zeros(n, dtype=np.int64)
    # draw a fixed number of values per read so every read's draws are fixed
    ev_len = sti.integers(1, indel_len_hi + 1, 2 * n).reshape(n, 2)
    ev_side = (sti.uniform(2 * n) < 0.5).reshape(n, 2)      # True: read-side insertion
    ev_pos_u = sti.uniform(2 * n).reshape(n, 2)
    u_start = stp.uniform(n)
    for i in range(n):
        mi = int(m[i])
        evs = []
        for e in range(int(n_ind[i])):
            rpos = 1 + int(ev_pos_u[i, e] * max(1, mi - 1))   # interior read position
            evs.append((rpos, bool(ev_side[i, e]), int(ev_len[i, e])))
        evs.sort()
        dels = sum(L for _, ins, L in evs if not ins)
        need = mi + dels
        s0 = int(u_start[i] * (G - need + 1))
        start[i] = s0
        out, c, emitted = [], s0, 0
        for rpos, ins, L in evs:
            rpos = max(rpos, emitted)
            take = min(rpos, mi) - emitted
            if take > 0:
                out.append(genome.seq[c:c + take]); c += take; emitted += take
            if emitted >= mi:
                break
            if ins:
                L = min(L, mi - emitted)
                out.append(random_bases(stb, L, 0.5)); emitted += L
            else:
                c += L
        if emitted < mi:
            out.append(genome.seq[c:c + (mi - emitted)]); c += mi - emitted
        span[i] = c - s0
        pieces.append(np.concatenate(out) if len(out) > 1 else out[0].copy())
    lens = np.array([p.size for p in pieces], dtype=np.uint64)
    off = np.zeros(n + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens)
    seq = np.concatenate(pieces) if pieces else np.zeros(0, np.uint8)
    per_base_rate = np.repeat(rate, lens.astype(np.int64))
    seq = substitute(Stream(seed, "reads.subst"), seq, per_base_rate)
    # strand
    for i in np.nonzero(strand)[0]:
        a, b = int(off[i]), int(off[i + 1])
        seq[a:b] = _revcomp(seq[a:b])
    if damage:
        std = Stream(seed, "reads.damage")
        u5 = std.uniform(seq.size)
        u3 = std.uniform(seq.size)
        pos = np.arange(seq.size, dtype=np.int64)
        rid = np.repeat(np.arange(n), lens.astype(np.int64))
        d5 = pos - off[:-1].astype(np.int64)[rid]
        d3 = off[1:].astype(np.int64)[rid] - 1 - pos
        p5 = np.where(d5 < 10, 0.3 * (1.0 - d5 / 10.0), 0.0)
        p3 = np.where(d3 < 10, 0.3 * (1.0 - d3 / 10.0), 0.0)
        ct = (seq == ord("C")) & (u5 < p5)
        seq[ct] = ord("T")
        ga = (seq == ord("G")) & (u3 < p3)
        seq[ga] = ord("A")
    return Reads(seq, off, start, span, strand, rate, n_ind)


def sample_qualities(reads: Reads, seed: int, q_hi: int = 40, q_lo: int = 2) -> np.ndarray:
    """Phred base qualities for `reads` as Phred+33 ASCII (uint8, the same CSR
    layout as reads.seq).  Per base: 38 - 14 (d/m)^2 + 4 z rounded and clipped
    to [q_lo, q_hi], where d is the distance from the read's first base, m
    its length and z ~ N(0, 1) (Box-Muller on the seeded stream), so the
    quality falls along the read with noise."""
    st = Stream(seed, "reads.qual")
    lens = np.diff(reads.offsets.astype(np.int64))
    nb = int(lens.sum())
    u1 = np.maximum(st.uniform(nb), 1e-300)
    u2 = st.uniform(nb)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    rid = np.repeat(np.arange(lens.size), lens)
    d = np.arange(nb, dtype=np.int64) - reads.offsets[:-1].astype(np.int64)[rid]
    m = np.maximum(lens[rid], 1).astype(np.float64)
    q = np.rint(38.0 - 14.0 * (d / m) ** 2 + 4.0 * z)
    return (np.clip(q, q_lo, q_hi).astype(np.int64) + 33).astype(np.uint8)


# ---------------------------------------------------------------- workloads

@dataclass
class Workload:
    name: str
    genome: Genome
    reads: Reads
    F: int
    M: int = 1
    X: int = -1
    gap: int = -2
    pad: int = 100
    max_read_len: int = 100


_GENOME_CACHE: dict = {}


def _genome(kind: str, seed: int) -> Genome:
    key = (kind, seed)
    if key not in _GENOME_CACHE:
        if kind == "uniform50k":
            _GENOME_CACHE[key] = uniform_genome(50_000, seed)
        elif kind == "bacterial":
            _GENOME_CACHE[key] = bacterial_genome(seed)
        elif kind == "chromosome":
            _GENOME_CACHE[key] = chromosome_genome(seed)
        else:
            raise KeyError(kind)
    return _GENOME_CACHE[key]


def workload(name: str, n_reads: int | None = None, read_seed: int | None = None) -> Workload:
    """One of the five workloads, optionally with fewer reads (a prefix of the
    full read set is NOT guaranteed; use Reads.subset on the full set for that)."""
    if name == "tiny":
        g = _genome("uniform50k", 11)
        r = sample_reads(g, n_reads or 200, read_seed or 12, [100], 0.1, 0.1)
        return Workload(name, g, r, F=2048, max_read_len=100)
    if name == "bacterial":
        g = _genome("bacterial", 21)
        r = sample_reads(g, n_reads or 100_000, read_seed or 22, [100], 0.1, 0.3, indel_max=2)
        return Workload(name, g, r, F=2048, max_read_len=100)
    if name == "chromosome":
        g = _genome("chromosome", 31)
        r = sample_reads(g, n_reads or 20_000, read_seed or 32, [36, 51, 100, 150, 250],
                         0.1, 0.3, indel_max=2)
        return Workload(name, g, r, F=4096, max_read_len=250)
    if name == "proposal_train":
        g = _genome("bacterial", 21)
        r = sample_reads(g, n_reads or 200_000, read_seed or 42, [100], 0.1, 0.3, indel_max=2)
        return Workload(name, g, r, F=2048, max_read_len=100)
    if name == "damaged":
        g = _genome("chromosome", 31)
        r = sample_reads(g, n_reads or 50_000, read_seed or 52, (36, 80), 0.15, 0.30,
                         indel_max=1, damage=True, length_mode="range")
        return Workload(name, g, r, F=4096, max_read_len=80)
    raise KeyError(name)


# ------------------------------------------------- learned-proposal inputs

def mlp_init(seed: int, d: int = 256, hidden: int = 256) -> np.ndarray:
    """Initial parameters of the 512-256-1 proposal network (float32, layout
    W1 row-major, b1, w2, b2): W1 and w2 uniform in +-sqrt(6/(fan_in+fan_out))
    (Glorot & Bengio, 2010), biases 0."""
    st = Stream(seed, "mlp.init")
    a1 = np.sqrt(6.0 / (2 * d + hidden))
    a2 = np.sqrt(6.0 / (hidden + 1))
    W1 = (st.uniform(hidden * 2 * d) * 2 - 1) * a1
    w2 = (st.uniform(hidden) * 2 - 1) * a2
    return np.concatenate([W1, np.zeros(hidden), w2, [0.0]]).astype(np.float32)


def sample_negatives(seed: int, step: int, labels: np.ndarray, second: np.ndarray, NF: int,
                     n_neg: int = 63) -> np.ndarray:
    """Negative fragments for a batch (B, n_neg) int32: the second-best
    fragment first when it exists and differs from the label, then distinct
    uniform draws over the fragments other than the label (repeats only when
    fewer than n_neg other fragments exist)."""
    labels = np.asarray(labels, dtype=np.int64)
    second = np.asarray(second, dtype=np.int64)
    B = labels.size
    st = Stream(seed, "train.neg.%d" % step)
    D = n_neg + 48
    others = max(NF - 1, 1)
    x = st.integers(0, others, B * D).reshape(B, D)
    x = x + (x >= labels[:, None])                        # skip the label
    has2 = (second >= 0) & (second < NF) & (second != labels)
    # a draw is dropped when it repeats an earlier draw of its row or equals
    # the `second` already placed first; survivors keep their draw order
    order = np.argsort(x, axis=1, kind="stable")
    xs = np.take_along_axis(x, order, axis=1)
    drop_s = np.zeros_like(xs, dtype=bool)
    drop_s[:, 1:] = xs[:, 1:] == xs[:, :-1]
    drop = np.zeros_like(drop_s)
    np.put_along_axis(drop, order, drop_s, axis=1)
    drop |= (x == second[:, None]) & has2[:, None]
    pos = np.arange(D)[None, :]
    keep = np.argsort(np.where(drop, D + pos, pos), axis=1, kind="stable")
    x = np.where(np.take_along_axis(drop, keep, axis=1), NF, np.take_along_axis(x, keep, axis=1))
    out = np.empty((B, n_neg), dtype=np.int64)
    out[:, 0] = np.where(has2, second, x[:, 0])
    out[:, 1:] = np.where(has2[:, None], x[:, :n_neg - 1], x[:, 1:n_neg])
    bad = out >= NF                                        # tiny genomes: too few fragments
    if bad.any():
        for b in np.nonzero(bad.any(axis=1))[0]:
            pool = [f for f in range(NF) if f != labels[b]] or [int(labels[b])]
            out[b] = [pool[k % len(pool)] for k in range(n_neg)]
    return out.astype(np.int32)
