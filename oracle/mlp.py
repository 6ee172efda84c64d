"""Float64 oracle of the learned fragment proposal -- TEST INFRASTRUCTURE ONLY.

The paper has no learned component.  These functions define, plainly and in
float64, the proposal added on top of the exact scan; the GPU path
must match them within the tolerances derived in the tests.  Only `tests/`,
the smoke check and the benchmark's CPU-baseline leg may import this module.

Definitions:
  * 4-mer profile of a sequence x: c[j] = number of positions t such that
    x[t..t+3] holds no N and j = 64 x[t] + 16 x[t+1] + 4 x[t+2] + x[t+3]
    (A 0, C 1, G 2, T 3); v = c / ||c||_2, or 0 when every count is 0.
    Read profiles are taken per strand; a fragment's profile counts the
    4-mers that *start* in [fF, fF+F) (bases past the genome end are N).
  * bf16(x): round x to float32 (nearest even), then to bfloat16 (nearest
    even on the 16 dropped bits).  Weights and profiles enter the network
    in bf16.
  * MLP: z = [v_read ; v_frag] (512), h = ReLU(W1 z + b1) (W1: 256 x 512),
    y = w2 . h + b2.  Parameters, flattened in this order: W1 (row-major),
    b1, w2, b2 -- 131,585 numbers.
  * Decomposed form used for inference: W1 z = W1[:, :256] v_read +
    W1[:, 256:] v_frag.
  * Training loss per read: softmax cross-entropy over its 64 candidate
    fragments, the label fragment at position 0; the batch loss is the mean.
  * Adam (Kingma & Ba, 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    theta -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
  * Proposal: s_f = max over strands of y(read strand profile, fragment f);
    order by (s desc, f asc); the K first are the candidates; margin =
    s_(1) - s_(2); a read falls back to the full scan when margin < tau.
  * Random numbers of the training (the builder's design, stated in the
    library's header): SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) in
    counter mode, draw k of stream s under a seed = mix64(key + (k+1) gamma),
    key = mix64(seed gamma + s), gamma = 0x9E3779B97F4A7C15; unit double =
    top 53 bits / 2^53; integer in [0, n) = floor(unit n).  Streams: 1
    initial weights, 2 negatives, 16 + e read order of epoch e.
  * Initial weights: Glorot uniform (W1 element i = (2u_i - 1) sqrt(6/768),
    w2 element k = (2u_{131072+k} - 1) sqrt(6/257), biases 0) or the
    profile-matching start (W1[k][k] = 8, W1[k][256+k] = 1, b1 = -0.2,
    w2 = 1, b2 = 0).
  * Training batches: epoch e orders the labelled training reads by (draw r
    of stream 16+e, r); step t takes positions t B .. t B + B - 1 of the
    epochs laid end to end.  Candidates of slot b: the label, the second
    best (if it is another fragment), distinct uniform draws over the other
    fragments (draw (t B + b) 512 + k of stream 2, k < 512; f = floor(u
    (NF-1)), plus 1 when f >= label) up to 63 negatives, then the other
    fragments in increasing order, then the negatives found repeated.
"""
from __future__ import annotations

import numpy as np

D = 256             # profile dimension (4^4)
H = 256             # hidden units
N_PARAMS = H * 2 * D + H + H + 1   # 131,585

_CODE = np.full(256, 4, dtype=np.int64)
for _i, _c in enumerate(b"ACGT"):
    _CODE[_c] = _i
    _CODE[ord(chr(_c).lower())] = _i
_COMP = {0: 3, 1: 2, 2: 1, 3: 0, 4: 4}


def codes(seq) -> np.ndarray:
    a = np.frombuffer(bytes(seq), dtype=np.uint8) if not isinstance(seq, np.ndarray) else seq
    return _CODE[a.astype(np.int64)]


def kmer_counts(c: np.ndarray) -> np.ndarray:
    """Counts of 4-mers without N in a code array (plain loop)."""
    out = np.zeros(D, dtype=np.int64)
    for t in range(len(c) - 3):
        w = c[t:t + 4]
        if (w == 4).any():
            continue
        out[64 * w[0] + 16 * w[1] + 4 * w[2] + w[3]] += 1
    return out


def normalise(cnt: np.ndarray) -> np.ndarray:
    n = float(np.sqrt(np.sum(cnt.astype(np.float64) ** 2)))
    return cnt.astype(np.float64) / n if n > 0 else np.zeros(D)


def read_profiles(read) -> np.ndarray:
    """(2, 256): forward strand, reverse complement."""
    c = codes(read)
    rc = np.array([_COMP[int(x)] for x in c[::-1]], dtype=np.int64)
    return np.stack([normalise(kmer_counts(c)), normalise(kmer_counts(rc))])


def fragment_profile(genome, F: int, f: int) -> np.ndarray:
    g = codes(genome)
    G = len(g)
    start = f * F
    ext = np.full(F + 3, 4, dtype=np.int64)
    seg = g[start:min(G, start + F + 3)]
    ext[:len(seg)] = seg
    return normalise(kmer_counts(ext))


def fragment_profiles(genome, F: int) -> np.ndarray:
    g = codes(genome)
    NF = (len(g) + F - 1) // F
    return np.stack([fragment_profile(genome, F, f) for f in range(NF)])


def bf16(x) -> np.ndarray:
    """Round to float32, then to bfloat16 (round to nearest, ties to even);
    returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    assert p.size == N_PARAMS
    W1 = p[:H * 2 * D].reshape(H, 2 * D)
    b1 = p[H * 2 * D:H * 2 * D + H]
    w2 = p[H * 2 * D + H:H * 2 * D + 2 * H]
    b2 = p[-1]
    return W1, b1, w2, b2


def pack(W1, b1, w2, b2) -> np.ndarray:
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(w2), [float(b2)]])


def shadow(params) -> np.ndarray:
    """The parameters as the network sees them: W1 and w2 in bf16, biases in
    float32."""
    W1, b1, w2, b2 = unpack(params)
    return pack(bf16(W1), np.asarray(b1, np.float32).astype(np.float64),
                bf16(w2), float(np.float32(b2)))


def forward(params, z: np.ndarray):
    """Plain MLP on z (P, 512): returns (y, pre-activation, h)."""
    W1, b1, w2, b2 = unpack(params)
    pre = z @ W1.T + b1
    h = np.maximum(pre, 0.0)
    return h @ w2 + b2, pre, h


def forward_decomposed(params, v_read: np.ndarray, v_frag: np.ndarray) -> np.ndarray:
    """y for every (read row, fragment row) pair: (R, Fn)."""
    W1, b1, w2, b2 = unpack(params)
    A = v_read @ W1[:, :D].T + b1          # (R, H)
    B = v_frag @ W1[:, D:].T               # (Fn, H)
    h = np.maximum(A[:, None, :] + B[None, :, :], 0.0)
    return h @ w2 + b2


def loss_and_grad(params, v_read: np.ndarray, v_cand: np.ndarray, parts: bool = False):
    """Mean softmax cross-entropy over reads.  v_read: (B, 256) profile of
    each read in its label strand; v_cand: (B, 64, 256) candidate fragment
    profiles, label first.  Returns (loss, y (B, 64), gradient (N_PARAMS,)),
    and with `parts` also a dict of the intermediate terms (z, pre, h, dy, dh)
    for error analysis."""
    W1, b1, w2, b2 = unpack(params)
    Bn, C, _ = v_cand.shape
    z = np.concatenate([np.repeat(v_read[:, None, :], C, axis=1), v_cand], axis=2)
    y, pre, h = forward(params, z.reshape(Bn * C, 2 * D))
    y = y.reshape(Bn, C)
    ymax = y.max(axis=1, keepdims=True)
    lse = ymax[:, 0] + np.log(np.exp(y - ymax).sum(axis=1))
    loss = float(np.mean(lse - y[:, 0]))
    p = np.exp(y - lse[:, None])
    dy = p.copy()
    dy[:, 0] -= 1.0
    dy /= Bn
    dyf = dy.reshape(-1)
    dw2 = h.T @ dyf
    db2 = dyf.sum()
    dh = np.outer(dyf, w2) * (pre > 0)
    db1 = dh.sum(axis=0)
    dW1 = dh.T @ z.reshape(Bn * C, 2 * D)
    g = pack(dW1, db1, dw2, db2)
    if parts:
        return loss, y, g, dict(z=z.reshape(Bn * C, 2 * D), pre=pre, h=h, dy=dyf, dh=dh)
    return loss, y, g


class Adam:
    def __init__(self, n: int, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = b1, b2, eps

    def step(self, theta: np.ndarray, g: np.ndarray, lr: float) -> np.ndarray:
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - lr * mh / (np.sqrt(vh) + self.eps)


def propose(scores: np.ndarray, K: int):
    """scores: (n, NF) per-fragment MLP scores (max over strands).  Returns
    (candidates (n, K) sorted by fragment id, margin (n,))."""
    n, NF = scores.shape
    K = min(K, NF)
    cands = np.zeros((n, K), dtype=np.int64)
    margin = np.zeros(n)
    for i in range(n):
        order = sorted(range(NF), key=lambda f: (-scores[i, f], f))
        cands[i] = sorted(order[:K])
        margin[i] = scores[i, order[0]] - scores[i, order[1]] if NF > 1 else np.inf
    return cands, margin


def top2_among(values: np.ndarray, cand) -> tuple:
    """Top-2 (fragment, value) among the candidate fragments by (value desc,
    id asc), from a row of exact fragment values."""
    order = sorted((int(f) for f in cand), key=lambda f: (-int(values[f]), f))
    f1 = order[0]
    f2 = order[1] if len(order) > 1 else -1
    return f1, int(values[f1]), f2, (int(values[f2]) if f2 >= 0 else -1)


# ----------------------------------------------------- training random numbers

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    """SplitMix64's output function (plain Python integers)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def sm_key(seed: int, stream: int) -> int:
    return mix64((seed * GAMMA + stream) & MASK64)


def sm_draw(key: int, k: int) -> int:
    return mix64((key + (k + 1) * GAMMA) & MASK64)


def sm_unit(x: int) -> float:
    return (x >> 11) * (1.0 / 9007199254740992.0)


def init_params(seed: int, kind: int) -> np.ndarray:
    """Initial parameters (float32) of the two initialisations (0 Glorot,
    1 profile matching)."""
    p = np.zeros(N_PARAMS, dtype=np.float32)
    nw1 = H * 2 * D
    if kind == 1:
        for k in range(H):
            p[k * 2 * D + k] = 8.0
            p[k * 2 * D + D + k] = 1.0
            p[nw1 + k] = -0.2
            p[nw1 + H + k] = 1.0
        return p
    key = sm_key(seed, 1)
    a1 = np.sqrt(6.0 / (2 * D + H))
    a2 = np.sqrt(6.0 / (H + 1))
    for i in range(nw1):
        p[i] = np.float32((2.0 * sm_unit(sm_draw(key, i)) - 1.0) * a1)
    for k in range(H):
        p[nw1 + H + k] = np.float32((2.0 * sm_unit(sm_draw(key, nw1 + k)) - 1.0) * a2)
    return p


def epoch_order(seed: int, e: int, valid) -> list:
    key = sm_key(seed, 16 + e)
    return [r for _, r in sorted((sm_draw(key, r), r) for r in valid)]


def batch_reads(seed: int, t: int, B: int, valid) -> list:
    """Read indices of step t."""
    out, cache = [], {}
    for b in range(B):
        p = t * B + b
        e = p // len(valid)
        if e not in cache:
            cache[e] = epoch_order(seed, e, valid)
        out.append(cache[e][p % len(valid)])
    return out


def batch_candidates(seed: int, t: int, B: int, b: int, label: int, second: int, NF: int) -> list:
    """The 64 candidates (label first) of slot b of step t, without hard
    negatives."""
    row = [label]
    if 0 <= second < NF and second != label:
        row.append(second)
    if NF > 1:
        key = sm_key(seed, 2)
        for k in range(512):
            if len(row) == 64:
                break
            f = int(sm_unit(sm_draw(key, (t * B + b) * 512 + k)) * (NF - 1))
            if f >= label:
                f += 1
            if f not in row:
                row.append(f)
    for f in range(NF):
        if len(row) == 64:
            break
        if f != label and f not in row:
            row.append(f)
    n = len(row)
    while len(row) < 64:
        j = len(row)
        row.append(row[1 + (j - n) % (n - 1)] if n > 1 else label)
    return row
