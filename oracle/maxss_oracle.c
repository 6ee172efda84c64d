/*
 * maxss_oracle.c -- plain, slow, obviously-correct CPU oracle for the MaxSSmap
 * hot path (Turki & Roshan, "MaxSSmap: A GPU program for mapping divergent
 * short reads to genomes with the maximum scoring subsequence").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library) never calls it, and this file shares no code, header,
 * table or constant with the HIP path.
 *
 * Everything here is the plain definition written out as nested loops over
 * ASCII characters, in int32, with no blocking, packing or fusion:
 *
 *   - maximum scoring subsequence (Methods, "Maximum scoring subsequence"):
 *     the largest sum of a contiguous run of the per-position substitution
 *     scores of two equal-length ungapped sequences; the empty run (sum 0)
 *     is allowed, so every score is >= 0 (reading of the garbled index range
 *     in that definition);
 *   - fragments (Introduction; Methods, "Overview" and "Coalescent global
 *     memory access" with Figure 2): the genome is cut into disjoint
 *     fragments of F bases, the last one padded with N;
 *   - sliding window per fragment (Methods, "First phase of MaxSSmap" and
 *     Figure 1): every start offset o in [0,F) of fragment f is scored with a
 *     full read-length window that may run into the next fragment (junctions)
 *     and past the genome end into N padding;
 *   - best and second-best fragment per read (Introduction; "First phase");
 *   - Needleman-Wunsch of the read against the region of the best fragment
 *     (Methods, "Second phase of MaxSSmap").
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - N (genome, padding or read) scores `mismatch` against everything;
 *   - both strands are scanned; a fragment's value is the max over strands;
 *   - inside a fragment the representative is the smallest strand, then the
 *     smallest offset, among the maxima; across fragments the higher score
 *     wins, then the smaller fragment id; top2 is the best *other* fragment;
 *   - NW region = [max(0, fF-pad), min(G, fF+F+m-1+pad)); fitting mode by
 *     default (whole read, free ends in the region), global mode on a flag;
 *     traceback priority on ties: diagonal, then up (I), then left (D).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)

#define OR_ONE_STRAND 1u  /* scan the read as given only */
#define OR_FAST 2u        /* MaxSSmap_fast: score every other read base */
#define OR_EXCL_ADJ 4u    /* top2 skips the fragments next to top1 */

/* Output record of the scan: 32 bytes, little-endian, no implicit padding. */
typedef struct {
  int32_t frag[2];
  int32_t score[2];
  int32_t offset[2];
  int8_t strand[2];
  int8_t pad_[6];
} oracle_top2;

/* ---------------------------------------------------------------- bases */

/* Upper-case base letter, or 0 if the character is not one of ACGTN/acgtn. */
static char norm_base(char c) {
  switch (c) {
    case 'A': case 'a': return 'A';
    case 'C': case 'c': return 'C';
    case 'G': case 'g': return 'G';
    case 'T': case 't': return 'T';
    case 'N': case 'n': return 'N';
    default: return 0;
  }
}

static char complement(char c) {
  switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    default: return 'N';
  }
}

/* Substitution score of two upper-case bases: match if equal and not N. */
static int32_t subst(char a, char b, int32_t M, int32_t X) {
  return (a == b && a != 'N') ? M : X;
}

/* Genome base at absolute position p; positions >= G are N padding. */
static char genome_at(const char* g, uint64_t G, uint64_t p) {
  return p < G ? g[p] : 'N';
}

int oracle_check_seq(const char* s, uint64_t n) {
  for (uint64_t i = 0; i < n; i++)
    if (!norm_base(s[i])) return OR_EINVAL;
  return OR_OK;
}

/* Upper-case copy (caller frees).  Returns NULL on a bad character. */
static char* normalise(const char* s, uint64_t n) {
  char* out = (char*)malloc(n ? n : 1);
  if (!out) return NULL;
  for (uint64_t i = 0; i < n; i++) {
    out[i] = norm_base(s[i]);
    if (!out[i]) { free(out); return NULL; }
  }
  return out;
}

void oracle_revcomp(const char* in, uint32_t m, char* out) {
  for (uint32_t k = 0; k < m; k++) out[k] = complement(norm_base(in[m - 1 - k]));
}

uint32_t oracle_num_fragments(uint64_t G, uint32_t F) {
  return (uint32_t)((G + F - 1) / F);
}

/* ------------------------------------------------ maximum scoring subsequence */

/* Linear-time maximum scoring subsequence (Bentley / Bates-Constable, i.e.
 * Kadane) of an arbitrary int32 sequence; the empty run scores 0. */
int32_t oracle_maxss_seq(const int32_t* x, uint32_t n) {
  int32_t H = 0, B = 0; /* H: best sum of a run ending here; B: best so far */
  for (uint32_t k = 0; k < n; k++) {
    H = H + x[k];
    if (H < 0) H = 0;
    if (H > B) B = H;
  }
  return B;
}

/* Position-specific scores from base qualities (Methods, paragraph on base
 * qualities and the position specific scoring matrix).  With x = 1 -
 * 10^(-Q/10) the probability that read base k is right (Q = qual[k] - 33,
 * Phred+33), a match scores M x and a mismatch X x / 3 (the formula as
 * printed), in integer units of 1/scale: sm[k] = lround(M * x * scale) and
 * sx[k] = lround(X * x * scale / 3), evaluated left to right in double. */
static int qual_scores(const char* qual, uint32_t m, int32_t M, int32_t X, int32_t scale,
                       int32_t* sm, int32_t* sx) {
  for (uint32_t k = 0; k < m; k++) {
    const int c = (unsigned char)qual[k];
    if (c < 33 || c > 126) return OR_EINVAL;
    const double x = 1.0 - pow(10.0, -(double)(c - 33) / 10.0);
    sm[k] = (int32_t)lround((double)M * x * (double)scale);
    sx[k] = (int32_t)lround((double)X * x * (double)scale / 3.0);
  }
  return OR_OK;
}

/* Substitution score of read base k (q) against genome base g: M / X, or the
 * read's position-specific pair when sm is given. */
static inline int32_t pos_subst(char q, char g, uint32_t k, int32_t M, int32_t X,
                                const int32_t* sm, const int32_t* sx) {
  if (!sm) return subst(q, g, M, X);
  return (q == g && q != 'N') ? sm[k] : sx[k];
}

/* MaxSS score of read q (length m, upper-case) against the genome window
 * starting at absolute position p: the maximum scoring subsequence of the
 * ungapped substitution scores subst(q[k], g[p+k]), k = 0..m-1.  With
 * step 2 (MaxSSmap_fast, Methods paragraph of that name) only the read
 * positions k = 0, 2, 4, ... enter the sequence, each against g[p+k]. */
static int32_t window_score(const char* q, uint32_t m, const char* g, uint64_t G,
                            uint64_t p, int32_t M, int32_t X, uint32_t step,
                            const int32_t* sm, const int32_t* sx) {
  int32_t H = 0, B = 0;
  for (uint32_t k = 0; k < m; k += step) {
    H = H + pos_subst(q[k], genome_at(g, G, p + k), k, M, X, sm, sx);
    if (H < 0) H = 0;
    if (H > B) B = H;
  }
  return B;
}

int oracle_window_score(const char* read, uint32_t m, const char* genome, uint64_t G,
                        uint64_t p, int32_t M, int32_t X, uint32_t step, const char* qual,
                        int32_t qscale, int32_t* out) {
  if (step != 1 && step != 2) return OR_EINVAL;
  char* q = normalise(read, m);
  char* g = normalise(genome, G);
  int32_t* sm = qual ? (int32_t*)malloc(sizeof(int32_t) * (m ? m : 1)) : NULL;
  int32_t* sx = qual ? (int32_t*)malloc(sizeof(int32_t) * (m ? m : 1)) : NULL;
  int st = (!q || !g || (qual && (!sm || !sx))) ? OR_EINVAL : OR_OK;
  if (st == OR_OK && qual) st = qual_scores(qual, m, M, X, qscale, sm, sx);
  if (st == OR_OK) *out = window_score(q, m, g, G, p, M, X, step, sm, sx);
  free(q); free(g); free(sm); free(sx);
  return st;
}

/* --------------------------------------------------------- scan + top-2 */

/* Score of every fragment for one read (both strands unless one_strand):
 * v[f], with representative strand s[f] and offset o[f]. */
static void fragment_values(const char* q_fwd, const char* q_rc, uint32_t m,
                            const char* g, uint64_t G, uint32_t F, uint32_t NF,
                            int32_t M, int32_t X, int one_strand, uint32_t step,
                            const int32_t* const* sm, const int32_t* const* sx,
                            int32_t* v, int32_t* s_out, int32_t* o_out) {
  for (uint32_t f = 0; f < NF; f++) {
    int32_t best = -1, bs = 0, bo = 0;
    for (int s = 0; s < (one_strand ? 1 : 2); s++) {
      const char* q = s == 0 ? q_fwd : q_rc;
      for (uint32_t o = 0; o < F; o++) {
        uint64_t p = (uint64_t)f * F + o;
        int32_t sc = window_score(q, m, g, G, p, M, X, step, sm[s], sx[s]);
        if (sc > best) { best = sc; bs = s; bo = (int32_t)o; } /* strict: keeps smallest s, o */
      }
    }
    v[f] = best; s_out[f] = bs; o_out[f] = bo;
  }
}

/* Top-2 over fragments: the highest value, smallest id on ties; top2 is the
 * same rule over the fragments other than top1, and with excl_adj also other
 * than top1 - 1 and top1 + 1 (a read whose alignment crosses a junction, an
 * indel near it for instance, also scores in the neighbouring fragment; that
 * is the same locus, not a second one). */
static void top_two(const int32_t* v, const int32_t* s, const int32_t* o, uint32_t NF,
                    int excl_adj, oracle_top2* r) {
  int32_t f1 = -1, f2 = -1;
  for (uint32_t f = 0; f < NF; f++)
    if (f1 < 0 || v[f] > v[f1]) f1 = (int32_t)f;
  for (uint32_t f = 0; f < NF; f++) {
    if ((int32_t)f == f1) continue;
    if (excl_adj && ((int32_t)f == f1 - 1 || (int32_t)f == f1 + 1)) continue;
    if (f2 < 0 || v[f] > v[f2]) f2 = (int32_t)f;
  }
  memset(r, 0, sizeof(*r));
  r->frag[0] = f1; r->score[0] = v[f1]; r->offset[0] = o[f1]; r->strand[0] = (int8_t)s[f1];
  if (f2 >= 0) {
    r->frag[1] = f2; r->score[1] = v[f2]; r->offset[1] = o[f2]; r->strand[1] = (int8_t)s[f2];
  } else {
    r->frag[1] = -1; r->score[1] = -1; r->offset[1] = -1; r->strand[1] = -1;
  }
}

typedef struct {
  const char* g; uint64_t G; uint32_t F, NF;
  const char* reads; const uint64_t* offsets; uint32_t n;
  int32_t M, X; int one_strand; uint32_t step;
  const char* quals; int32_t qscale; /* optional Phred+33 qualities (CSR as reads) */
  int excl_adj;
  int tid, nthreads;
  oracle_top2* out;
  int32_t* all_v; /* optional n x NF matrix of fragment values */
  int status;
} scan_job;

static void* scan_worker(void* arg) {
  scan_job* J = (scan_job*)arg;
  int32_t* v = (int32_t*)malloc(sizeof(int32_t) * J->NF);
  int32_t* s = (int32_t*)malloc(sizeof(int32_t) * J->NF);
  int32_t* o = (int32_t*)malloc(sizeof(int32_t) * J->NF);
  if (!v || !s || !o) { J->status = OR_ENOMEM; free(v); free(s); free(o); return NULL; }
  for (uint32_t i = (uint32_t)J->tid; i < J->n; i += (uint32_t)J->nthreads) {
    uint32_t m = (uint32_t)(J->offsets[i + 1] - J->offsets[i]);
    char* q = normalise(J->reads + J->offsets[i], m);
    char* rc = (char*)malloc(m ? m : 1);
    if (!q || !rc) { free(q); free(rc); J->status = OR_EINVAL; break; }
    oracle_revcomp(q, m, rc);
    /* position-specific scores of each strand (reverse strand: reversed) */
    int32_t* sm[2] = {NULL, NULL};
    int32_t* sx[2] = {NULL, NULL};
    if (J->quals) {
      for (int t = 0; t < 2; t++) {
        sm[t] = (int32_t*)malloc(sizeof(int32_t) * m);
        sx[t] = (int32_t*)malloc(sizeof(int32_t) * m);
      }
      int bad = !sm[0] || !sm[1] || !sx[0] || !sx[1] ||
                qual_scores(J->quals + J->offsets[i], m, J->M, J->X, J->qscale, sm[0], sx[0]);
      if (!bad)
        for (uint32_t k = 0; k < m; k++) {
          sm[1][k] = sm[0][m - 1 - k];
          sx[1][k] = sx[0][m - 1 - k];
        }
      if (bad) {
        for (int t = 0; t < 2; t++) { free(sm[t]); free(sx[t]); }
        free(q); free(rc); J->status = OR_EINVAL; break;
      }
    }
    fragment_values(q, rc, m, J->g, J->G, J->F, J->NF, J->M, J->X, J->one_strand, J->step,
                    (const int32_t* const*)sm, (const int32_t* const*)sx, v, s, o);
    for (int t = 0; t < 2; t++) { free(sm[t]); free(sx[t]); }
    top_two(v, s, o, J->NF, J->excl_adj, &J->out[i]);
    if (J->all_v) memcpy(J->all_v + (uint64_t)i * J->NF, v, sizeof(int32_t) * J->NF);
    free(q); free(rc);
  }
  free(v); free(s); free(o);
  return NULL;
}

/* Full scan: top-2 record per read.  reads is a CSR concatenation (offsets has
 * n+1 entries).  all_v (may be NULL) receives the n x NF fragment values.
 * flags: OR_ONE_STRAND, OR_FAST (every other read base, per strand),
 * OR_EXCL_ADJ (top2 never a neighbour of top1).  quals
 * (may be NULL): Phred+33 qualities laid out as the reads, scored with the
 * position-specific pairs of qual_scores at scale qscale. */
int oracle_scan(const char* genome, uint64_t G, uint32_t F, const char* reads,
                const uint64_t* offsets, uint32_t n, int32_t M, int32_t X, uint32_t flags,
                int nthreads, oracle_top2* out, int32_t* all_v, const char* quals,
                int32_t qscale) {
  if (G == 0 || F == 0) return OR_EINVAL;
  for (uint32_t i = 0; i < n; i++)
    if (offsets[i + 1] <= offsets[i]) return OR_EINVAL;
  char* g = normalise(genome, G);
  if (!g) return OR_EINVAL;
  if (nthreads < 1) nthreads = 1;
  uint32_t NF = oracle_num_fragments(G, F);
  scan_job* jobs = (scan_job*)calloc((size_t)nthreads, sizeof(scan_job));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !th) { free(g); free(jobs); free(th); return OR_ENOMEM; }
  for (int t = 0; t < nthreads; t++) {
    scan_job J = {g, G, F, NF, reads, offsets, n, M, X, (flags & OR_ONE_STRAND) != 0,
                  (flags & OR_FAST) ? 2u : 1u, quals, qscale, (flags & OR_EXCL_ADJ) != 0,
                  t, nthreads, out, all_v, OR_OK};
    jobs[t] = J;
    pthread_create(&th[t], NULL, scan_worker, &jobs[t]);
  }
  int st = OR_OK;
  for (int t = 0; t < nthreads; t++) {
    pthread_join(th[t], NULL);
    if (jobs[t].status != OR_OK) st = jobs[t].status;
  }
  free(jobs); free(th); free(g);
  return st;
}

/* ------------------------------------------------------- Needleman-Wunsch */

#define OR_NW_GLOBAL 1

/* Full-DP Needleman-Wunsch with a linear gap of the read q (m bases) against
 * the reference r (n bases).  Fitting mode (mode 0): the whole read is
 * aligned, the reference ends are free (D[0][j]=0, end column free).  Global
 * mode: both sequences end to end.  Outputs the score, the aligned reference
 * span [*jb, *je) in column units, and the expanded operation string
 * ('=' match, 'X' mismatch, 'I' read base against a gap, 'D' reference base
 * against a gap) in alignment order, NUL-terminated. */
int oracle_nw(const char* read, uint32_t m, const char* ref, uint32_t n, int32_t M,
              int32_t X, int32_t gap, int mode, const char* qual, int32_t qscale,
              int32_t* score, int32_t* jb, int32_t* je, char* ops, uint32_t ops_cap,
              uint32_t* ops_len) {
  char* q = normalise(read, m);
  char* r = normalise(ref, n);
  if (!q || !r) { free(q); free(r); return OR_EINVAL; }
  /* with qualities (in the read's orientation as given): row i scores with
   * the pair of read base i, and the gap is in the same 1/scale units */
  int32_t* sm = NULL;
  int32_t* sx = NULL;
  if (qual) {
    sm = (int32_t*)malloc(sizeof(int32_t) * (m ? m : 1));
    sx = (int32_t*)malloc(sizeof(int32_t) * (m ? m : 1));
    if (!sm || !sx || qual_scores(qual, m, M, X, qscale, sm, sx)) {
      free(sm); free(sx); free(q); free(r); return OR_EINVAL;
    }
    gap = gap * qscale;
  }
  uint64_t W = (uint64_t)n + 1;
  int32_t* D = (int32_t*)malloc(sizeof(int32_t) * (uint64_t)(m + 1) * W);
  if (!D) { free(sm); free(sx); free(q); free(r); return OR_ENOMEM; }
#define DP(i, j) D[(uint64_t)(i) * W + (j)]
  for (uint32_t j = 0; j <= n; j++) DP(0, j) = (mode == OR_NW_GLOBAL) ? (int32_t)j * gap : 0;
  for (uint32_t i = 1; i <= m; i++) {
    DP(i, 0) = (int32_t)i * gap;
    for (uint32_t j = 1; j <= n; j++) {
      int32_t d = DP(i - 1, j - 1) + pos_subst(q[i - 1], r[j - 1], i - 1, M, X, sm, sx);
      int32_t u = DP(i - 1, j) + gap;
      int32_t l = DP(i, j - 1) + gap;
      int32_t b = d;
      if (u > b) b = u;
      if (l > b) b = l;
      DP(i, j) = b;
    }
  }
  uint32_t jend;
  if (mode == OR_NW_GLOBAL) {
    jend = n;
  } else {
    jend = 0;
    for (uint32_t j = 1; j <= n; j++)
      if (DP(m, j) > DP(m, jend)) jend = j; /* strict: smallest j among maxima */
  }
  *score = DP(m, jend);
  *je = (int32_t)jend;
  /* traceback, collected backwards */
  uint64_t cap = (uint64_t)m + n + 1;
  char* rev = (char*)malloc(cap);
  if (!rev) { free(D); free(sm); free(sx); free(q); free(r); return OR_ENOMEM; }
  uint64_t len = 0;
  uint32_t i = m, j = jend;
  while (i > 0 || (mode == OR_NW_GLOBAL && j > 0)) {
    if (i > 0 && j > 0 &&
        DP(i, j) == DP(i - 1, j - 1) + pos_subst(q[i - 1], r[j - 1], i - 1, M, X, sm, sx)) {
      rev[len++] = (q[i - 1] == r[j - 1] && q[i - 1] != 'N') ? '=' : 'X';
      i--; j--;
    } else if (i > 0 && DP(i, j) == DP(i - 1, j) + gap) {
      rev[len++] = 'I';
      i--;
    } else {
      rev[len++] = 'D';
      j--;
    }
  }
  *jb = (int32_t)j;
  int st = OR_OK;
  if (len + 1 > ops_cap) {
    st = OR_EINVAL;
  } else {
    for (uint64_t t = 0; t < len; t++) ops[t] = rev[len - 1 - t];
    ops[len] = 0;
  }
  *ops_len = (uint32_t)len;
#undef DP
  free(rev); free(D); free(sm); free(sx); free(q); free(r);
  return st;
}

/* Run-length CIGAR of an expanded operation string, e.g. "==X=" -> "2=1X1=". */
int oracle_cigar_rle(const char* ops, char* out, uint32_t cap) {
  uint32_t w = 0;
  uint32_t L = (uint32_t)strlen(ops);
  for (uint32_t a = 0; a < L;) {
    uint32_t b = a;
    while (b < L && ops[b] == ops[a]) b++;
    char num[16];
    int k = 0;
    uint32_t run = b - a;
    char tmp[16];
    int t = 0;
    do { tmp[t++] = (char)('0' + run % 10); run /= 10; } while (run);
    while (t) num[k++] = tmp[--t];
    if (w + (uint32_t)k + 2 > cap) return OR_EINVAL;
    memcpy(out + w, num, (size_t)k);
    w += (uint32_t)k;
    out[w++] = ops[a];
    a = b;
  }
  if (w + 1 > cap) return OR_EINVAL;
  out[w] = 0;
  return OR_OK;
}

/* Alignment record of the second phase. */
typedef struct {
  int32_t score;
  int8_t strand;
  int8_t flags;
  int8_t pad_[2];
  int64_t ref_begin, ref_end;
  uint32_t cigar_len;
  uint32_t pad2_;
} oracle_aln;

/* Second phase for one read: NW of the read (in the orientation of its best
 * strand) against the region of its best fragment, padded by `pad` bases on
 * each side and clipped to the genome.  CIGAR (run-length) goes to cigar. */
int oracle_align_one(const char* genome, uint64_t G, uint32_t F, const char* read,
                     uint32_t m, int32_t frag, int32_t strand, uint32_t pad, int32_t M,
                     int32_t X, int32_t gap, int mode, const char* qual, int32_t qscale,
                     oracle_aln* out, char* cigar, uint32_t cigar_cap) {
  if (frag < 0 || m == 0) return OR_EINVAL;
  char* q = normalise(read, m);
  if (!q) return OR_EINVAL;
  char* qq = (char*)malloc(m);
  char* ql = qual ? (char*)malloc(m) : NULL;
  if (!qq || (qual && !ql)) { free(q); free(qq); free(ql); return OR_ENOMEM; }
  if (strand) oracle_revcomp(q, m, qq); else memcpy(qq, q, m);
  if (qual)  /* qualities follow the read: reversed on the reverse strand */
    for (uint32_t k = 0; k < m; k++) ql[k] = strand ? qual[m - 1 - k] : qual[k];
  int64_t start = (int64_t)frag * F;
  int64_t a = start - (int64_t)pad;
  if (a < 0) a = 0;
  int64_t b = start + (int64_t)F + (int64_t)m - 1 + (int64_t)pad;
  if (b > (int64_t)G) b = (int64_t)G;
  if (b <= a) { free(q); free(qq); free(ql); return OR_EINVAL; }
  uint32_t n = (uint32_t)(b - a);
  uint32_t cap = m + n + 1;
  char* ops = (char*)malloc(cap);
  if (!ops) { free(q); free(qq); free(ql); return OR_ENOMEM; }
  int32_t sc, jb, je;
  uint32_t olen;
  int st = oracle_nw(qq, m, genome + a, n, M, X, gap, mode, ql, qscale, &sc, &jb, &je, ops, cap,
                     &olen);
  if (st == OR_OK) {
    memset(out, 0, sizeof(*out));
    out->score = sc;
    out->strand = (int8_t)strand;
    out->ref_begin = a + jb;
    out->ref_end = a + je;
    st = oracle_cigar_rle(ops, cigar, cigar_cap);
    out->cigar_len = st == OR_OK ? (uint32_t)strlen(cigar) : 0;
  }
  free(ops); free(q); free(qq); free(ql);
  return st;
}
