/*
 * maxss.h -- C ABI of libmaxss, an MI355X (gfx950) implementation of the
 * MaxSSmap hot path (Turki & Roshan, "MaxSSmap: A GPU program for mapping
 * divergent short reads to genomes with the maximum scoring subsequence").
 *
 * The mapping problem, as the paper states it (Methods, "Overview", "First
 * phase of MaxSSmap", "Second phase of MaxSSmap"): the genome is cut into
 * disjoint fragments of a user-given length; every read is scored against
 * every fragment with the maximum scoring subsequence of the ungapped
 * substitution scores of a read-length window slid along the fragment; the
 * best and second-best fragments are reported; the read is then aligned with
 * Needleman-Wunsch to the genome region of the best fragment.
 *
 * Conventions shared by every call:
 *   - Every call returns a maxss_status; on failure maxss_last_error() gives a
 *     thread-local message.  No C++ exception crosses this boundary.  On
 *     failure the outputs are unspecified and the inputs are untouched.
 *   - The caller owns every read, output and CIGAR buffer; the library owns
 *     indexes and frees them only in maxss_index_free.  The library never
 *     frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     With device-resident reads (maxss_reads.on_device = 1) every pointer
 *     argument of the call must be device memory and the call is
 *     asynchronous on `stream`; with host reads every pointer is host memory
 *     and the call returns when the results are in the host buffers.
 *   - Bases are ASCII A, C, G, T, N in either case.  N (in the genome, in a
 *     read, or the padding past the genome end) scores `mismatch` against
 *     everything, including N.
 *   - All scores are exact integers (with base qualities: integers in units of
 *     1/qual_scale, see maxss_params).
 */
#ifndef MAXSS_H
#define MAXSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MAXSS_OK = 0,
  MAXSS_EINVAL = -1,   /* bad argument, bad character, bad parameter range   */
  MAXSS_ENOMEM = -2,   /* host or device allocation failed                   */
  MAXSS_EDEVICE = -3,  /* a HIP runtime call or kernel launch failed         */
  MAXSS_ETOOLONG = -4, /* a read is empty or longer than max_read_len        */
  MAXSS_ESTATE = -5    /* the call does not fit the object's state           */
} maxss_status;

/* maxss_params.flags */
#define MAXSS_ONE_STRAND 1u /* scan only the read as given (no reverse complement) */
#define MAXSS_NW_GLOBAL 2u  /* end-to-end NW instead of fitting the whole read     */
#define MAXSS_FAST 4u       /* MaxSSmap_fast (Methods paragraph of that name): the
                             * first phase scores read positions 0, 2, 4, ... of
                             * each strand only, each against the genome base
                             * at the same distance from the window start      */
#define MAXSS_EXCLUDE_ADJACENT 8u /* the second-best fragment is never a neighbour
                             * (frag[0] - 1 or frag[0] + 1) of the best one: a
                             * read that crosses a junction also scores in the
                             * neighbouring fragment, at the same locus, and
                             * would otherwise lower its own mapping quality
                             * (the ratio test of the first phase).  Reads whose
                             * second is a neighbour are scanned a second time
                             * with the three fragments left out (through the
                             * learned proposal: among the same candidates). */

/* Scoring and fragmenting parameters, fixed when the genome is indexed.
 *   match        M, score of two equal bases (not N); 1..127.
 *   mismatch     X, score of any other pair; -127..0.
 *   gap          linear gap score of the second phase (NW); -1000000..0.
 *   frag_len     F, fragment length; > 0 and a multiple of 16 (Methods,
 *                "Byte packing for faster global memory access").
 *   max_read_len longest read any later call may pass; 1..8192 and
 *                max_read_len * match <= 65535 (the scan's 16-bit exact range).
 *   flags        MAXSS_ONE_STRAND, MAXSS_NW_GLOBAL, MAXSS_FAST,
 *                MAXSS_EXCLUDE_ADJACENT.
 *   qual_scale   0: plain match / mismatch scores.  > 0: reads carry base
 *                qualities and both phases score with a position-specific
 *                matrix (Methods, paragraph on base qualities and the
 *                position specific scoring matrix): with x = 1 - 10^(-Q/10)
 *                (Q = Phred+33 quality - 33) a match scores M x and a
 *                mismatch X x / 3, in integer units of 1/qual_scale rounded
 *                half away from zero (lround of M*x*s and X*x*s/3 in double,
 *                left to right); N scores the mismatch of its position; the
 *                gap of the second phase is gap*qual_scale.  Requires
 *                match*qual_scale <= 127, -mismatch*qual_scale <= 381 and
 *                max_read_len*match*qual_scale <= 65535. */
typedef struct {
  int32_t match;
  int32_t mismatch;
  int32_t gap;
  uint32_t frag_len;
  uint32_t max_read_len;
  uint32_t flags;
  uint32_t qual_scale;
} maxss_params;

typedef struct maxss_index maxss_index; /* opaque, immutable once built */

/* A batch of reads of any lengths, concatenated (CSR): read i is
 * seq[offsets[i], offsets[i+1]).  offsets has n+1 entries, offsets[0] may be
 * non-zero.  on_device: 1 if seq and offsets are device pointers. */
typedef struct {
  const char* seq;
  const uint64_t* offsets;
  uint32_t n;
  uint32_t on_device;
  const char* qual;  /* Phred+33 qualities laid out as seq (same offsets, same
                      * memory kind), or NULL; required when the index has
                      * qual_scale > 0, ignored otherwise.  A quality outside
                      * '!'..'~' makes the read invalid like a bad base. */
} maxss_reads;

/* Per-read result of the scan (32 bytes).  Entry 0 is the best fragment,
 * entry 1 the best other fragment (-1 in every field when the genome has one
 * fragment).  score: the fragment's value, the largest window score over both
 * strands and every start offset o in [0, F) of the fragment.  strand (0 =
 * read as given, 1 = reverse complement) and offset are those of the
 * fragment's representative window: the smallest strand, then the smallest
 * offset, among the windows reaching the value.  Ties between fragments go to
 * the smaller fragment id.  For device-resident reads, a read that is empty,
 * longer than max_read_len or holds a character other than ACGTN gets
 * frag[0] = MAXSS_READ_INVALID and no other field is meaningful. */
typedef struct {
  int32_t frag[2];
  int32_t score[2];
  int32_t offset[2];
  int8_t strand[2];
  int8_t _pad[6];
} maxss_top2;

#define MAXSS_READ_INVALID (-2)

/* Per-read result of the second phase (32 bytes).  score: the NW score;
 * strand: orientation of the read that was aligned; [ref_begin, ref_end): the
 * genome span the alignment covers (0-based, half-open); cigar_len: length of
 * the run-length CIGAR string written for the read ('=' match, 'X' mismatch,
 * 'I' read base against a gap, 'D' genome base against a gap).  flags bit 0:
 * the CIGAR did not fit cigar_stride and was truncated; bit 1: the read was
 * invalid, or its top[i] record named no valid fragment (frag[0] outside
 * [0, NF) or strand[0] not 0/1), and was not aligned. */
typedef struct {
  int32_t score;
  int8_t strand;
  int8_t flags;
  int8_t _pad[2];
  int64_t ref_begin;
  int64_t ref_end;
  uint32_t cigar_len;
  uint32_t _pad2;
} maxss_aln;

#define MAXSS_ALN_TRUNCATED 1
#define MAXSS_ALN_SKIPPED 2

/* Index a genome (Methods, "Overview"; "Coalescent global memory access";
 * "Byte packing").  seq: host pointer to len ASCII bases.  The genome is cut
 * into NF = ceil(len / F) fragments; positions past len are N.  The index is
 * built on the current HIP device and holds the genome there 2-bit packed with
 * an N mask.  Errors: EINVAL (len = 0, a bad character, a parameter out of the
 * ranges above, NULL pointer), ENOMEM, EDEVICE.  *out is set only on success. */
maxss_status maxss_index_genome(const char* seq, uint64_t len, const maxss_params* params,
                                maxss_index** out);

/* Free an index (NULL is a no-op).  Must not race with calls using it. */
void maxss_index_free(maxss_index* index);

/* Genome length, fragment count and fragment length of an index (any output
 * pointer may be NULL).  Errors: EINVAL on a NULL index. */
maxss_status maxss_index_info(const maxss_index* index, uint64_t* genome_len,
                              uint32_t* num_fragments, uint32_t* frag_len);

/* First phase (Methods, "First phase of MaxSSmap"; Figure 1): for every read,
 * the maximum scoring subsequence score of every (strand, fragment, offset)
 * window -- the window of read length m starting at genome position
 * f*F + o may run into the next fragment and past the genome end -- reduced to
 * the best and second-best fragments (one maxss_top2 per read, in read
 * order).  Reads of any lengths may be mixed in one call.
 * out: n records, host or device memory as the reads.  With MAXSS_FAST the
 * windows score every other read base; with qual_scale > 0 they score with the
 * reads' position-specific scores (reads->qual required); with
 * MAXSS_EXCLUDE_ADJACENT the second fragment is the best one other than
 * frag[0] - 1, frag[0] and frag[0] + 1 (none, frag[1] = -1, when no other
 * fragment is left).
 * Errors: EINVAL (NULL pointers, n = 0 is allowed and does nothing, qualities
 * missing on a quality-mode index, a host quality outside '!'..'~'), ETOOLONG
 * (host reads only: a read of length 0 or > max_read_len), ENOMEM, EDEVICE. */
maxss_status maxss_scan_reads(const maxss_index* index, const maxss_reads* reads,
                              maxss_top2* out, void* stream);

/* maxss_scan_reads without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same records as maxss_scan_reads, written to `out`
 * (n device records), asynchronously on `stream`; reads->on_device must be 1.
 * Every scratch buffer of the call (encoded reads, length order and
 * histogram, work counter, per-chunk partial top-2, and with
 * MAXSS_EXCLUDE_ADJACENT the second pass's buffers) comes from one 64 MiB
 * device array that the library holds per device until the process ends.
 * A call needs, in 256-byte aligned pieces, 4*(n*2*(S/8)+64) + (n*S+64) +
 * 4*(n+1) [+ 2*(n*S+64) with qual_scale > 0] + 4*n + 4*(max_read_len+1) + 4
 * [+ 40*n with MAXSS_EXCLUDE_ADJACENT] + at least 16*n bytes, where
 * S = max_read_len rounded up to 64 (about 27 MB for 100,000 reads with
 * max_read_len <= 128); what is left becomes partial top-2 space, and fewer
 * fragment chunks per read are used when it is small (same records).
 * All calls on one device share the array: calls that overlap on one device
 * (different streams or host threads) race and must be serialised by the
 * caller.  Errors: EINVAL (NULL, host reads, qualities missing on a
 * quality-mode index, a batch needing more than the 64 MiB), ESTATE (index
 * on another device), EDEVICE. */
maxss_status maxss_scan_reads_noalloc(const maxss_index* index, const maxss_reads* reads,
                                      maxss_top2* out, void* stream);

/* Second phase (Methods, "Second phase of MaxSSmap"): for every read,
 * Needleman-Wunsch with a linear gap of the read, in the orientation of
 * top[i].strand[0], against the genome region
 *   [max(0, f*F - pad), min(G, f*F + F + m - 1 + pad)),  f = top[i].frag[0],
 * i.e. the scanned (extended) best fragment widened by pad bases each side.
 * Fitting mode (default): the whole read against a free-ended stretch of the
 * region; MAXSS_NW_GLOBAL: the read against the whole region.  Traceback
 * prefers diagonal, then I, then D; in fitting mode the end column is the
 * smallest one reaching the best score.
 * top: n records from maxss_scan_reads; out: n records; cigar: n *
 * cigar_stride bytes, read i's NUL-terminated CIGAR at cigar + i*cigar_stride
 * (cigar_stride >= 2; a CIGAR that does not fit is truncated and flagged).
 * With qual_scale > 0 each DP row scores with its read base's position-specific
 * pair (reversed qualities for strand 1) and the gap is gap * qual_scale.
 * Pointers are host or device memory as the reads.  Errors: EINVAL (also:
 * qualities missing on a quality-mode index), ETOOLONG (host reads), ENOMEM,
 * EDEVICE. */
maxss_status maxss_align_top(const maxss_index* index, const maxss_reads* reads,
                             const maxss_top2* top, uint32_t pad, maxss_aln* out,
                             char* cigar, uint64_t cigar_stride, void* stream);

/* ---- Batching: reusable plans, HIP graphs, tile autotuning ---------------
 * Not in the paper (which launches one grid per read); these serve mixed-
 * length batches of device-resident reads with one persistent scan launch. */

typedef struct maxss_plan maxss_plan; /* opaque, library-owned */

/* A plan owns all scratch of one step (first phase + second phase) for up to
 * `capacity` device-resident reads, with NW padding `pad` and CIGAR stride
 * `cigar_stride` fixed.  Allocates device memory once, here.  A plan serves
 * one stream at a time: calls that overlap on different streams race.
 * Errors: EINVAL, ESTATE (index on another device), ENOMEM, EDEVICE. */
maxss_status maxss_plan_create(const maxss_index* index, uint32_t capacity, uint32_t pad,
                               uint64_t cigar_stride, maxss_plan** out);
void maxss_plan_free(maxss_plan* plan);

/* One step on device reads (reads->on_device must be 1, reads->n <=
 * capacity): the same records maxss_scan_reads writes to `top` and, if `aln`
 * and `cigar` are not NULL, those of maxss_align_top (with the plan's pad and
 * stride).  No allocation and no host synchronisation: asynchronous on
 * `stream`, and capturable into a HIP graph.  Errors: EINVAL, EDEVICE. */
maxss_status maxss_plan_run(maxss_plan* plan, const maxss_reads* reads, maxss_top2* top,
                            maxss_aln* aln, char* cigar, void* stream);

/* maxss_plan_run recorded once into a HIP graph and replayed: the first call,
 * or a call whose buffers, read count or stream differ from the recorded
 * ones, captures the step on `stream` (must not be NULL); later calls replay
 * it (new buffer contents are fine).  Errors: as maxss_plan_run. */
maxss_status maxss_plan_run_graph(maxss_plan* plan, const maxss_reads* reads, maxss_top2* top,
                                  maxss_aln* aln, char* cigar, void* stream);

/* Autotuner result: the tile shape chosen (np = offset pairs per lane,
 * reads_per_tile, rounds = work items per resident wave; 0 = built-in), the
 * timed scan of the sample with it and with the built-in shape, how many
 * candidates were tried, how many were rejected because a record differed
 * from the built-in shape's (never chosen), and whether it came from the
 * cache file. */
typedef struct {
  int32_t np;
  uint32_t reads_per_tile;
  uint32_t rounds;
  float best_ms;
  float default_ms;
  uint32_t tried;
  uint32_t rejected;
  uint32_t from_cache;
} maxss_tune_result;

/* Time candidate tile shapes of the scan on `sample` (host or device reads)
 * and set the fastest one whose records are byte-identical to the built-in
 * shape's on the index (used by every later scan on it).  With cache_path
 * (may be NULL), a matching entry (device architecture, fragment geometry,
 * read-length and batch-size bucket) is reused without timing, and a new
 * result is appended; an entry whose shape maxss_index_set_tiles would
 * reject is ignored.  Must not run concurrently with scans on the index.
 * Errors: EINVAL, ETOOLONG (host sample), ENOMEM, EDEVICE. */
maxss_status maxss_autotune(maxss_index* index, const maxss_reads* sample, const char* cache_path,
                            maxss_tune_result* result);

/* Scan kernel variants, by the cost of their Kadane inner loop per packed
 * pair of 16-bit cells and step (maxss_scan_kernel_info):
 *   STEP_MAX       score select, saturating add and running max: 3 VALU
 *                  instructions (score bounds above 31744);
 *   TWO_STEP       select and add, one three-way max per two steps: 2.5;
 *   REGISTER_BANK  the four per-base score pairs of every window word kept
 *                  in registers (one v_perm_b32 each when the word enters):
 *                  add, half a max, a quarter of a select: 1.75
 *                  (16 offsets pairs per lane).  With base-quality scores
 *                  it takes the reads whose scored bases all map to one
 *                  (match, mismatch) pair, each read with its own pair; a
 *                  second launch of TWO_STEP takes the other reads. */
#define MAXSS_KERNEL_STEP_MAX 0
#define MAXSS_KERNEL_TWO_STEP 1
#define MAXSS_KERNEL_REGISTER_BANK 2

/* The offset pairs per lane (np) and the kernel variant (kind) that the next
 * scan on the index launches with its current tile setting (built-in,
 * maxss_index_set_tiles or maxss_autotune).  Output pointers may be NULL.
 * Errors: EINVAL on a NULL index. */
maxss_status maxss_scan_kernel_info(const maxss_index* index, int32_t* np, int32_t* kind);

/* Force a tile shape (np 0/8/16/32, reads_per_tile 0..64, rounds 0..1024;
 * 0 = built-in).  Results never depend on it.  Errors: EINVAL. */
maxss_status maxss_index_set_tiles(maxss_index* index, int32_t np, uint32_t reads_per_tile,
                                   uint32_t rounds);

/* ---- Learned fragment proposal ----------------------------------------------
 * Not in the paper.  A small network ranks the fragments of each read from
 * 4-mer count profiles so that only the best K are scanned exactly; a margin
 * test sends unclear reads to the full scan.  The scores of scanned
 * fragments are the exact MaxSS scores of the first phase.
 *
 * Profiles: c[j] = number of 4-mers without N with j = 64x0+16x1+4x2+x3
 * (A0 C1 G2 T3), v = c/||c||_2 (0 if no 4-mer), computed in float64 and
 * rounded to float32, then to bf16 (nearest even).  Reads: one profile per
 * strand.  Fragment f: the 4-mers that start in [fF, fF+F).
 * Network: z = [v_read ; v_frag], h = ReLU(W1 z + b1) (W1: 256 x 512),
 * y = w2 . h + b2; W1 and w2 in bf16, b1 and b2 in fp32, fp32 accumulation.
 * Parameters (MAXSS_MLP_PARAMS floats, this order): W1 row-major, b1, w2, b2.
 * A fragment's score for a read is the max of y over the read's strands. */
#define MAXSS_MLP_PARAMS 131585

typedef struct maxss_model maxss_model; /* opaque, library-owned */

/* Initialisations of maxss_model_create.
 *   MAXSS_INIT_GLOROT: W1 and w2 uniform in +-sqrt(6 / (fan_in + fan_out))
 *     (Glorot & Bengio, 2010), biases 0.  The draws come from SplitMix64
 *     (Steele, Lea & Flood, OOPSLA 2014) in counter mode: draw k of stream s
 *     under `seed` is mix64(key + (k + 1) * 0x9E3779B97F4A7C15) with
 *     key = mix64(seed * 0x9E3779B97F4A7C15 + s), mix64 the generator's
 *     output function; a unit double is the top 53 bits times 2^-53.  W1
 *     element i is (2u - 1) a1 with u from draw i of stream 1, w2 element k
 *     from draw 131072 + k; computed in double, rounded to float.
 *   MAXSS_INIT_PROFILE_MATCH: hidden unit k compares bin k of the two
 *     profiles: W1[k][k] = 8 (read), W1[k][256 + k] = 1 (fragment), every
 *     other weight 0, b1 = -0.2, w2 = 1, b2 = 0.  A read's 4-mers that the
 *     fragment holds then add the fragment's share of them, which ranks
 *     fragments much like the cosine of the two profiles; `seed` is unused. */
#define MAXSS_INIT_GLOROT 0u
#define MAXSS_INIT_PROFILE_MATCH 1u

/* Create a model on the current device with initial parameters `init`
 * (fp32 master copy; Adam state zero).  Errors: EINVAL (NULL, unknown init),
 * ENOMEM, EDEVICE. */
maxss_status maxss_model_create(uint32_t seed, uint32_t init, maxss_model** out);

/* Create a model from MAXSS_MLP_PARAMS host floats instead (Adam state
 * zero).  Errors: EINVAL, ENOMEM, EDEVICE. */
maxss_status maxss_model_from_params(const float* params, maxss_model** out);
void maxss_model_free(maxss_model* model);

/* Copy the fp32 master parameters to `out` (host, MAXSS_MLP_PARAMS floats). */
maxss_status maxss_model_get_params(const maxss_model* model, float* out);

/* Save / load parameters, Adam state and step count (binary, format
 * version 1).  Errors: EINVAL (I/O, bad file), ENOMEM, EDEVICE. */
maxss_status maxss_model_save(const maxss_model* model, const char* path);
maxss_status maxss_model_load(const char* path, maxss_model** out);

/* The fp32 profiles (before bf16 rounding): read_prof (device, n*2*256,
 * strand-major per read) of device reads, and/or frag_prof (device,
 * NF*256).  Either may be NULL (reads may be NULL with read_prof NULL).
 * Asynchronous on `stream`.  Errors: EINVAL, ENOMEM, EDEVICE. */
maxss_status maxss_profiles(const maxss_index* index, const maxss_reads* reads, float* read_prof,
                            float* frag_prof, void* stream);

/* Network score of every (read, fragment): scores (device, n*NF floats,
 * read-major) = max over strands of y.  Device reads.  Errors: as above. */
maxss_status maxss_proposal_scores(const maxss_index* index, maxss_model* model,
                                   const maxss_reads* reads, float* scores, void* stream);

/* First phase through the proposal: per read, the K fragments with the
 * highest scores (ties to the smaller id) are scanned exactly and the top-2
 * among them are reported; a read whose two best scores differ by less than
 * `margin` is scanned in full instead (fell_back[i] = 1; device, may be
 * NULL).  With min_score >= 0 (the exact-score guard) the candidates of
 * every read are scanned first, and a read whose margin is below `margin`
 * still keeps that record when its best candidate's exact MaxSS score is at
 * least min_score; min_score < 0 turns the guard off.  Records have the layout and tie rules of maxss_scan_reads; they
 * equal the full scan's whenever its top-2 fragments are among the K.
 * With MAXSS_EXCLUDE_ADJACENT the second is the best candidate other than
 * the best one's neighbours.  Device reads.  Errors: EINVAL (K = 0 or >
 * 4096), ENOMEM, EDEVICE. */
maxss_status maxss_scan_reads_proposed(const maxss_index* index, maxss_model* model,
                                       const maxss_reads* reads, uint32_t K, float margin,
                                       int32_t min_score, maxss_top2* out, uint8_t* fell_back,
                                       void* stream);

/* The proposal alone: per read, the K candidate fragments (device, n*K
 * int32, ascending ids; -1 past min(K, NF)), the margin between the two best
 * scores (device, n floats; +inf with one fragment) and the fall-back flag
 * (margin < `margin`, invalid reads never fall back).  Device reads.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
maxss_status maxss_proposal_candidates(const maxss_index* index, maxss_model* model,
                                       const maxss_reads* reads, uint32_t K, float margin,
                                       int32_t* cand, float* margins, uint8_t* fell_back,
                                       void* stream);

/* One training step on a batch of B device reads: cand (device, B*64 int32)
 * holds, per read, the label fragment first and 63 other fragments; strand
 * (device, B int8) the label strand, whose profile is used for all 64
 * pairs.  Loss: mean over reads of the softmax cross-entropy of the 64
 * scores with the label at position 0.  Writes the mean loss to `loss`
 * (device float, may be NULL) and the gradient to `grad` (device,
 * MAXSS_MLP_PARAMS floats, may be NULL); then, if lr > 0, one Adam step
 * (beta1 0.9, beta2 0.999, eps 1e-8) on the fp32 master weights and a
 * refresh of the bf16 copies.  Errors: EINVAL, ENOMEM, EDEVICE. */
maxss_status maxss_model_train_step(maxss_model* model, const maxss_index* index,
                                    const maxss_reads* batch, const int32_t* cand,
                                    const int8_t* strand, float lr, float* loss, float* grad,
                                    void* stream);

/* Training on plain-scan labels, in the library.  reads: device reads;
 * labels: their maxss_scan_reads records (device).  The first n - n_val
 * reads train, the last n_val = floor(n * val_fraction) are held out; reads
 * whose label is invalid are skipped.  Step t takes reads t*batch ..
 * t*batch + batch - 1 of the concatenated epochs, epoch e ordering the
 * training reads by (draw r of stream 16 + e, r) (SplitMix64 as for
 * MAXSS_INIT_GLOROT, seed = opts->seed).  Each read trains on its label's
 * strand profile against 64 candidates, the label first, then: the
 * second-best fragment (when there is one), up to hard_negatives of the
 * model's own best fragments other than the label (the top hard_negatives + 1
 * by score, ascending ids, re-ranked every step), and distinct uniform draws
 * (draw (t*batch + b)*512 + k of stream 2, f = floor(u (NF - 1)), plus 1 if
 * f >= label) until 63 negatives are found; with fewer fragments the list is
 * repeated.  Loss and Adam as maxss_model_train_step.  Every eval_every
 * steps (and at the end) the held-out recall@K is measured, and the model
 * keeps the parameters of the best one (the initial ones if no step
 * improved it).  Then, on the held-out reads, the thresholds of
 * maxss_scan_reads_proposed are chosen by maxss_choose_acceptance for
 * target_agreement.  Synchronous on `stream`.  Errors: EINVAL (NULL, host
 * reads, options out of range, no labelled training read), ESTATE (devices
 * differ), ENOMEM, EDEVICE. */
typedef struct {
  uint32_t steps;          /* Adam steps (0: thresholds only)                */
  uint32_t batch;          /* reads per step, 1..65536                       */
  float lr;                /* Adam learning rate, >= 0                       */
  uint32_t seed;           /* read order and negative draws                  */
  uint32_t hard_negatives; /* 0..62                                          */
  uint32_t eval_every;     /* steps between held-out evaluations (0: end)    */
  uint32_t K;              /* candidates per read, 1..4096                   */
  float val_fraction;      /* 0..0.9                                          */
  float target_agreement;  /* held-out top-1 agreement for the thresholds    */
  float* loss_trace;       /* host, `steps` floats (batch losses), or NULL   */
  int32_t* cand_trace;     /* host, steps * batch * 64 ints: every step's
                            * candidate rows (label first), or NULL; a copy
                            * per step, for checking the draws              */
} maxss_train_opts;

typedef struct {
  uint32_t n_train, n_val;       /* reads trained on / held out               */
  uint32_t steps_run, best_step; /* best_step: parameters kept (0 = initial)  */
  float loss_first, loss_last;   /* batch loss of the first and last step     */
  float val_recall_init;         /* held-out recall@K before training         */
  float val_recall_best;         /* and of the parameters kept (-1: no reads) */
  float tau;                     /* margin threshold (+inf: margins accept none) */
  int32_t min_score;             /* exact-score threshold (-1: none accepted) */
  float val_accept;              /* held-out fraction accepted by the two     */
  float val_agreement;           /* held-out top-1 agreement with them        */
} maxss_train_stats;

maxss_status maxss_model_train(maxss_model* model, const maxss_index* index,
                               const maxss_reads* reads, const maxss_top2* labels,
                               const maxss_train_opts* opts, maxss_train_stats* stats,
                               void* stream);

/* Thresholds of the proposed scan from n held-out reads (host arrays): the
 * network's margin, the best candidate's exact score (-1 if none) and
 * whether the best candidate is the full scan's best fragment.  A read is
 * accepted when margin >= tau or best_score >= min_score; an accepted read
 * agrees when `correct`, a fallen-back read always agrees.  min_score is the
 * smallest score whose acceptance keeps the agreement >= target (-1 if even
 * the best score would break it); then tau is the smallest margin that keeps
 * it among the reads left (+inf if none).  accept_frac and agreement (may be
 * NULL) report the result.  Host only.  Errors: EINVAL (NULL, target outside
 * [0, 1]). */
maxss_status maxss_choose_acceptance(uint32_t n, const float* margin, const int32_t* best_score,
                                     const uint8_t* correct, float target, float* tau,
                                     int32_t* min_score, float* accept_frac, float* agreement);

/* ---------------------------------------------------------------- SAM output
 * Mapping quality and SAM records (Methods, paragraph on mapping qualities,
 * read lengths, SAM output and source code; the 0.9 ratio rule of the
 * first-phase paragraph; the threshold 62 of the ancient-DNA Results). */

/* Per read: mapq[i] = the integer part of -100 log2(score[1] / score[0]),
 * capped at 254; 254 when there is no second fragment or its score is 0; 0
 * when the best score is 0 or the read is invalid.  mapped[i] (may be NULL)
 * = 1 when score[0] > 0, max(score[1], 0) * ratio_den < score[0] * ratio_num
 * (exact integers; 9/10 is the paper's rule) and mapq[i] > min_mapq (-1
 * disables; 62 is the strict setting).  Device pointers (top: n records,
 * mapq and mapped: n bytes), asynchronous on `stream`.
 * Errors: EINVAL (NULL, ratio_den = 0), EDEVICE. */
maxss_status maxss_mapq(const maxss_top2* top, uint32_t n, uint32_t ratio_num,
                        uint32_t ratio_den, int32_t min_mapq, uint8_t* mapq, uint8_t* mapped,
                        void* stream);

/* SAM header: @HD (VN:1.6, SO:unsorted), @SQ (SN:rname, LN:G), @PG.  Host
 * buffer of `cap` bytes, not NUL-terminated; *len = bytes written, or needed
 * when the call fails with EINVAL because cap is too small.
 * Errors: EINVAL (NULL, rname empty or not printable without spaces, cap). */
maxss_status maxss_sam_header(const maxss_index* index, const char* rname, char* buf,
                              uint64_t cap, uint64_t* len);

/* One SAM line per read, in read order, from host copies of the first and
 * second phase's outputs: QNAME (names[i], or "r<i>" when names is NULL),
 * FLAG (0, 16 for the reverse strand, 4 unmapped), RNAME, POS (ref_begin+1),
 * MAPQ, CIGAR (the extended =/X/I/D string, "*" if truncated), RNEXT "*",
 * PNEXT 0, TLEN 0, SEQ (the read on the forward genome strand: reverse
 * complement for strand 1), QUAL (reads->qual in the order of SEQ, reversed
 * for strand 1; "*" when reads->qual is NULL), then AS:i:<NW score>.  An
 * unmapped read has RNAME "*", POS 0, MAPQ 0, CIGAR "*", SEQ as given (upper
 * case) and QUAL as given; a read the scan marked invalid has SEQ and QUAL
 * "*".  All pointers are host pointers:
 * reads (on_device = 0), top and aln (n records), cigar (n * cigar_stride
 * bytes, NUL-terminated rows as written by maxss_align_top), mapq and mapped
 * (n bytes, from maxss_mapq).  Output as for maxss_sam_header.
 * Errors: EINVAL (NULL, device reads, bad names, a quality outside '!'..'~',
 * cap), with *len = needed. */
maxss_status maxss_sam_records(const maxss_reads* reads, const maxss_top2* top,
                               const maxss_aln* aln, const char* cigar, uint64_t cigar_stride,
                               const uint8_t* mapq, const uint8_t* mapped, const char* rname,
                               const char* const* names, char* buf, uint64_t cap,
                               uint64_t* len);

/* Kernel timing for measurement.  maxss_profile_enable(1) clears the records
 * and brackets every later launch of the library's kernels with HIP events on
 * the launch stream; maxss_profile_enable(0) stops recording.
 * maxss_profile_read waits for the recorded events of the kernel `name`
 * ("encode", "scan", "merge", "rescan", "nw", "profile", "gemm", "pair",
 * "topk") and returns their summed
 * duration in milliseconds and the number of launches.  Not for use while a
 * stream is being captured into a graph.  Errors: EINVAL (NULL), EDEVICE. */
maxss_status maxss_profile_enable(int on);
maxss_status maxss_profile_read(const char* name, double* total_ms, uint32_t* launches);

/* Measured roof of the scan's instruction class on the current device: the
 * issue rate of packed 16-bit saturating integer adds (v_pk_add_i16), in
 * 16-bit lane operations per second, from four launches of a kernel whose
 * lanes each run eight independent add chains with eight waves per SIMD (the
 * best of the last three).  The nominal figure it is set beside is CUs x 64
 * lanes x 2 halves x clock.  Synchronous on `stream` (NULL = default);
 * allocates a small buffer.  Errors: EINVAL (NULL), EDEVICE. */
maxss_status maxss_roof_int16(double* ops_per_s, void* stream);

/* Test hook for the out-of-memory paths: the n-th device allocation the
 * library makes from now on (any thread, any call) fails with MAXSS_ENOMEM
 * without allocating, as an exhausted device would; later allocations
 * succeed again.  n = 0 turns the hook off.  Every call releases what it
 * allocated before the failure and leaves its inputs untouched.  Host only;
 * always MAXSS_OK. */
maxss_status maxss_fail_alloc_after(uint32_t n);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* maxss_last_error(void);

/* Library version string. */
const char* maxss_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MAXSS_H */
