// First phase: MaxSS scan of every read against every fragment, top-2
// fragments per read (HIP, gfx950).
//
// What is computed (Methods, "Maximum scoring subsequence" and "First phase of
// MaxSSmap"; Figure 1): for read i, strand s, fragment f and offset o in
// [0, F), the window starting at p = f*F + o is scored with the maximum
// scoring subsequence of the substitution scores sigma(q_s[k], g[p+k]),
// k < m, i.e. the Kadane recurrence H = max(0, H + sigma), B = max(B, H).
// A fragment's value is the max over (s, o); a read keeps its two best
// fragments.
//
// How (gfx950 design, not the paper's Fermi layout):
//   * A wave owns 128*NP start offsets of one fragment: lane l holds NP
//     packed pairs of offsets (l*NP + j, l*NP + j + 64*NP), or, when every
//     other read base is scored, (2(l*NP + j), 2(l*NP + j) + 1).  The read
//     base of step k is wave-uniform.
//   * The two 16-bit substitution scores of a pair come from one v_perm_b32:
//     the selector word (from the genome, staged in LDS) picks, for each of
//     the two genome bases, a byte of the step's 8-byte score pool and the
//     byte's sign extension (pool bytes 1,3,5,7 hold the scores against
//     A,C,G,T; bytes 0,2 the score and sign of a genome N).  The pool is
//     built on the scalar unit from the read base's 4-bit code, staged in
//     LDS per read tile: pool = all-mismatch pool ^ ((M ^ X) << 8*code).
//   * Kadane runs on packed int16 with a -32768 bias: with H' = H - 32768,
//     max(0, H + sigma) is exactly the signed-saturating add H' + sigma
//     (v_pk_add_i16 with clamp) as long as H + sigma stays below 65536, which
//     max_read_len * match <= 65535 guarantees.  When the bound is at most
//     31744, two steps share one v_pk_minimum3_f16 for B' = max(B', H'_t,
//     H'_t+1) (the biased values read as binary16 fall as h grows), so each
//     pair of cells costs five VALU instructions per two steps; above it,
//     B' = max(B', H') is one v_pk_max_i16 per step (three per step).
//   * NP = 16 with plain scores (scan_kernel_bank): the select moves out of
//     the loop.  The four per-base score pairs of every window word are
//     built once, when the word enters the register window, and a step
//     reads the bank of its read base through the VGPR index mode, so the
//     loop is 1.75 instructions per pair and step (add, half a minimum3, a
//     quarter of a v_perm_b32).
//   * The window of selector words a lane needs slides by one per step; it is
//     kept in registers (2*NP words) and refilled from LDS every NP steps.
//   * A persistent grid pulls (read tile x fragment chunk) work items from an
//     atomic counter; per-read top-2 live in lane-indexed registers; a merge
//     kernel combines chunks; the two winners are re-scanned exactly for the
//     representative strand and offset.
#include <math.h>
#include <stdint.h>

#include <cmath>
#include <map>
#include <mutex>
#include <utility>

#include "internal.h"

namespace maxss {

typedef short s16x2 __attribute__((ext_vector_type(2)));

// Selector halfword of a base code: (low byte selector, high byte selector).
__device__ inline uint32_t sel16(uint32_t code) {
  // A: (1, 8)  C: (3, 9)  G: (5, 10)  T: (7, 11)  N: (0, 2)
  return code == kN ? 0x0200u : ((2u * code + 1u) | ((8u + code) << 8));
}

__device__ inline uint32_t genome_code(const uint32_t* __restrict__ g2,
                                       const uint32_t* __restrict__ nm, uint64_t Lpad,
                                       uint64_t P) {
  if (P >= Lpad) return kN;
  if ((nm[P >> 5] >> (P & 31)) & 1u) return kN;
  return (g2[P >> 4] >> (2 * (P & 15))) & 3u;
}

// LDS slot of window word w: one padding word every NP words, so that the
// 64 lanes reading words l*NP + c hit 64 distinct banks.
template <int NP>
__device__ inline uint32_t phys(uint32_t w) {
  return w + w / NP;
}

struct ScanArgs {
  const uint32_t* g2;
  const uint32_t* nmask;
  uint64_t Lpad;
  uint32_t F, NF, nseg;
  const uint32_t* sel4;   // [n][2][cwg] 4-bit pool-shift codes
  uint32_t cwg;           // code words per read strand in sel4 (mstride / 8)
  uint32_t cw;            // code words per read strand in LDS (cwg + NP / 8 + 1)
  uint32_t win_slots;     // LDS words reserved for the genome window
  uint64_t xpool;         // all-mismatch score pool
  uint64_t dpool;         // (M ^ X) & 0xFF: flips one pool byte to the match score
  const uint32_t* lens;
  const uint32_t* order;
  uint32_t n;
  uint32_t R, ntiles, nchunks;
  uint32_t total_work;
  uint32_t* work_ctr;
  int4* partial;
  uint32_t nstrands;
  uint32_t mp_max;  // largest padded read length of the call
  const int32_t* cand;  // NULL, or per read K candidate fragments (ascending)
  uint32_t K;
  uint32_t nfe;         // fragments (or candidates) each tile iterates
  uint32_t step;        // 1, or 2 for the fast scan (every other read base)
  const uint16_t* qsc;  // quality mode: [n][mp_max] (match | mismatch << 8) per position
  uint32_t cq;          // LDS words of position-score pairs per read strand
  const int32_t* excl;  // NULL, or per read a fragment e: e-1, e, e+1 never enter its top-2
  // quality mode, one of two launches: 1 takes the reads whose positions all
  // share one (match, mismatch) pair, 2 the others; 0: every read
  uint32_t qsplit;
};

// The all-mismatch score pool of mismatch score x (int8): bytes
// [X, X, sign(X), X, 0, X, 0, X].
__host__ __device__ inline uint64_t mismatch_pool(uint32_t x8) {
  x8 &= 0xFFu;
  const uint64_t sx = (x8 & 0x80u) ? 0xFFull : 0ull;
  return (uint64_t)x8 | ((uint64_t)x8 << 8) | (sx << 16) | ((uint64_t)x8 << 24) |
         ((uint64_t)x8 << 40) | ((uint64_t)x8 << 56);
}

template <int NP>
__device__ inline uint32_t staged_words(uint32_t mp) {
  return 64u * NP + mp + 2u * NP;
}

// LDS words the genome window of a tile needs (with the bank padding).
inline uint32_t win_slots_for(int NP, uint32_t mp_max) {
  const uint32_t w = 64u * NP + mp_max + 2u * NP;
  return w + w / NP + 1;
}

// 8 codes (4 bits each) of positions [k, k+8) of a strand, from its LDS code
// words (uniform; scalar after readfirstlane).
__device__ inline uint32_t codes8(const uint32_t* __restrict__ lc, uint32_t k) {
  const uint32_t w = k >> 3, sh = 4u * (k & 7u);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(lc[w]);
  const uint32_t hi = __builtin_amdgcn_readfirstlane(lc[w + 1]);
  return (uint32_t)((((uint64_t)hi << 32) | lo) >> sh);
}

// LDS word x (uniform) of the window that starts at lane*NP: with one pad
// word every NP words, its slot is lane*(NP+1) + x + x/NP (lane*NP is a
// multiple of NP, so only the uniform part needs the division).
template <int NP>
__device__ inline uint32_t win_word(const uint32_t* __restrict__ lds, uint32_t lbase,
                                    uint32_t x) {
  return lds[lbase + (x + x / NP)];
}

// The score pool of one step.  Plain scoring: the all-mismatch pool with the
// read base's byte flipped to the match score.  Quality mode: the same
// construction from the position's own pair (low byte match, high byte
// mismatch, int8 each): bytes [X, X, sign(X), X, 0, X, 0, X], then the read
// base's byte flipped to M.
template <bool QS>
__device__ inline uint64_t step_pool(uint32_t c, uint32_t pair, uint64_t xpool, uint64_t dpool) {
  if constexpr (QS) {
    const uint32_t sm = pair & 0xFFu, sx = (pair >> 8) & 0xFFu;
    const uint32_t sg = (sx & 0x80u) ? 0xFFu : 0u;
    const uint32_t lo = sx | (sx << 8) | (sg << 16) | (sx << 24);
    const uint32_t hi = (sx << 8) | (sx << 24);
    const uint64_t xp = ((uint64_t)hi << 32) | lo;
    return xp ^ ((uint64_t)((sm ^ sx) & 0xFFu) << (c << 3));
  } else {
    (void)pair;
    return xpool ^ (dpool << (c << 3));
  }
}

// One Kadane step of one offset pair: v_perm_b32 for the two scores,
// v_pk_add_i16 with clamp for H, v_pk_max_i16 for B.
__device__ inline void kadane_one(s16x2& H, s16x2& B, uint32_t w, uint32_t lo, uint32_t hi) {
  H = __builtin_elementwise_add_sat(H, __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(hi, lo, w)));
  B = __builtin_elementwise_max(B, H);
}

// Two Kadane steps of two offset pairs (interleaved, so that no add reads
// the result of the instruction right before it).  The biased values
// h - 32768 (h in [0, 31744]) read as binary16 are -0 and negative numbers
// that decrease strictly as h grows (subnormals included, which the kernels
// keep), so the IEEE minimum of three such values is the largest h:
// B' = max(B', H'_t, H'_t+1) is one v_pk_minimum3_f16, five VALU
// instructions per pair and two steps.
__device__ inline void kadane_two(s16x2& Ha, s16x2& Ba, uint32_t wa0, uint32_t wa1, s16x2& Hb,
                                  s16x2& Bb, uint32_t wb0, uint32_t wb1, uint32_t lo0,
                                  uint32_t hi0, uint32_t lo1, uint32_t hi1) {
  typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
  const s16x2 sa0 = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(hi0, lo0, wa0));
  const s16x2 sb0 = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(hi0, lo0, wb0));
  const s16x2 ha = __builtin_elementwise_add_sat(Ha, sa0);
  const s16x2 hb = __builtin_elementwise_add_sat(Hb, sb0);
  const s16x2 sa1 = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(hi1, lo1, wa1));
  const s16x2 sb1 = __builtin_bit_cast(s16x2, __builtin_amdgcn_perm(hi1, lo1, wb1));
  Ha = __builtin_elementwise_add_sat(ha, sa1);
  Hb = __builtin_elementwise_add_sat(hb, sb1);
  Ba = __builtin_bit_cast(
      s16x2, __builtin_elementwise_minimum(
                 __builtin_elementwise_minimum(__builtin_bit_cast(f16x2, Ba),
                                               __builtin_bit_cast(f16x2, ha)),
                 __builtin_bit_cast(f16x2, Ha)));
  Bb = __builtin_bit_cast(
      s16x2, __builtin_elementwise_minimum(
                 __builtin_elementwise_minimum(__builtin_bit_cast(f16x2, Bb),
                                               __builtin_bit_cast(f16x2, hb)),
                 __builtin_bit_cast(f16x2, Hb)));
}

// Pair of scan position t of a block whose pairs were read into qw (two
// positions per word, the block starting at an even position).
__device__ inline uint32_t pair_at(const uint32_t* qw, int t) {
  return (qw[t >> 1] >> (16 * (t & 1))) & 0xFFFFu;
}

// SUB Kadane steps (SUB <= 8) at read positions [k, k+SUB) (k even), with the
// window loaded from LDS for exactly these steps.  WIDE (scores may pass
// 31744): B' = max(B', H') after every step; otherwise two steps at a time
// with one packed minimum3 for B (kadane_two).
template <int NP, int SUB, bool QS, bool WIDE>
__device__ inline void kadane_sub(const uint32_t* __restrict__ lds, uint32_t lbase,
                                  const uint32_t* __restrict__ lc,
                                  const uint32_t* __restrict__ lq, uint32_t k, uint64_t xpool,
                                  uint64_t dpool, s16x2 (&H)[NP], s16x2 (&B)[NP]) {
  uint32_t win[NP + SUB - 1];
#pragma unroll
  for (int i = 0; i < NP + SUB - 1; i++) win[i] = win_word<NP>(lds, lbase, k + i);
  const uint32_t cc = codes8(lc, k);
  uint32_t qw[(SUB + 1) / 2];
#pragma unroll
  for (int i = 0; i < (SUB + 1) / 2; i++)
    qw[i] = QS ? __builtin_amdgcn_readfirstlane(lq[k / 2 + i]) : 0u;
  constexpr int PAIRED = WIDE ? 0 : SUB & ~1;
#pragma unroll
  for (int t = 0; t < PAIRED; t += 2) {
    const uint64_t p0 = step_pool<QS>((cc >> (4 * t)) & 15u, pair_at(qw, t), xpool, dpool);
    const uint64_t p1 =
        step_pool<QS>((cc >> (4 * t + 4)) & 15u, pair_at(qw, t + 1), xpool, dpool);
#pragma unroll
    for (int j = 0; j < NP; j += 2)
      kadane_two(H[j], B[j], win[j + t], win[j + t + 1], H[j + 1], B[j + 1], win[j + t + 1],
                 win[j + t + 2], (uint32_t)p0, (uint32_t)(p0 >> 32), (uint32_t)p1,
                 (uint32_t)(p1 >> 32));
  }
#pragma unroll
  for (int t = PAIRED; t < SUB; t++) {
    const uint64_t pool = step_pool<QS>((cc >> (4 * t)) & 15u, pair_at(qw, t), xpool, dpool);
#pragma unroll
    for (int j = 0; j < NP; j++)
      kadane_one(H[j], B[j], win[j + t], (uint32_t)pool, (uint32_t)(pool >> 32));
  }
}

// One NP-step block: steps kb..kb+NP-1 use window words first[0..NP) (words
// kb..kb+NP-1 of the lane) and second[0..NP) (words kb+NP..kb+2NP-1).
// first[t] is last read at step t, so right after step t it is reloaded with
// word kb+2NP+t: the block after next finds it there as its `second` half.
template <int NP, bool QS, bool WIDE>
__device__ inline void kadane_block(uint32_t (&first)[NP], const uint32_t (&second)[NP],
                                    const uint32_t* __restrict__ lw, const uint32_t (&cc)[NP / 8],
                                    const uint32_t* __restrict__ lqb, uint64_t xpool,
                                    uint64_t dpool, s16x2 (&H)[NP], s16x2 (&B)[NP]) {
  uint32_t qw[NP / 2];
#pragma unroll
  for (int i = 0; i < NP / 2; i++) qw[i] = QS ? __builtin_amdgcn_readfirstlane(lqb[i]) : 0u;
  if constexpr (WIDE) {
#pragma unroll
    for (int t = 0; t < NP; t++) {
      const uint64_t pool =
          step_pool<QS>((cc[t >> 3] >> (4 * (t & 7))) & 15u, pair_at(qw, t), xpool, dpool);
#pragma unroll
      for (int j = 0; j < NP; j++)
        kadane_one(H[j], B[j], (j + t < NP) ? first[j + t] : second[j + t - NP], (uint32_t)pool,
                   (uint32_t)(pool >> 32));
      first[t] = lw[t];
    }
  } else {
#pragma unroll
    for (int t = 0; t < NP; t += 2) {
      const uint64_t p0 =
          step_pool<QS>((cc[t >> 3] >> (4 * (t & 7))) & 15u, pair_at(qw, t), xpool, dpool);
      const uint64_t p1 = step_pool<QS>((cc[(t + 1) >> 3] >> (4 * ((t + 1) & 7))) & 15u,
                                        pair_at(qw, t + 1), xpool, dpool);
#pragma unroll
      for (int j = 0; j < NP; j += 2) {
        const uint32_t w0 = (j + t < NP) ? first[j + t] : second[j + t - NP];
        const uint32_t w1 = (j + t + 1 < NP) ? first[j + t + 1] : second[j + t + 1 - NP];
        const uint32_t w2 = (j + t + 2 < NP) ? first[j + t + 2] : second[j + t + 2 - NP];
        kadane_two(H[j], B[j], w0, w1, H[j + 1], B[j + 1], w1, w2, (uint32_t)p0,
                   (uint32_t)(p0 >> 32), (uint32_t)p1, (uint32_t)(p1 >> 32));
      }
      first[t] = lw[t];  // words t and t+1 are last read by the steps above
      first[t + 1] = lw[t + 1];
    }
  }
}

// Kadane over one read strand of length m for this lane's NP offset pairs.
// lc: the strand's 4-bit codes in LDS.  Full NP-step blocks first (window in
// two register halves that swap roles every block), then the last m % NP
// steps as unrolled sub-blocks of 8/4/2/1 steps, so no padding step is
// computed.  Returns the lane's per-pair maxima (biased by -32768) in B.
template <int NP, bool QS, bool WIDE>
__device__ inline void kadane_pairs(const uint32_t* __restrict__ lds, uint32_t lane,
                                    const uint32_t* __restrict__ lc,
                                    const uint32_t* __restrict__ lq, uint32_t m,
                                    uint64_t xpool, uint64_t dpool, s16x2 (&B)[NP]) {
  constexpr int CW = NP / 8;
  s16x2 H[NP];
  const s16x2 lo = {(short)-32768, (short)-32768};
#pragma unroll
  for (int j = 0; j < NP; j++) {
    H[j] = lo;
    B[j] = lo;
  }
  const uint32_t lbase = lane * (NP + 1);
  const uint32_t mfull = m / NP * NP;
  if (mfull) {
    uint32_t wA[NP], wB[NP];
    uint32_t cn[CW];
#pragma unroll
    for (int i = 0; i < NP; i++) {
      wA[i] = win_word<NP>(lds, lbase, i);
      wB[i] = win_word<NP>(lds, lbase, NP + i);
    }
#pragma unroll
    for (int i = 0; i < CW; i++) cn[i] = __builtin_amdgcn_readfirstlane(lc[i]);
    // pb = kb + kb/NP: slot offset of word kb; word kb + 2*NP + i (i < NP)
    // sits at pb + 2*(NP+1) + i.  Reloads stay inside the staged window
    // (lane*NP + m + 2*NP words), code prefetches inside m/8 + NP/8 + 1.
    uint32_t pb = 0, kb = 0;
    for (; kb + 2 * NP <= mfull; kb += 2 * NP, pb += 2 * (NP + 1)) {
      uint32_t cc[CW];
#pragma unroll
      for (int i = 0; i < CW; i++) cc[i] = cn[i];
#pragma unroll
      for (int i = 0; i < CW; i++) cn[i] = __builtin_amdgcn_readfirstlane(lc[(kb + NP) / 8 + i]);
      kadane_block<NP, QS, WIDE>(wA, wB, lds + lbase + pb + 2 * (NP + 1), cc, lq + kb / 2, xpool,
                           dpool, H, B);
#pragma unroll
      for (int i = 0; i < CW; i++) cc[i] = cn[i];
#pragma unroll
      for (int i = 0; i < CW; i++)
        cn[i] = __builtin_amdgcn_readfirstlane(lc[(kb + 2 * NP) / 8 + i]);
      kadane_block<NP, QS, WIDE>(wB, wA, lds + lbase + pb + 3 * (NP + 1), cc, lq + (kb + NP) / 2,
                           xpool, dpool, H, B);
    }
    if (kb < mfull) {  // one block left
      uint32_t cc[CW];
#pragma unroll
      for (int i = 0; i < CW; i++) cc[i] = cn[i];
      kadane_block<NP, QS, WIDE>(wA, wB, lds + lbase + pb + 2 * (NP + 1), cc, lq + kb / 2, xpool,
                           dpool, H, B);
    }
  }
  const uint32_t rem = m - mfull;
  uint32_t k = mfull;
  if (NP > 16 && (rem & 16)) {
    kadane_sub<NP, 8, QS, WIDE>(lds, lbase, lc, lq, k, xpool, dpool, H, B);
    kadane_sub<NP, 8, QS, WIDE>(lds, lbase, lc, lq, k + 8, xpool, dpool, H, B);
    k += 16;
  }
  if (NP > 8 && (rem & 8)) {
    kadane_sub<NP, 8, QS, WIDE>(lds, lbase, lc, lq, k, xpool, dpool, H, B);
    k += 8;
  }
  if (rem & 4) { kadane_sub<NP, 4, QS, WIDE>(lds, lbase, lc, lq, k, xpool, dpool, H, B); k += 4; }
  if (rem & 2) { kadane_sub<NP, 2, QS, WIDE>(lds, lbase, lc, lq, k, xpool, dpool, H, B); k += 2; }
  if (rem & 1) kadane_sub<NP, 1, QS, WIDE>(lds, lbase, lc, lq, k, xpool, dpool, H, B);
}

// ---------------------------------------------------------------------------
// Register-bank Kadane (NP = 16, plain scores, score bound <= 31744).
//
// For each of the lane's 32 window words (the current block's 16 and the
// next block's 16) and each read base b in {A, C, G, T}, the pair of scores
// sigma(b, genome) is computed once, when the word enters the window, by one
// v_perm_b32 from b's score pool: 128 bank registers, bank b holding slot s
// in v[64 + 32 b + s].  A Kadane step then has no select: with the VGPR
// index mode set to 32 b on source 0 for the step's read base b, one
// v_pk_add_i16 per offset pair reads the right bank.  A read N mismatches
// every genome base, so its steps add the constant pair (X, X) (a branch on
// the uniform code).  Per offset pair and two steps: two adds and one
// minimum3, plus four perms per window word, i.e. per 16 pairs.
//
// Register map: banks v64..v191, H v192..v207 (pair j in v192 + j), T (the
// value after an even step) v208..v223 (pair j in v208 + (j + 1) % 16), B
// v224..v239 (pair j in v224 + (j + 2) % 16), staging of the words that
// enter the window v240..v255.  The rotations put the three sources of each
// minimum3 in three different VGPR banks (register number mod 4); measured
// 0.3% faster than the same slot for all three.  The kernels that use these helpers limit the compiler to
// v0..v63 (amdgpu_num_vgpr), so the state persists between the asm
// statements below; each statement lists the registers it touches as
// clobbers, so that the kernel allocates them.  M0, which the index mode
// overwrites, is saved and restored inside each statement.

#pragma clang diagnostic push
// v64..v255 are outside the compiler's range in the bank kernel; listing them
// as clobbers is what makes the kernel allocate them.
#pragma clang diagnostic ignored "-Winline-asm"
#define MAXSS_V10(p) p "0", p "1", p "2", p "3", p "4", p "5", p "6", p "7", p "8", p "9"
#define MAXSS_BANK_CLOBBERS                                                               \
  "v64", "v65", "v66", "v67", "v68", "v69", MAXSS_V10("v7"), MAXSS_V10("v8"),            \
      MAXSS_V10("v9"), MAXSS_V10("v10"), MAXSS_V10("v11"), MAXSS_V10("v12"),             \
      MAXSS_V10("v13"), MAXSS_V10("v14"), MAXSS_V10("v15"), MAXSS_V10("v16"),            \
      MAXSS_V10("v17"), MAXSS_V10("v18"), MAXSS_V10("v19"), MAXSS_V10("v20"),            \
      MAXSS_V10("v21"), MAXSS_V10("v22"), MAXSS_V10("v23"), MAXSS_V10("v24"), "v250",    \
      "v251", "v252", "v253", "v254", "v255"

#define MAXSS_IRP16 "0,1,2,3,4,5,6,7,8,9,10,11,12,13,14,15"

// The read codes reach these helpers as bytes 16c (c = 1, 3, 5, 7 for A, C,
// G, T; 4 for N), four per word.  16c = 32b + 16 for base b, so an add that
// names v[48 + slot] reads bank b at v[64 + 32b + slot] when the index is
// the code byte itself; s_set_gpr_idx_on takes the low byte of its operand.

// Code word of step t (c0..c3 hold steps 0-3, 4-7, 8-11, 12-15), and an
// instruction PRE cN POST on it.
#define MAXSS_BANK_CW                                                             \
  ".if \\t < 4\n.set maxss_cwn, 0\n.elseif \\t < 8\n.set maxss_cwn, 1\n"          \
  ".elseif \\t < 12\n.set maxss_cwn, 2\n.else\n.set maxss_cwn, 3\n.endif\n"
#define MAXSS_SEL4(PRE, POST)                                                     \
  ".if maxss_cwn == 0\n" PRE "%[c0]" POST "\n"                                    \
  ".elseif maxss_cwn == 1\n" PRE "%[c1]" POST "\n"                                \
  ".elseif maxss_cwn == 2\n" PRE "%[c2]" POST "\n"                                \
  ".else\n" PRE "%[c3]" POST "\n.endif\n"

// The adds of step t (even: T = bank + H; odd: H = bank + T), index mode on.
#define MAXSS_BANK_ADDS                                                           \
  ".irp j, " MAXSS_IRP16 "\n"                                                     \
  ".if (\\t & 1) == 0\n"                                                          \
  "v_pk_add_i16 v[208+((\\j+1)&15)], v[48+((\\j+\\t+%[f])&31)], v[192+\\j] clamp\n"  \
  ".else\n"                                                                       \
  "v_pk_add_i16 v[192+\\j], v[48+((\\j+\\t+%[f])&31)], v[208+((\\j+1)&15)] clamp\n"  \
  ".endif\n"                                                                      \
  ".endr\n"

// B = max(B, T, H) after an odd step.
#define MAXSS_BANK_MAX3                                                           \
  ".irp j, " MAXSS_IRP16 "\n"                                                     \
  "v_pk_minimum3_f16 v[224+((\\j+2)&15)], v[224+((\\j+2)&15)], v[208+((\\j+1)&15)], v[192+\\j]\n" \
  ".endr\n"

// Step t of a block with no N: the index switches on at even steps (the code
// word itself at steps 0, 4, 8, 12), changes at odd steps, and switches off
// before the minimum3.
#define MAXSS_BANK_FAST_STEP                                                      \
  MAXSS_BANK_CW                                                                   \
  ".if (\\t & 3) == 0\n"                                                          \
  MAXSS_SEL4("s_set_gpr_idx_on ", ", gpr_idx(SRC0)")                              \
  ".else\n"                                                                       \
  MAXSS_SEL4("s_lshr_b32 %[sc], ", ", 8*(\\t&3)")                                 \
  ".if (\\t & 1) == 0\n"                                                          \
  "s_set_gpr_idx_on %[sc], gpr_idx(SRC0)\n"                                       \
  ".else\n"                                                                       \
  "s_set_gpr_idx_idx %[sc]\n"                                                     \
  ".endif\n"                                                                      \
  ".endif\n"                                                                      \
  MAXSS_BANK_ADDS                                                                 \
  ".if (\\t & 1) == 1\n"                                                          \
  "s_set_gpr_idx_off\n" MAXSS_BANK_MAX3                                           \
  ".endif\n"

// Step t of a block with an N (or of the tail): code byte, N branch.
#define MAXSS_BANK_SLOW_STEP(L)                                                   \
  MAXSS_BANK_CW                                                                   \
  MAXSS_SEL4("s_bfe_u32 %[sc], ", ", (8*(\\t&3))|0x80000")                        \
  "s_cmp_eq_u32 %[sc], 0x40\n"                                                    \
  "s_cbranch_scc1 .L" L "N%=_\\t\n"                                               \
  "s_set_gpr_idx_on %[sc], gpr_idx(SRC0)\n"                                       \
  MAXSS_BANK_ADDS                                                                 \
  "s_set_gpr_idx_off\n"                                                           \
  ".L" L "R%=_\\t:\n"                                                             \
  ".if (\\t & 1) == 1\n" MAXSS_BANK_MAX3 ".endif\n"

// The out-of-line N steps of MAXSS_BANK_SLOW_STEP: add (X, X).
#define MAXSS_BANK_NSTEP(L)                                                       \
  ".L" L "N%=_\\t:\n"                                                             \
  ".irp j, " MAXSS_IRP16 "\n"                                                     \
  ".if (\\t & 1) == 0\n"                                                          \
  "v_pk_add_i16 v[208+((\\j+1)&15)], %[xx], v[192+\\j] clamp\n"                      \
  ".else\n"                                                                       \
  "v_pk_add_i16 v[192+\\j], %[xx], v[208+((\\j+1)&15)] clamp\n"                      \
  ".endif\n"                                                                      \
  ".endr\n"                                                                       \
  "s_branch .L" L "R%=_\\t\n"

// The four bank words of window slot S from the staged selector word W.
#define MAXSS_BANK_FILL(S, W)                                                     \
  "v_perm_b32 v[64+" S "], %[h0], %[l0], v[240+" W "]\n"                          \
  "v_perm_b32 v[96+" S "], %[h1], %[l1], v[240+" W "]\n"                          \
  "v_perm_b32 v[128+" S "], %[h2], %[l2], v[240+" W "]\n"                         \
  "v_perm_b32 v[160+" S "], %[h3], %[l3], v[240+" W "]\n"

#define MAXSS_BANK_POOLS                                                          \
  [l0] "v"(pl[0]), [l1] "v"(pl[1]), [l2] "v"(pl[2]), [l3] "v"(pl[3]), [h0] "s"(ph[0]), \
      [h1] "s"(ph[1]), [h2] "s"(ph[2]), [h3] "s"(ph[3])

__device__ inline uint32_t lds_byte_addr(const uint32_t* p) {
  typedef __attribute__((address_space(3))) const uint32_t lds_u32;
  return (uint32_t)(uintptr_t)(lds_u32*)p;
}

// H = B = 0 (biased) and the banks of window words 0..31 (LDS words at byte
// address la: words 0..15, then a pad word, then words 16..31).
__device__ inline void bank_init(uint32_t la, const uint32_t (&pl)[4], const uint32_t (&ph)[4]) {
  asm volatile(
      ".irp i, 0,2,4,6,8,10,12,14\n"
      "ds_read2_b32 v[240+\\i:241+\\i], %[la] offset0:\\i offset1:\\i+1\n"
      ".endr\n"
      ".irp j, 0,2,4,6,8,10,12,14\n"
      "v_mov_b64 v[192+\\j:193+\\j], %[zero]\n"
      "v_mov_b64 v[224+\\j:225+\\j], %[zero]\n"
      ".endr\n"
      "s_waitcnt lgkmcnt(0)\n"
      // words 16..23 are loaded while slots 8..15 fill, words 24..31 while
      // slots 16..23 fill
      ".irp s, 0,1,2,3,4,5,6,7\n" MAXSS_BANK_FILL("\\s", "\\s") ".endr\n"
      ".irp i, 0,2,4,6\n"
      "ds_read2_b32 v[240+\\i:241+\\i], %[la] offset0:17+\\i offset1:18+\\i\n"
      ".endr\n"
      ".irp s, 8,9,10,11,12,13,14,15\n" MAXSS_BANK_FILL("\\s", "\\s") ".endr\n"
      ".irp i, 8,10,12,14\n"
      "ds_read2_b32 v[240+\\i:241+\\i], %[la] offset0:17+\\i offset1:18+\\i\n"
      ".endr\n"
      "s_waitcnt lgkmcnt(4)\n"
      ".irp s, 0,1,2,3,4,5,6,7\n" MAXSS_BANK_FILL("16+\\s", "\\s") ".endr\n"
      "s_waitcnt lgkmcnt(0)\n"
      ".irp s, 8,9,10,11,12,13,14,15\n" MAXSS_BANK_FILL("16+\\s", "\\s") ".endr\n"
      :
      : [la] "v"(la), [zero] "s"(0x8000800080008000ull), MAXSS_BANK_POOLS
      : "memory", MAXSS_BANK_CLOBBERS);
}

// One block of 16 steps whose current window words sit in slots FIRST..
// FIRST+15 (the next block's in the other 16).  The 16 words that replace
// the current ones (LDS byte address la) are staged at the start and fill
// slot FIRST+s four steps after its last use (slots 12..15 at the end).
// c0..c3: the code bytes of the 16 read positions.  A block without N
// (every code byte has bit 4 set) takes the fast step sequence.  The last
// block of a read (RELOAD false) stages nothing: the tail fills the few
// words it still needs.
#define MAXSS_BANK_RELOAD                                                         \
  ".if %[rl]\n"                                                                   \
  ".if \\t == 4\n"                                                                \
  "s_waitcnt lgkmcnt(0)\n"                                                        \
  ".endif\n"                                                                      \
  ".if \\t >= 4\n" MAXSS_BANK_FILL("%[f]+\\t-4", "\\t-4") ".endif\n"             \
  ".endif\n"

template <int FIRST, bool RELOAD>
__device__ inline void bank_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                  uint32_t la, const uint32_t (&pl)[4],
                                  const uint32_t (&ph)[4], uint32_t xx) {
  uint32_t sc, sm;
  asm volatile(
      "s_mov_b32 %[sm], m0\n"
      ".if %[rl]\n"
      ".irp i, 0,2,4,6,8,10,12,14\n"
      "ds_read2_b32 v[240+\\i:241+\\i], %[la] offset0:\\i offset1:\\i+1\n"
      ".endr\n"
      ".endif\n"
      "s_and_b32 %[sc], %[c0], %[c1]\n"
      "s_and_b32 %[sc], %[sc], %[c2]\n"
      "s_and_b32 %[sc], %[sc], %[c3]\n"
      "s_and_b32 %[sc], %[sc], 0x10101010\n"
      "s_cmp_eq_u32 %[sc], 0x10101010\n"
      "s_cbranch_scc0 .LbS%=\n"
      ".irp t, " MAXSS_IRP16 "\n" MAXSS_BANK_FAST_STEP MAXSS_BANK_RELOAD ".endr\n"
      ".if %[rl]\n"
      ".irp s, 12,13,14,15\n" MAXSS_BANK_FILL("%[f]+\\s", "\\s") ".endr\n"
      ".endif\n"
      "s_branch .LbE%=\n"
      ".LbS%=:\n"
      ".irp t, " MAXSS_IRP16 "\n" MAXSS_BANK_SLOW_STEP("b") MAXSS_BANK_RELOAD ".endr\n"
      ".if %[rl]\n"
      ".irp s, 12,13,14,15\n" MAXSS_BANK_FILL("%[f]+\\s", "\\s") ".endr\n"
      ".endif\n"
      "s_branch .LbE%=\n"
      ".irp t, " MAXSS_IRP16 "\n" MAXSS_BANK_NSTEP("b") ".endr\n"
      ".LbE%=:\n"
      "s_mov_b32 m0, %[sm]\n"
      : [sc] "=&s"(sc), [sm] "=&s"(sm)
      : [c0] "s"(c0), [c1] "s"(c1), [c2] "s"(c2), [c3] "s"(c3), [la] "v"(la), [xx] "s"(xx),
        [f] "n"(FIRST), [rl] "n"(RELOAD ? 1 : 0), MAXSS_BANK_POOLS
      : "scc", "memory", MAXSS_BANK_CLOBBERS);
}

// The last rem (1..15) steps of the read, window in slots FIRST.. as in
// bank_block.  nf words (read positions mfull+16.., LDS byte address la)
// go into the other half first; no other reloads.  An even last step folds
// T into B on exit.
template <int FIRST>
__device__ inline void bank_tail(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                 uint32_t rem, uint32_t xx, uint32_t nf, uint32_t la,
                                 const uint32_t (&pl)[4], const uint32_t (&ph)[4]) {
  uint32_t sc, sm;
  asm volatile(
      "s_mov_b32 %[sm], m0\n"
      // the first nf words of the other half (LDS byte address la), which
      // the last block did not stage
      "s_cmp_eq_u32 %[nf], 0\n"
      "s_cbranch_scc1 .LtP%=\n"
      ".irp i, 0,2,4,6,8,10,12,14\n"
      "ds_read2_b32 v[240+\\i:241+\\i], %[la] offset0:\\i offset1:\\i+1\n"
      ".endr\n"
      "s_waitcnt lgkmcnt(0)\n"
      ".irp s, 0,1,2,3,4,5,6,7,8,9,10,11,12,13,14\n"
      "s_cmp_le_u32 %[nf], \\s\n"
      "s_cbranch_scc1 .LtP%=\n"
      MAXSS_BANK_FILL("%[g]+\\s", "\\s")
      ".endr\n"
      ".LtP%=:\n"
      ".irp t, 0,1,2,3,4,5,6,7,8,9,10,11,12,13,14\n"
      MAXSS_BANK_SLOW_STEP("t")
      "s_cmp_eq_u32 %[rem], \\t+1\n"
      ".if (\\t & 1) == 0\n"
      "s_cbranch_scc1 .LtX%=\n"
      ".else\n"
      "s_cbranch_scc1 .LtE%=\n"
      ".endif\n"
      ".endr\n"
      "s_branch .LtE%=\n"
      ".irp t, 0,1,2,3,4,5,6,7,8,9,10,11,12,13,14\n" MAXSS_BANK_NSTEP("t") ".endr\n"
      ".LtX%=:\n"
      ".irp j, " MAXSS_IRP16 "\n"
      "v_pk_minimum3_f16 v[224+((\\j+2)&15)], v[224+((\\j+2)&15)], v[208+((\\j+1)&15)], v[208+((\\j+1)&15)]\n"
      ".endr\n"
      ".LtE%=:\n"
      "s_mov_b32 m0, %[sm]\n"
      : [sc] "=&s"(sc), [sm] "=&s"(sm)
      : [c0] "s"(c0), [c1] "s"(c1), [c2] "s"(c2), [c3] "s"(c3), [rem] "s"(rem), [xx] "s"(xx),
        [f] "n"(FIRST), [g] "n"(FIRST ^ 16), [nf] "s"(nf), [la] "v"(la), MAXSS_BANK_POOLS
      : "scc", "memory", MAXSS_BANK_CLOBBERS);
}

__device__ inline void bank_extract(s16x2 (&B)[16]) {
  uint32_t o[16];
  asm volatile(
      "v_mov_b32 %[o0], v226\n v_mov_b32 %[o1], v227\n v_mov_b32 %[o2], v228\n"
      "v_mov_b32 %[o3], v229\n v_mov_b32 %[o4], v230\n v_mov_b32 %[o5], v231\n"
      "v_mov_b32 %[o6], v232\n v_mov_b32 %[o7], v233\n v_mov_b32 %[o8], v234\n"
      "v_mov_b32 %[o9], v235\n v_mov_b32 %[o10], v236\n v_mov_b32 %[o11], v237\n"
      "v_mov_b32 %[o12], v238\n v_mov_b32 %[o13], v239\n v_mov_b32 %[o14], v224\n"
      "v_mov_b32 %[o15], v225\n"
      : [o0] "=v"(o[0]), [o1] "=v"(o[1]), [o2] "=v"(o[2]), [o3] "=v"(o[3]), [o4] "=v"(o[4]),
        [o5] "=v"(o[5]), [o6] "=v"(o[6]), [o7] "=v"(o[7]), [o8] "=v"(o[8]), [o9] "=v"(o[9]),
        [o10] "=v"(o[10]), [o11] "=v"(o[11]), [o12] "=v"(o[12]), [o13] "=v"(o[13]),
        [o14] "=v"(o[14]), [o15] "=v"(o[15]));
#pragma unroll
  for (int j = 0; j < 16; j++) B[j] = __builtin_bit_cast(s16x2, o[j]);
}

// max(bm, B[0..15]) as one pair, by eight minimum3 on the biased values.
__device__ inline uint32_t bank_fold(uint32_t bm) {
  uint32_t r;
  asm volatile(
      "v_pk_minimum3_f16 v224, v224, v225, v226\n"
      "v_pk_minimum3_f16 v227, v227, v228, v229\n"
      "v_pk_minimum3_f16 v230, v230, v231, v232\n"
      "v_pk_minimum3_f16 v233, v233, v234, v235\n"
      "v_pk_minimum3_f16 v236, v236, v237, v238\n"
      "v_pk_minimum3_f16 v224, v224, v227, v230\n"
      "v_pk_minimum3_f16 v233, v233, v236, v239\n"
      "s_nop 0\n"
      "v_pk_minimum3_f16 %[r], v224, v233, %[bm]\n"
      : [r] "=v"(r)
      : [bm] "v"(bm)
      : "v224", "v227", "v230", "v233", "v236");
  return r;
}

// Kadane over one read strand of length m for this lane's 16 offset pairs
// with the register banks (same window layout as kadane_pairs<16, ...>); the
// per-pair maxima stay in v224..v239 (bank_extract, bank_fold).  lc: the
// strand's code bytes (four per word).  xx: the pair (X, X).
__device__ inline void kadane_pairs_bank(const uint32_t* __restrict__ lds, uint32_t lane,
                                         const uint32_t* __restrict__ lc, uint32_t m,
                                         uint64_t xpool, uint64_t dpool, uint32_t xx) {
  constexpr uint32_t NP = 16;
  uint32_t pl[4], ph[4];
#pragma unroll
  for (int b = 0; b < 4; b++) {
    const uint64_t pool = xpool ^ (dpool << (8 * (2 * b + 1)));
    pl[b] = (uint32_t)pool;
    ph[b] = (uint32_t)(pool >> 32);
  }
  const uint32_t la = lds_byte_addr(lds + lane * (NP + 1));
  bank_init(la, pl, ph);
  const uint32_t mfull = m / NP * NP, nblk = m / NP;
  // the next block's codes are read before the current block's asm, so the
  // LDS latency hides behind it
  uint32_t n[4];
#pragma unroll
  for (int i = 0; i < 4; i++) n[i] = lc[i];
  uint32_t c[4];
  // block b covers read positions 16b..16b+15; pb: padded LDS index of word
  // 16b.  Every block but the last stages the 16 words two blocks ahead.
  uint32_t b = 0, pb = 0;
  for (; b + 2 <= nblk; b += 2, pb += 2 * (NP + 1)) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      c[i] = __builtin_amdgcn_readfirstlane(n[i]);
      n[i] = lc[(b + 1) * (NP / 4) + i];
    }
    bank_block<0, true>(c[0], c[1], c[2], c[3], la + 4u * (pb + 2 * (NP + 1)), pl, ph, xx);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      c[i] = __builtin_amdgcn_readfirstlane(n[i]);
      n[i] = lc[(b + 2) * (NP / 4) + i];
    }
    if (b + 2 < nblk)
      bank_block<16, true>(c[0], c[1], c[2], c[3], la + 4u * (pb + 3 * (NP + 1)), pl, ph, xx);
    else
      bank_block<16, false>(c[0], c[1], c[2], c[3], 0u, pl, ph, xx);
  }
  bool odd = false;
  if (b < nblk) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      c[i] = __builtin_amdgcn_readfirstlane(n[i]);
      n[i] = lc[(b + 1) * (NP / 4) + i];
    }
    bank_block<0, false>(c[0], c[1], c[2], c[3], 0u, pl, ph, xx);
    odd = true;
  }
  const uint32_t rem = m - mfull;
  if (rem) {
#pragma unroll
    for (int i = 0; i < 4; i++) c[i] = __builtin_amdgcn_readfirstlane(n[i]);
    // words mfull+16 .. mfull+14+rem, which the last block did not stage
    const uint32_t nf = __builtin_amdgcn_readfirstlane((nblk > 0 && rem > 1) ? rem - 1 : 0u);
    const uint32_t w = mfull + NP;
    const uint32_t lt = la + 4u * (w + w / NP);
    if (odd) bank_tail<16>(c[0], c[1], c[2], c[3], rem, xx, nf, lt, pl, ph);
    else bank_tail<0>(c[0], c[1], c[2], c[3], rem, xx, nf, lt, pl, ph);
  }
}

#pragma clang diagnostic pop

// Maximum over the wave, by DPP within the VALU (no LDS round trip): an
// inclusive max scan (row shifts 1, 2, 4, 8, then the broadcasts of lanes 15
// and 31 into the rows above) leaves the maximum in lane 63.
__device__ inline int wave_max_i32(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xF, 0xF, false));  // row_shr:1
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xF, 0xF, false));  // row_shr:2
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xF, 0xF, false));  // row_shr:4
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xF, 0xF, false));  // row_shr:8
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// Whether every scored position of read `rid` (length L) has the pair of
// its first position, and that pair.
__device__ inline bool one_pair(const uint16_t* __restrict__ qsc, uint32_t mp_max, uint32_t rid,
                                uint32_t L, uint32_t& pair) {
  const uint16_t* qr = qsc + (uint64_t)rid * mp_max;
  pair = L ? qr[0] : 0u;
  const uint32_t two = pair * 0x10001u;
  const uint32_t* q2 = reinterpret_cast<const uint32_t*>(qr);  // rows are 128-byte aligned
  bool one = true;
  for (uint32_t k = 0; k < L / 2; k++) one &= q2[k] == two;
  if (L & 1) one &= qr[L - 1] == pair;
  return one;
}

// QB: the register-bank kernel of the quality split (qsplit 1), each read
// scored with its own pair as plain scores.
template <int NP, bool QS, bool WIDE, bool BANK, bool QB = false>
__device__ __forceinline__ void scan_body(const ScanArgs& a) {
  extern __shared__ uint32_t lds[];
  constexpr uint32_t HALF = 64u * NP, S = 128u * NP;
  const uint32_t lane = threadIdx.x;
  uint32_t* lcodes = lds + a.win_slots;
  // (X, X) as two int16 (the pool's byte 0 is X)
  const uint32_t xx = (uint32_t)(uint16_t)(int16_t)(int8_t)(a.xpool & 0xFFu) * 0x10001u;
  (void)xx;
  uint32_t* lqs = lcodes + a.R * 2 * a.cw;  // quality mode: position-score pairs
  for (;;) {
    uint32_t w = 0;
    if (lane == 0) w = atomicAdd(a.work_ctr, 1u);
    w = __builtin_amdgcn_readfirstlane(__shfl(w, 0, 64));
    if (w >= a.total_work) break;
    // tile-major order over the length-sorted tiles: every chunk of the
    // longest tile first, the shortest tiles' chunks last.  Chunks are
    // balanced (sizes differ by at most one fragment), so the items come in
    // nonincreasing cost and the last ones to start are the cheapest.
    const uint32_t tile = w / a.nchunks, chunk = w - tile * a.nchunks;
    const uint32_t rbase = tile * a.R;
    const uint32_t rcount = min(a.R, a.n - rbase);
    const uint32_t my_read = lane < rcount ? a.order[rbase + lane] : 0u;
    // Kadane steps of the read: its length, or half of it rounded up when
    // every other base is scored
    uint32_t my_len = lane < rcount ? (a.lens[my_read] + a.step - 1) / a.step : 0u;
    // quality split: this launch's reads only (a read of the other kind is
    // skipped like an empty one, and its record is the other launch's)
    uint32_t my_pair = 0;
    bool mine = true;
    if (QB || (QS && a.qsplit)) {
      if (lane < rcount) {
        mine = one_pair(a.qsc, a.mp_max, my_read, a.lens[my_read], my_pair) == QB;
        if (!mine) my_len = 0;
      }
    }
    const uint32_t my_mp = (my_len + NP - 1) / NP * NP;
    const uint32_t mp_tile = (uint32_t)wave_max_i32((int)my_mp);
    const uint32_t nwords = staged_words<NP>(mp_tile);
    if (mp_tile == 0) continue;  // a tile of skipped reads (length 0)
    int t1s = -1, t1f = -1, t2s = -1, t2f = -1;
    const uint32_t f0 = (uint32_t)((uint64_t)chunk * a.nfe / a.nchunks);
    const uint32_t f1 = (uint32_t)((uint64_t)(chunk + 1) * a.nfe / a.nchunks);
    // candidate mode: one read per tile, fragments from its sorted list
    const int32_t* clist =
        a.cand ? a.cand + (uint64_t)__builtin_amdgcn_readfirstlane(my_read) * a.K : nullptr;
    // exclusion pass: this lane's read keeps fragments f with f + 1 - e > 2
    // (unsigned), i.e. every f but e - 1, e and e + 1
    const uint32_t ex = (a.excl && lane < rcount) ? (uint32_t)a.excl[my_read] : 0x80000000u;
    // the tile's read codes, both strands, into LDS (N-padded to cw words)
    __syncthreads();
    for (uint32_t idx = lane; idx < rcount * 2 * a.cw; idx += 64) {
      const uint32_t r = idx / (2 * a.cw), rem = idx - r * 2 * a.cw;
      const uint32_t s = rem / a.cw, wd = rem - s * a.cw;
      const uint32_t rid = a.order[rbase + r];
      if constexpr (BANK) {
        // code bytes 16c, four positions per word (two LDS words per code word)
        const uint32_t nw = wd >> 1;
        const uint32_t v =
            nw < a.cwg ? a.sel4[((uint64_t)rid * 2 + s) * a.cwg + nw] : 0x44444444u;
        const uint32_t h = (wd & 1) ? v >> 16 : v & 0xFFFFu;
        lcodes[idx] = ((h & 0xFu) << 4) | ((h & 0xF0u) << 8) | ((h & 0xF00u) << 12) |
                      ((h & 0xF000u) << 16);
      } else {
        lcodes[idx] = wd < a.cwg ? a.sel4[((uint64_t)rid * 2 + s) * a.cwg + wd] : 0x44444444u;
      }
    }
    if constexpr (QS) {
      // position-score pairs of the scanned positions, two per word; strand
      // 1 reads the read's pairs backwards
      for (uint32_t idx = lane; idx < rcount * 2 * a.cq; idx += 64) {
        const uint32_t r = idx / (2 * a.cq), rem = idx - r * 2 * a.cq;
        const uint32_t s = rem / a.cq, wd = rem - s * a.cq;
        const uint32_t rid = a.order[rbase + r];
        const uint32_t mfull = a.lens[rid];
        const uint16_t* qr = a.qsc + (uint64_t)rid * a.mp_max;
        uint32_t v = 0;
#pragma unroll
        for (uint32_t h = 0; h < 2; h++) {
          const uint32_t kk = a.step * (2 * wd + h);  // position in the strand
          if (kk < mfull) v |= (uint32_t)qr[s ? mfull - 1 - kk : kk] << (16 * h);
        }
        lqs[idx] = v;
      }
    }
    for (uint32_t fi = f0; fi < f1; fi++) {
      const uint32_t f = clist ? (uint32_t)clist[fi] : fi;
      int fv = -1;  // lane r: value of fragment f for read r
      // A segment holds the S window offsets seg*S .. seg*S+S-1.  With step 1
      // the pair of x (x < HALF) is (seg*S + x, seg*S + HALF + x); with step 2
      // (every other read base scored) it is (seg*S + 2x, seg*S + 2x + 1), the
      // two parities side by side.  Window word w holds the genome at
      // base + step*w and at HALF (step 1) or 1 (step 2) further, so one Kadane
      // step advances the window by one LDS word either way.
      for (uint32_t seg = 0; seg < a.nseg; seg++) {
        const uint64_t base = (uint64_t)f * a.F + (uint64_t)seg * S;
        const uint32_t hi_off = a.step == 1 ? HALF : 1u;
        __syncthreads();  // previous segment's readers are done with LDS
        for (uint32_t wd = lane; wd < nwords; wd += 64) {
          const uint64_t P = base + (uint64_t)a.step * wd;
          const uint32_t c0 = genome_code(a.g2, a.nmask, a.Lpad, P);
          const uint32_t c1 = genome_code(a.g2, a.nmask, a.Lpad, P + hi_off);
          lds[phys<NP>(wd)] = sel16(c0) | (sel16(c1) << 16);
        }
        __syncthreads();
        // window offsets left in the fragment from the segment start, and the
        // pairs whose low / high offset is one of them
        const int left = (int)a.F - (int)(seg * S);
        const bool partial_seg = left < (int)S;
        const int left_lo = a.step == 1 ? left : (left + 1) / 2;
        const int left_hi = a.step == 1 ? left - (int)HALF : left / 2;
        const int lo_cnt = min(max(left_lo - (int)(lane * NP), 0), NP);
        const int hi_cnt = min(max(left_hi - (int)(lane * NP), 0), NP);
        for (uint32_t r = 0; r < rcount; r++) {
          const uint32_t m = __builtin_amdgcn_readlane(my_len, r);
          if (m == 0) continue;
          uint32_t bm = 0x80008000u;
          for (uint32_t s = 0; s < a.nstrands; s++) {
            s16x2 B[NP];
            if constexpr (BANK) {
              uint64_t xp = a.xpool, dp = a.dpool;
              uint32_t x2 = xx;
              if constexpr (QB) {
                // the read's pair: match in the low byte, mismatch in the high
                const uint32_t pr = __builtin_amdgcn_readlane(my_pair, r);
                xp = mismatch_pool(pr >> 8);
                dp = (pr ^ (pr >> 8)) & 0xFFu;
                x2 = (uint32_t)(uint16_t)(int16_t)(int8_t)(pr >> 8) * 0x10001u;
              }
              kadane_pairs_bank(lds, lane, lcodes + (r * 2 + s) * a.cw, m, xp, dp, x2);
              if (!partial_seg) {
                bm = bank_fold(bm);
                continue;
              }
              bank_extract(B);
            } else {
              kadane_pairs<NP, QS, WIDE>(lds, lane, lcodes + (r * 2 + s) * a.cw,
                                         lqs + (r * 2 + s) * a.cq, m, a.xpool, a.dpool, B);
            }
            if (partial_seg) {
#pragma unroll
              for (int j = 0; j < NP; j++) {
                uint32_t b = __builtin_bit_cast(uint32_t, B[j]);
                if (j >= lo_cnt) b = (b & 0xFFFF0000u) | 0x8000u;
                if (j >= hi_cnt) b = (b & 0x0000FFFFu) | 0x80000000u;
                B[j] = __builtin_bit_cast(s16x2, b);
              }
            }
            s16x2 mx = __builtin_bit_cast(s16x2, bm);
#pragma unroll
            for (int j = 0; j < NP; j++) mx = __builtin_elementwise_max(mx, B[j]);
            bm = __builtin_bit_cast(uint32_t, mx);
          }
          const int lv = max((int)(short)(bm & 0xFFFFu), (int)(short)(bm >> 16));
          const int v = wave_max_i32(lv) + 32768;
          if (lane == r) fv = max(fv, v);
        }
      }
      // fragments arrive in increasing id order: strict '>' keeps the
      // smallest id among equal values
      if (lane < rcount && fv >= 0 && f + 1u - ex > 2u) {
        if (fv > t1s) {
          t2s = t1s; t2f = t1f; t1s = fv; t1f = (int)f;
        } else if (fv > t2s) {
          t2s = fv; t2f = (int)f;
        }
      }
    }
    if (lane < rcount && mine)
      a.partial[(uint64_t)my_read * a.nchunks + chunk] = make_int4(t1s, t1f, t2s, t2f);
  }
}

template <int NP, bool QS, bool WIDE>
__global__ __launch_bounds__(64) void scan_kernel(ScanArgs a) {
  scan_body<NP, QS, WIDE, false>(a);
}

// NP = 16, plain scores, score bound <= 31744: the register-bank Kadane, with
// the compiler confined to v0..v63 so that v64..v255 hold the banks.
__global__ __launch_bounds__(64) __attribute__((amdgpu_num_vgpr(32))) void scan_kernel_bank(
    ScanArgs a) {
  scan_body<16, false, false, true>(a);
}

// The same kernel for the quality split's reads with one score pair.
__global__ __launch_bounds__(64) __attribute__((amdgpu_num_vgpr(32))) void scan_kernel_bank_qual(
    ScanArgs a) {
  scan_body<16, false, false, true, true>(a);
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, uint32_t n) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Counting sort of the reads by length, longest first (invalid reads, length
// 0, last).  Ties are placed in atomic order: the order only shapes the read
// tiles, never a result.
__global__ void len_hist_kernel(const uint32_t* __restrict__ lens, uint32_t n,
                                uint32_t* __restrict__ hist) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t L = i < n ? lens[i] : 0xFFFFFFFFu;
  // one atomic per distinct length in the wave
  uint64_t todo = __ballot(i < n);
  while (todo) {
    const uint32_t lead = (uint32_t)__builtin_ctzll(todo);
    const uint32_t Ll = __shfl(L, lead, 64);
    const uint64_t same = __ballot(L == Ll) & todo;
    if ((threadIdx.x & 63) == lead) atomicAdd(&hist[Ll], (uint32_t)__builtin_popcountll(same));
    todo &= ~same;
  }
}

// hist[L] -> first output position of length L in descending-length order.
// One block of 1024 threads; nb = number of bins (max length + 1).
__global__ __launch_bounds__(1024) void len_starts_kernel(uint32_t* __restrict__ hist,
                                                          uint32_t nb) {
  __shared__ uint32_t part[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (nb + 1023) / 1024;
  // thread t owns bins (descending length) [t*per, (t+1)*per)
  uint32_t sum = 0;
  for (uint32_t k = t * per; k < min(nb, (t + 1) * per); k++) sum += hist[nb - 1 - k];
  part[t] = sum;
  __syncthreads();
  for (uint32_t o = 1; o < 1024; o <<= 1) {
    uint32_t v = t >= o ? part[t - o] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;  // exclusive prefix
  for (uint32_t k = t * per; k < min(nb, (t + 1) * per); k++) {
    const uint32_t L = nb - 1 - k;
    const uint32_t c = hist[L];
    hist[L] = run;
    run += c;
  }
}

__global__ void len_scatter_kernel(const uint32_t* __restrict__ lens, uint32_t n,
                                   uint32_t* __restrict__ starts, uint32_t* __restrict__ order) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t L = i < n ? lens[i] : 0xFFFFFFFFu;
  uint64_t todo = __ballot(i < n);
  while (todo) {
    const uint32_t lead = (uint32_t)__builtin_ctzll(todo);
    const uint32_t Ll = __shfl(L, lead, 64);
    const uint64_t same = __ballot(L == Ll) & todo;
    uint32_t base = 0;
    if (lane == lead) base = atomicAdd(&starts[Ll], (uint32_t)__builtin_popcountll(same));
    base = __shfl(base, lead, 64);
    if ((same >> lane) & 1ull) {
      const uint32_t rank = (uint32_t)__builtin_popcountll(same & ((1ull << lane) - 1ull));
      order[base + rank] = i;
    }
    todo &= ~same;
  }
}

// (score desc, fragment asc) order of candidates; negative fragment = none.
__device__ inline bool better(int s, int f, int bs, int bf) {
  if (f < 0) return false;
  if (bf < 0) return true;
  return s > bs || (s == bs && f < bf);
}

// Combine the per-chunk top-2 of every read.
__global__ void merge_kernel(const int4* __restrict__ partial, uint32_t nchunks,
                             const uint32_t* __restrict__ lens, uint32_t n,
                             maxss_top2* __restrict__ out) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  maxss_top2 r;
  for (int k = 0; k < 6; k++) r._pad[k] = 0;
  if (lens[i] == 0) {
    r.frag[0] = MAXSS_READ_INVALID; r.frag[1] = -1;
    r.score[0] = r.score[1] = -1;
    r.offset[0] = r.offset[1] = -1;
    r.strand[0] = r.strand[1] = -1;
    out[i] = r;
    return;
  }
  int s1 = -1, f1 = -1, s2 = -1, f2 = -1;
  for (uint32_t c = 0; c < nchunks; c++) {
    int4 p = partial[(uint64_t)i * nchunks + c];
    int cs[2] = {p.x, p.z}, cf[2] = {p.y, p.w};
    for (int t = 0; t < 2; t++) {
      if (better(cs[t], cf[t], s1, f1)) {
        s2 = s1; f2 = f1; s1 = cs[t]; f1 = cf[t];
      } else if (better(cs[t], cf[t], s2, f2)) {
        s2 = cs[t]; f2 = cf[t];
      }
    }
  }
  r.frag[0] = f1; r.score[0] = s1;
  r.frag[1] = f2; r.score[1] = f2 >= 0 ? s2 : -1;
  r.offset[0] = r.offset[1] = -1;
  r.strand[0] = r.strand[1] = -1;
  out[i] = r;
}

// Reads whose second fragment is a neighbour of the best one are scanned
// again with the best and its two neighbours left out (lens2 = their length,
// excl = the best fragment); every other read is skipped (lens2 = 0).
__global__ void excl_select_kernel(const maxss_top2* __restrict__ top,
                                   const uint32_t* __restrict__ lens, uint32_t n,
                                   uint32_t* __restrict__ lens2, int32_t* __restrict__ excl) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int f1 = top[i].frag[0], f2 = top[i].frag[1];
  const bool again = lens[i] > 0 && f1 >= 0 && f2 >= 0 && (f2 == f1 - 1 || f2 == f1 + 1);
  lens2[i] = again ? lens[i] : 0u;
  excl[i] = f1;
}

// The second fragment of a re-scanned read becomes the best fragment of its
// exclusion pass (none when every fragment was left out).
__global__ void excl_combine_kernel(const maxss_top2* __restrict__ again,
                                    const uint32_t* __restrict__ lens2, uint32_t n,
                                    maxss_top2* __restrict__ top) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || lens2[i] == 0) return;
  const maxss_top2 b = again[i];
  const bool has = b.frag[0] >= 0;
  top[i].frag[1] = has ? b.frag[0] : -1;
  top[i].score[1] = has ? b.score[0] : -1;
  top[i].offset[1] = has ? b.offset[0] : -1;
  top[i].strand[1] = has ? b.strand[0] : (int8_t)-1;
}

// Exact re-scan of one winning fragment of one read (int32, one offset per
// thread and strand) to find its representative window: the smallest strand,
// then the smallest offset, among the windows reaching the fragment's value.
// With STEP 2 only read positions 0, 2, 4, ... of each strand are scored;
// QS scores with the reads' position-specific pairs.
template <uint32_t STEP, bool QS>
__global__ __launch_bounds__(256) void rescan_kernel(
    const uint8_t* __restrict__ gcodes, uint32_t F, const uint8_t* __restrict__ rcodes,
    const uint32_t* __restrict__ lens, uint32_t mstride, int M, int X, uint32_t nstrands,
    const uint16_t* __restrict__ qsc, uint32_t n, maxss_top2* __restrict__ out) {
  extern __shared__ uint8_t sh[];
  const uint32_t i = blockIdx.x, which = blockIdx.y;
  const uint32_t m = lens[i];
  const int f = out[i].frag[which];
  if (m == 0 || f < 0) return;
  uint8_t* lg = sh;                    // F + m - 1 genome codes
  uint8_t* lq = sh + F + mstride;      // 2*m read codes: forward, reverse complement
  // quality mode: 2*m position-score pairs in the same two orientations
  uint16_t* lp = (uint16_t*)(sh + ((F + 3 * mstride + 3) & ~3u));
  const uint64_t gb = (uint64_t)f * F;
  for (uint32_t t = threadIdx.x; t < F + m - 1; t += blockDim.x) lg[t] = gcodes[gb + t];
  const uint8_t* rc = rcodes + (uint64_t)i * mstride;
  for (uint32_t k = threadIdx.x; k < m; k += blockDim.x) {
    uint8_t c = rc[k];
    lq[k] = c;
    lq[m + (m - 1 - k)] = c == kN ? kN : (uint8_t)(3 - c);
    if constexpr (QS) {
      const uint16_t v = qsc[(uint64_t)i * mstride + k];
      lp[k] = v;
      lp[m + (m - 1 - k)] = v;
    }
  }
  __syncthreads();
  // The fragment's value is known (the merge wrote it): windows are taken
  // in (strand, offset) order, a block-wide chunk at a time, and the scan
  // stops after the first chunk in which some window reaches the value (the
  // smallest such window lies there, every later one is larger).
  const int target = out[i].score[which];
  uint64_t best = 0;
  bool done = false;
  for (uint32_t s = 0; s < nstrands && !done; s++) {
    const uint8_t* q = lq + s * m;
    for (uint32_t o0 = 0; o0 < F && !done; o0 += blockDim.x) {
      const uint32_t o = o0 + threadIdx.x;
      int H = 0, B = -1;
      if (o < F) {
        B = 0;
        for (uint32_t k = 0; k < m; k += STEP) {
          const uint8_t g = lg[o + k], c = q[k];
          if constexpr (QS) {
            const uint16_t v = lp[s * m + k];
            H += (g == c && c != kN) ? (int)(int8_t)(v & 0xFFu) : (int)(int8_t)(v >> 8);
          } else {
            H += (g == c && c != kN) ? M : X;
          }
          H = max(H, 0);
          B = max(B, H);
        }
        const uint64_t key = ((uint64_t)(uint32_t)B << 32) | (0xFFFFFFFFu - (s * F + o));
        best = key > best ? key : best;
      }
      done = __syncthreads_or(B == target) != 0;
    }
  }
  // block max of the 64-bit keys
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t x = __shfl_xor(best, o, 64);
    best = x > best ? x : best;
  }
  __shared__ uint64_t wbest[4];
  if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 1; t < (int)(blockDim.x >> 6); t++) best = wbest[t] > best ? wbest[t] : best;
    const uint32_t code = 0xFFFFFFFFu - (uint32_t)(best & 0xFFFFFFFFu);
    out[i].strand[which] = (int8_t)(code / F);
    out[i].offset[which] = (int32_t)(code % F);
  }
}

struct Tiles {
  int NP;
  bool qs;                 // quality mode (position-specific scores)
  bool wide;               // scores may pass 31744: per-step max for B
  bool qb;                 // the register-bank launch of the quality split
  uint32_t R, ntiles, nchunks, nseg, grid;
  uint32_t win_slots, cw, cq;
  size_t lds;
};

// The scan kernel instance of (NP, quality mode, wide scores).
template <bool QS, bool WIDE>
static const void* scan_fn_np(int NP) {
  if (NP == 8) return (const void*)scan_kernel<8, QS, WIDE>;
  if (NP == 16) {
    if constexpr (!QS && !WIDE) return (const void*)scan_kernel_bank;
    else return (const void*)scan_kernel<16, QS, WIDE>;
  }
  return (const void*)scan_kernel<32, QS, WIDE>;
}

static const void* scan_fn(int NP, bool qs, bool wide, bool qb = false) {
  if (qb) return (const void*)scan_kernel_bank_qual;
  if (qs) return wide ? scan_fn_np<true, true>(NP) : scan_fn_np<true, false>(NP);
  return wide ? scan_fn_np<false, true>(NP) : scan_fn_np<false, false>(NP);
}

template <int NP, bool QS, bool WIDE>
static void launch_np(const ScanArgs& a, uint32_t grid, size_t lds, hipStream_t st) {
  if constexpr (NP == 16 && !QS && !WIDE) scan_kernel_bank<<<grid, 64, lds, st>>>(a);
  else scan_kernel<NP, QS, WIDE><<<grid, 64, lds, st>>>(a);
}

template <bool QS, bool WIDE>
static void launch_qw(int NP, const ScanArgs& a, uint32_t grid, size_t lds, hipStream_t st) {
  if (NP == 8) launch_np<8, QS, WIDE>(a, grid, lds, st);
  else if (NP == 16) launch_np<16, QS, WIDE>(a, grid, lds, st);
  else launch_np<32, QS, WIDE>(a, grid, lds, st);
}

static maxss_status launch_scan(const Tiles& t, const ScanArgs& a, hipStream_t st) {
  if (t.lds > 65536) {
    maxss_status s = check_hip(hipFuncSetAttribute(scan_fn(t.NP, t.qs, t.wide, t.qb),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)t.lds),
                               "hipFuncSetAttribute(scan_kernel)");
    if (s) return s;
  }
  if (t.qb) {
    scan_kernel_bank_qual<<<t.grid, 64, t.lds, st>>>(a);
  } else if (t.qs) {
    if (t.wide) launch_qw<true, true>(t.NP, a, t.grid, t.lds, st);
    else launch_qw<true, false>(t.NP, a, t.grid, t.lds, st);
  } else {
    if (t.wide) launch_qw<false, true>(t.NP, a, t.grid, t.lds, st);
    else launch_qw<false, false>(t.NP, a, t.grid, t.lds, st);
  }
  return check_hip(hipGetLastError(), "scan_kernel");
}

// Resident scan waves per CU for (kernel instance, LDS bytes), queried once
// per shape and cached, so that a step being captured into a graph makes no
// runtime query.
static int occupancy_for(int NP, bool qs, bool wide, size_t lds, bool qb = false) {
  static std::mutex mu;
  static std::map<std::pair<int, size_t>, int> cache;
  std::lock_guard<std::mutex> g(mu);
  const int key = NP * 8 + (qb ? 4 : 0) + (qs ? 2 : 0) + (wide ? 1 : 0);
  auto it = cache.find({key, lds});
  if (it != cache.end()) return it->second;
  int blocks = 0;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, scan_fn(NP, qs, wide, qb), 64, lds);
  if (e != hipSuccess || blocks < 1) blocks = 1;
  cache[{key, lds}] = blocks;
  return blocks;
}

// Largest score a window can reach (every scored base a match).
static uint64_t score_bound(const Index* ix) {
  const uint64_t scale = qual_mode(ix) ? ix->p.qual_scale : 1u;
  return (uint64_t)ix->p.max_read_len * (uint64_t)(int64_t)ix->p.match * scale;
}

// Scores up to this bound keep the biased values (0x8000 + h) at or below
// 0xFC00, binary16 -infinity, where their minimum3 order is that of h.
static constexpr uint64_t kNarrowScoreMax = 31744;

// Per-wave LDS budget of the scan: the genome window plus the tile's codes.
static constexpr size_t kScanLdsBudget = 40 * 1024;

static int np_for(const Index* ix, const TileOverride* force) {
  const uint32_t F = ix->F;
  if (force && (force->NP == 8 || force->NP == 16 || force->NP == 32)) return force->NP;
  // scores within the narrow bound: NP = 16 runs the register-bank kernel
  // (in quality mode for the reads whose positions share one score pair)
  if (F % 2048 == 0 && score_bound(ix) <= kNarrowScoreMax) return 16;
  if (F % 4096 == 0) return 32;
  if (F % 2048 == 0) return 16;
  return 8;
}

// Tile shape: the widest wave segment (128*NP offsets) that divides F, read
// tiles of R reads (bounded by the LDS budget) and a fragment-chunk count
// that fills whole rounds of the resident waves.  partial_cap (0 = none)
// bounds reads x chunks, the size of the per-chunk top-2 buffer.
// Most reads per tile (a power of two up to 32) whose LDS fits the per-wave
// budget of kernel (NP, qs, wide, qb): at most kScanLdsBudget, and no more
// than lets every wave that the kernel's registers allow stay resident on a
// CU.
static uint32_t rmax_for(const Index* ix, const Tiles& t, size_t win_bytes, size_t per_read) {
  size_t budget = kScanLdsBudget;
  const int reg_waves = occupancy_for(t.NP, t.qs, t.wide, 0, t.qb);
  if (ix->lds_per_cu && reg_waves > 0 && ix->lds_per_cu / (size_t)reg_waves < budget)
    budget = ix->lds_per_cu / (size_t)reg_waves;
  uint32_t rmax = 32;
  while (rmax > 1 && win_bytes + rmax * per_read > budget) rmax /= 2;
  if (win_bytes + rmax * per_read > 64 * 1024 && rmax > 1) rmax = 1;
  return rmax;
}

// In quality mode with NP = 16 and narrow scores the scan is split in two
// launches (scan_core): the shape chosen here is the register-bank launch's
// (qb), and split_second() derives the position-specific launch's.
static Tiles choose_tiles(const Index* ix, uint32_t n, uint32_t mstride,
                          const TileOverride* force, uint64_t partial_cap) {
  if (!force) force = &ix->tune;
  Tiles t{};
  t.NP = np_for(ix, force);
  const uint32_t S = 128u * t.NP;
  t.nseg = (ix->F + S - 1) / S;
  t.win_slots = win_slots_for(t.NP, mstride);
  t.cw = mstride / 8 + (uint32_t)t.NP / 8 + 1;
  t.qs = qual_mode(ix);
  t.wide = score_bound(ix) > kNarrowScoreMax;
  if (t.qs && t.NP == 16 && !t.wide) {
    t.qs = false;
    t.qb = true;
  }
  if (t.NP == 16 && !t.qs && !t.wide) t.cw *= 2;  // register banks: code bytes
  t.cq = t.qs ? (mstride / scan_step(ix) + 1) / 2 + 1 : 0u;
  const size_t win_bytes = (size_t)t.win_slots * 4u;
  const size_t per_read = (size_t)2 * (t.cw + t.cq) * 4u;
  const uint32_t rmax = rmax_for(ix, t, win_bytes, per_read);
  t.R = force->R ? (force->R < rmax ? force->R : rmax) : rmax;
  t.lds = win_bytes + t.R * per_read;
  const uint32_t resident =
      (uint32_t)ix->num_cu * (uint32_t)occupancy_for(t.NP, t.qs, t.wide, t.lds, t.qb);
  if (!force->R)
    while (t.R > 4 && (uint64_t)((n + t.R - 1) / t.R) * ix->NF < 4ull * resident) t.R /= 2;
  t.lds = win_bytes + t.R * per_read;
  t.ntiles = (n + t.R - 1) / t.R;
  // Chunk count: the fragments are cut into nchunks balanced chunks, so all
  // items of a tile cost the same and a uniform read mix runs in rounds of
  // `resident` waves.  Pick the count whose item total best fills whole
  // rounds (at least `rounds` rounds when the work allows it; fewer chunks
  // on ties).
  const uint32_t rounds = force->rounds ? force->rounds : 8;
  const uint64_t min_items = (uint64_t)rounds * resident;
  uint64_t c_lo64 = (min_items + t.ntiles - 1) / t.ntiles;
  if (c_lo64 < 1) c_lo64 = 1;
  if (c_lo64 > ix->NF) c_lo64 = ix->NF;
  uint32_t c_lo = (uint32_t)c_lo64;
  uint32_t c_hi = c_lo * 4 < ix->NF ? c_lo * 4 : ix->NF;
  if (partial_cap) {
    const uint64_t cmax = partial_cap / (n ? n : 1);
    if (cmax < 1) c_hi = 1;
    else if (c_hi > cmax) c_hi = (uint32_t)cmax;
    if (c_lo > c_hi) c_lo = c_hi;
  }
  uint32_t best_c = c_lo;
  double best_eff = -1.0;
  for (uint32_t c = c_lo; c <= c_hi; c++) {
    const uint64_t items = (uint64_t)t.ntiles * c;
    const uint64_t nround = (items + resident - 1) / resident;
    const double eff = (double)items / ((double)nround * resident);
    if (eff > best_eff + 1e-3) {
      best_eff = eff;
      best_c = c;
    }
  }
  t.nchunks = best_c;
  const uint64_t total = (uint64_t)t.ntiles * t.nchunks;
  t.grid = (uint32_t)(total < resident ? total : resident);
  if (t.grid < 1) t.grid = 1;
  return t;
}

// The position-specific launch of the quality split, from the register-bank
// launch's shape tb: the same fragment chunks (both write one record per read
// and chunk), its own codes, position-score pairs and reads per tile (its
// LDS budget is smaller); one read per tile in candidate mode.
static Tiles split_second(const Index* ix, const Tiles& tb, uint32_t n, uint32_t mstride,
                          const TileOverride* force, bool one_read) {
  if (!force) force = &ix->tune;
  Tiles t = tb;
  t.qb = false;
  t.qs = true;
  t.cw = tb.cw / 2;
  t.cq = (mstride / scan_step(ix) + 1) / 2 + 1;
  const size_t win_bytes = (size_t)t.win_slots * 4u;
  const size_t per_read = (size_t)2 * (t.cw + t.cq) * 4u;
  const uint32_t rmax = rmax_for(ix, t, win_bytes, per_read);
  t.R = one_read ? 1u : (force->R ? (force->R < rmax ? force->R : rmax) : rmax);
  t.lds = win_bytes + t.R * per_read;
  t.ntiles = one_read ? n : (n + t.R - 1) / t.R;
  const uint32_t resident =
      (uint32_t)ix->num_cu * (uint32_t)occupancy_for(t.NP, t.qs, t.wide, t.lds);
  const uint64_t total = (uint64_t)t.ntiles * t.nchunks;
  t.grid = (uint32_t)(total < resident ? total : resident);
  if (t.grid < 1) t.grid = 1;
  return t;
}

uint64_t scan_partial_entries(const Index* ix, uint32_t n, const TileOverride* force) {
  const Tiles t = choose_tiles(ix, n, read_stride(ix), force, 0);
  return (uint64_t)n * t.nchunks;
}

maxss_status alloc_scan_work(const Index* ix, uint32_t n, uint64_t partial_cap, bool stream_ordered,
                             hipStream_t st, ScanWork* w) {
  maxss_status s;
  const uint32_t nb = ix->p.max_read_len + 1;
  w->partial_cap = partial_cap;
  if (stream_ordered) {
    if ((s = alloc_encoded(ix, n, st, &w->er))) return s;
    if ((s = check_hip(dev_malloc_async((void**)&w->order, sizeof(uint32_t) * n, st), "alloc order")) ||
        (s = check_hip(dev_malloc_async((void**)&w->hist, sizeof(uint32_t) * nb, st), "alloc hist")) ||
        (s = check_hip(dev_malloc_async((void**)&w->ctr, sizeof(uint32_t), st), "alloc counter")) ||
        (s = check_hip(dev_malloc_async((void**)&w->partial, sizeof(int4) * partial_cap, st),
                       "alloc partial")))
      return s;
    if ((ix->p.flags & MAXSS_EXCLUDE_ADJACENT) &&
        ((s = check_hip(dev_malloc_async((void**)&w->excl, sizeof(int32_t) * n, st), "alloc excl")) ||
         (s = check_hip(dev_malloc_async((void**)&w->lens2, sizeof(uint32_t) * n, st),
                        "alloc lens2")) ||
         (s = check_hip(dev_malloc_async((void**)&w->again, sizeof(maxss_top2) * n, st),
                        "alloc again"))))
      return s;
    return MAXSS_OK;
  }
  w->er.mstride = read_stride(ix);
  const uint64_t nw = (uint64_t)n * 2 * (w->er.mstride / 8) + 64;
  if ((s = check_hip(dev_malloc((void**)&w->er.sel4, sizeof(uint32_t) * nw), "alloc read codes")) ||
      (s = check_hip(dev_malloc((void**)&w->er.codes, (uint64_t)n * w->er.mstride + 64),
                     "alloc read bases")) ||
      (s = check_hip(dev_malloc((void**)&w->er.lens, sizeof(uint32_t) * ((uint64_t)n + 1)),
                     "alloc lens")) ||
      (s = check_hip(dev_malloc((void**)&w->order, sizeof(uint32_t) * n), "alloc order")) ||
      (s = check_hip(dev_malloc((void**)&w->hist, sizeof(uint32_t) * nb), "alloc hist")) ||
      (s = check_hip(dev_malloc((void**)&w->ctr, sizeof(uint32_t)), "alloc counter")) ||
      (s = check_hip(dev_malloc((void**)&w->partial, sizeof(int4) * partial_cap), "alloc partial")))
    return s;
  if (qual_mode(ix) &&
      (s = check_hip(dev_malloc((void**)&w->er.qsc, sizeof(uint16_t) * ((uint64_t)n * w->er.mstride + 64)),
                     "alloc position scores")))
    return s;
  if ((ix->p.flags & MAXSS_EXCLUDE_ADJACENT) &&
      ((s = check_hip(dev_malloc((void**)&w->excl, sizeof(int32_t) * n), "alloc excl")) ||
       (s = check_hip(dev_malloc((void**)&w->lens2, sizeof(uint32_t) * n), "alloc lens2")) ||
       (s = check_hip(dev_malloc((void**)&w->again, sizeof(maxss_top2) * n), "alloc again"))))
    return s;
  return MAXSS_OK;
}

void release_scan_work(ScanWork* w, bool stream_ordered, hipStream_t st) {
  void* ps[] = {w->order, w->hist, w->ctr, w->partial, w->excl, w->lens2, w->again};
  for (void* p : ps) {
    if (!p) continue;
    if (stream_ordered) (void)hipFreeAsync(p, st);
    else (void)hipFree(p);
  }
  if (stream_ordered) {
    release_encoded(&w->er, st);
  } else {
    if (w->er.sel4) (void)hipFree(w->er.sel4);
    if (w->er.codes) (void)hipFree(w->er.codes);
    if (w->er.lens) (void)hipFree(w->er.lens);
    if (w->er.qsc) (void)hipFree(w->er.qsc);
    w->er = EncodedReads{};
  }
  w->order = w->hist = w->ctr = nullptr;
  w->partial = nullptr;
  w->excl = nullptr;
  w->lens2 = nullptr;
  w->again = nullptr;
}

// Sort (by `lens`), scan, merge and re-scan for n encoded reads.  Reads with
// lens[i] == 0 are skipped and get an invalid record.  cand != NULL: scan
// only each read's Kc first candidates (K per read, ascending), one read per
// tile.
static maxss_status scan_core(const Index* ix, const EncodedReads& er, const uint32_t* lens,
                              uint32_t n, maxss_top2* dout, const ScanWork& w,
                              const TileOverride* force, const int32_t* cand, uint32_t K,
                              uint32_t Kc, hipStream_t st, const int32_t* excl = nullptr) {
  maxss_status s;
  const uint32_t nstrands = (ix->p.flags & MAXSS_ONE_STRAND) ? 1u : 2u;
  const uint32_t mstride = er.mstride;
  Tiles t = choose_tiles(ix, n, mstride, force, w.partial_cap);
  if (cand) {
    // one read per tile; enough candidate chunks to fill the resident waves
    t.R = 1;
    const size_t per_read = (size_t)2 * (t.cw + t.cq) * 4u;
    t.lds = (size_t)t.win_slots * 4u + per_read;
    const uint32_t resident =
      (uint32_t)ix->num_cu * (uint32_t)occupancy_for(t.NP, t.qs, t.wide, t.lds, t.qb);
    t.ntiles = n;
    uint64_t want = (8ull * resident + n - 1) / n;
    if (want < 1) want = 1;
    if (want > Kc) want = Kc;
    if (want * n > w.partial_cap) want = w.partial_cap / n ? w.partial_cap / n : 1;
    t.nchunks = (uint32_t)want;
    const uint64_t total = (uint64_t)t.ntiles * t.nchunks;
    t.grid = (uint32_t)(total < resident ? total : resident);
  }
  if ((uint64_t)n * t.nchunks > w.partial_cap)
    return fail(MAXSS_ESTATE, "partial buffer too small (%llu < %llu)",
                (unsigned long long)w.partial_cap, (unsigned long long)n * t.nchunks);
  const uint32_t M8 = (uint32_t)ix->p.match & 0xFFu, X8 = (uint32_t)ix->p.mismatch & 0xFFu;
  const uint64_t xpool = mismatch_pool(X8);
  // reads ordered by length, longest first
  const uint32_t nb = ix->p.max_read_len + 1;
  fill_u32_kernel<<<(nb + 255) / 256, 256, 0, st>>>(w.hist, 0u, nb);
  len_hist_kernel<<<(n + 255) / 256, 256, 0, st>>>(lens, n, w.hist);
  len_starts_kernel<<<1, 1024, 0, st>>>(w.hist, nb);
  len_scatter_kernel<<<(n + 255) / 256, 256, 0, st>>>(lens, n, w.hist, w.order);
  fill_u32_kernel<<<1, 64, 0, st>>>(w.ctr, 0u, 1u);
  if ((s = check_hip(hipGetLastError(), "length sort"))) return s;
  ScanArgs a{};
  a.g2 = ix->g2; a.nmask = ix->nmask; a.Lpad = ix->Lpad;
  a.F = ix->F; a.NF = ix->NF; a.nseg = t.nseg;
  a.sel4 = er.sel4; a.cwg = mstride / 8; a.cw = t.cw; a.win_slots = t.win_slots;
  a.xpool = xpool; a.dpool = (uint64_t)(M8 ^ X8);
  a.lens = lens; a.order = w.order; a.n = n;
  a.R = t.R; a.ntiles = t.ntiles; a.nchunks = t.nchunks;
  a.total_work = t.ntiles * t.nchunks; a.work_ctr = w.ctr; a.partial = w.partial;
  a.nstrands = nstrands; a.mp_max = mstride;
  a.cand = cand; a.K = K; a.nfe = cand ? Kc : ix->NF;
  a.step = scan_step(ix);
  const bool quality = t.qs || t.qb;
  a.qsc = quality ? er.qsc : nullptr;
  a.cq = t.cq;
  a.excl = excl;
  if (quality && !er.qsc) return fail(MAXSS_ESTATE, "quality mode without position scores");
  {
    ProfScope prof("scan", st);
    if (t.qb) {
      // Quality split.  A read whose scored positions all carry one (match,
      // mismatch) pair scores exactly as plain scores with that pair, so the
      // register-bank kernel takes those reads (each with its own pair) and
      // the position-specific kernel the others.  Both launches take the
      // reads in the same order and cut the fragments into the same chunks,
      // and each writes only its own reads' chunk records, so the merge
      // sees one complete set.
      a.qsplit = 1;
      if ((s = launch_scan(t, a, st))) return s;
      const Tiles tq = split_second(ix, t, n, mstride, force, cand != nullptr);
      ScanArgs aq = a;
      aq.cw = tq.cw;
      aq.cq = tq.cq;
      aq.R = tq.R;
      aq.ntiles = tq.ntiles;
      aq.total_work = tq.ntiles * tq.nchunks;
      aq.qsplit = 2;
      fill_u32_kernel<<<1, 64, 0, st>>>(w.ctr, 0u, 1u);
      s = launch_scan(tq, aq, st);
    } else {
      s = launch_scan(t, a, st);
    }
  }
  if (s) return s;
  {
    ProfScope prof("merge", st);
    merge_kernel<<<(n + 255) / 256, 256, 0, st>>>(w.partial, t.nchunks, lens, n, dout);
  }
  if ((s = check_hip(hipGetLastError(), "merge_kernel"))) return s;
  // genome window + both read orientations (+ their position scores)
  const size_t rl = (size_t)ix->F + 3 * (size_t)mstride + 16 + (a.qsc ? 4 * (size_t)mstride + 16 : 0);
  const bool fast = scan_step(ix) == 2, qs = a.qsc != nullptr;
  const void* fn = fast ? (qs ? (const void*)rescan_kernel<2, true> : (const void*)rescan_kernel<2, false>)
                        : (qs ? (const void*)rescan_kernel<1, true> : (const void*)rescan_kernel<1, false>);
  if (rl > 65536 &&
      (s = check_hip(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rl),
                     "hipFuncSetAttribute(rescan_kernel)")))
    return s;
  {
    ProfScope prof("rescan", st);
    const dim3 g(n, 2);
    if (fast && qs)
      rescan_kernel<2, true><<<g, 256, rl, st>>>(ix->codes, ix->F, er.codes, lens, mstride,
                                                 ix->p.match, ix->p.mismatch, nstrands, a.qsc, n,
                                                 dout);
    else if (fast)
      rescan_kernel<2, false><<<g, 256, rl, st>>>(ix->codes, ix->F, er.codes, lens, mstride,
                                                  ix->p.match, ix->p.mismatch, nstrands, a.qsc, n,
                                                  dout);
    else if (qs)
      rescan_kernel<1, true><<<g, 256, rl, st>>>(ix->codes, ix->F, er.codes, lens, mstride,
                                                 ix->p.match, ix->p.mismatch, nstrands, a.qsc, n,
                                                 dout);
    else
      rescan_kernel<1, false><<<g, 256, rl, st>>>(ix->codes, ix->F, er.codes, lens, mstride,
                                                  ix->p.match, ix->p.mismatch, nstrands, a.qsc, n,
                                                  dout);
  }
  return check_hip(hipGetLastError(), "rescan_kernel");
}

// MAXSS_EXCLUDE_ADJACENT: after the full scan (or the candidate scan, cand
// != NULL), the reads whose second fragment neighbours the best are scanned
// again (over the same fragments) with the best fragment and its neighbours
// left out, and that pass's best becomes their second.
static maxss_status exclusion_pass(const Index* ix, const EncodedReads& er, const uint32_t* lens,
                                   uint32_t n, maxss_top2* dout, const ScanWork& w,
                                   const TileOverride* force, hipStream_t st,
                                   const int32_t* cand = nullptr, uint32_t K = 0,
                                   uint32_t Kc = 0) {
  if (!(ix->p.flags & MAXSS_EXCLUDE_ADJACENT)) return MAXSS_OK;
  if (!w.excl || !w.lens2 || !w.again)
    return fail(MAXSS_ESTATE, "scan scratch lacks the exclusion buffers");
  maxss_status s;
  excl_select_kernel<<<(n + 255) / 256, 256, 0, st>>>(dout, lens, n, w.lens2, w.excl);
  if ((s = check_hip(hipGetLastError(), "excl_select_kernel"))) return s;
  // Few reads take this pass (their count stays on the device), so tiles of
  // one read and as many fragment chunks as the partial buffer holds spread
  // them over the resident waves; the offset pairs per lane stay as set.
  const TileOverride* base = force ? force : &ix->tune;
  const TileOverride one{base->NP, 1u, 1024u};
  if ((s = scan_core(ix, er, w.lens2, n, w.again, w, cand ? nullptr : &one, cand, K, Kc, st,
                     w.excl)))
    return s;
  excl_combine_kernel<<<(n + 255) / 256, 256, 0, st>>>(w.again, w.lens2, n, dout);
  return check_hip(hipGetLastError(), "excl_combine_kernel");
}

maxss_status scan_pipeline(const Index* ix, const DeviceReads& r, maxss_top2* dout,
                           const ScanWork& w, const TileOverride* force, hipStream_t st) {
  const uint32_t n = r.n;
  if (n == 0) return MAXSS_OK;
  if (qual_mode(ix) && !r.qual)
    return fail(MAXSS_ESTATE, "quality-mode scan of reads without qualities");
  maxss_status s;
  if ((s = encode_reads_into(ix, r, st, w.er))) return s;
  if ((s = scan_core(ix, w.er, w.er.lens, n, dout, w, force, nullptr, 0, 0, st))) return s;
  return exclusion_pass(ix, w.er, w.er.lens, n, dout, w, force, st);
}

maxss_status scan_pipeline_lens(const Index* ix, const EncodedReads& er, const uint32_t* lens,
                                uint32_t n, maxss_top2* dout, const ScanWork& w, hipStream_t st) {
  if (n == 0) return MAXSS_OK;
  maxss_status s;
  if ((s = scan_core(ix, er, lens, n, dout, w, nullptr, nullptr, 0, 0, st))) return s;
  return exclusion_pass(ix, er, lens, n, dout, w, nullptr, st);
}

maxss_status candidate_scan(const Index* ix, const EncodedReads& er, const uint32_t* lens,
                            uint32_t n, const int32_t* cand, uint32_t K, uint32_t Kc,
                            maxss_top2* dout, const ScanWork& w, hipStream_t st) {
  if (n == 0) return MAXSS_OK;
  maxss_status s;
  if ((s = scan_core(ix, er, lens, n, dout, w, nullptr, cand, K, Kc, st))) return s;
  return exclusion_pass(ix, er, lens, n, dout, w, nullptr, st, cand, K, Kc);
}

}  // namespace maxss

using namespace maxss;

extern "C" maxss_status maxss_scan_reads(const maxss_index* index, const maxss_reads* reads,
                                         maxss_top2* out, void* stream) {
  clear_error();
  const Index* ix = reinterpret_cast<const Index*>(index);
  if (!ix || !reads || !out) return fail(MAXSS_EINVAL, "NULL argument");
  if (reads->n == 0) return MAXSS_OK;
  if (!reads->seq || !reads->offsets) return fail(MAXSS_EINVAL, "NULL reads");
  hipStream_t st = (hipStream_t)stream;
  maxss_status s;
  if ((s = require_quals(ix, reads))) return s;
  if (!reads->on_device && (s = validate_host_reads(ix, reads))) return s;
  int cur = 0;
  if ((s = check_hip(hipGetDevice(&cur), "hipGetDevice"))) return s;
  if (cur != ix->device) return fail(MAXSS_ESTATE, "index lives on device %d, current is %d",
                                     ix->device, cur);
  DeviceReads dr;
  ScanWork w;
  maxss_top2* dout = nullptr;
  const uint32_t n = reads->n;
  do {
    if ((s = stage_reads(reads, st, &dr))) break;
    if ((s = alloc_scan_work(ix, n, scan_partial_entries(ix, n, nullptr), true, st, &w))) break;
    if (reads->on_device) {
      dout = out;
    } else if ((s = check_hip(dev_malloc_async((void**)&dout, sizeof(maxss_top2) * n, st),
                              "alloc out"))) {
      break;
    }
    if ((s = scan_pipeline(ix, dr, dout, w, nullptr, st))) break;
    if (!reads->on_device &&
        (s = check_hip(hipMemcpyAsync(out, dout, sizeof(maxss_top2) * n, hipMemcpyDeviceToHost, st),
                       "copy results")))
      break;
  } while (0);
  if (dout && dout != out) (void)hipFreeAsync(dout, st);
  release_scan_work(&w, true, st);
  release_reads(&dr, st);
  if (!reads->on_device && s == MAXSS_OK) s = check_hip(hipStreamSynchronize(st), "sync");
  return s;
}

extern "C" maxss_status maxss_scan_kernel_info(const maxss_index* index, int32_t* np,
                                               int32_t* kind) {
  clear_error();
  const Index* ix = reinterpret_cast<const Index*>(index);
  if (!ix) return fail(MAXSS_EINVAL, "NULL index");
  const int NP = np_for(ix, &ix->tune);
  const bool wide = score_bound(ix) > kNarrowScoreMax;
  if (np) *np = NP;
  if (kind)
    *kind = wide ? MAXSS_KERNEL_STEP_MAX
                 : (NP == 16 ? MAXSS_KERNEL_REGISTER_BANK : MAXSS_KERNEL_TWO_STEP);
  return MAXSS_OK;
}
