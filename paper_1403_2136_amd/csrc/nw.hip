// Second phase: Needleman-Wunsch of every read against the region of its best
// fragment (Methods, "Second phase of MaxSSmap"), HIP, gfx950.
//
// One 256-thread block per read (persistent over reads).  The DP is filled row
// by row (one row per read base); each thread owns a contiguous run of region
// columns.  Within a row the diagonal and up moves are independent per
// column; the left move is a max-plus prefix: with g = -gap >= 0,
//   D[i][j] = max_{j' <= j} (T[j'] - (j - j') g),  T = max(diag, up),
// so V[j] = D[i][j] + j g is the running maximum of T[j] + j g.  Each thread
// scans its run, a block-wide exclusive max-scan carries the prefix across
// threads, and the boundary column D[i][0] = i*gap seeds the carry.
// Every cell's move (diagonal, up = 'I', left = 'D', in that priority on ties)
// is stored in 2 bits in a per-block global scratch slab; one thread traces
// back and writes the run-length CIGAR.
#include <limits.h>
#include <stdint.h>

#include <algorithm>

#include "internal.h"

namespace maxss {

static constexpr int kNwThreads = 256;

struct NwArgs {
  const uint8_t* gcodes;  // genome codes
  uint64_t G;
  uint32_t F, NF;
  const uint8_t* rcodes;  // forward read codes [n][mstride]
  const uint16_t* qsc;    // quality mode: [n][mstride] (match | mismatch << 8), else null
  const uint32_t* lens;
  uint32_t mstride;
  const maxss_top2* top;
  uint32_t n;
  uint32_t pad;
  int M, X, gap;
  int global_mode;
  uint32_t cw;            // columns per thread (multiple of 4)
  uint32_t rowbytes;      // bytes of move codes per DP row
  uint8_t* slab;          // [gridDim.x][m_max][rowbytes]
  uint32_t m_max;
  uint32_t lds_moves;     // two-pass kernel: one-strip windows keep their moves in LDS
  maxss_aln* out;
  char* cigar;
  uint64_t cigar_stride;
};

__device__ inline long long block_excl_max(long long v, long long* sh) {
  // inclusive max-scan within the wave, then across the 4 waves
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    long long y = __shfl_up(x, o, 64);
    if (lane >= o) x = x > y ? x : y;
  }
  if (lane == 63) sh[wv] = x;
  long long ex = __shfl_up(x, 1, 64);
  __syncthreads();
  long long carry = LLONG_MIN;
  for (int w = 0; w < wv; w++) carry = sh[w] > carry ? sh[w] : carry;
  __syncthreads();
  if (lane > 0) carry = ex > carry ? ex : carry;
  return carry;  // max over all threads before this one (LLONG_MIN if none)
}

__global__ __launch_bounds__(kNwThreads) void nw_kernel(NwArgs a) {
  extern __shared__ uint8_t sh[];
  __shared__ long long scan_sh[4];
  __shared__ long long red_v[4];
  __shared__ int red_j[4];
  const uint32_t tid = threadIdx.x;
  const uint32_t ncols_max = kNwThreads * a.cw;
  int* rowA = (int*)sh;                            // ncols_max + 1
  int* rowB = rowA + ncols_max + 1;                // ncols_max + 1
  uint8_t* lq = (uint8_t*)(rowB + ncols_max + 1);  // m_max
  uint8_t* lg = lq + a.m_max;                      // ncols_max
  char* ops = (char*)(lg + ncols_max);             // m_max + ncols_max
  uint8_t* slab = a.slab + (uint64_t)blockIdx.x * a.m_max * a.rowbytes;
  const long long g = -(long long)a.gap;
  for (uint32_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const uint32_t m = a.lens[i];
    const int f = a.top[i].frag[0];
    maxss_aln* o = a.out + i;
    char* cg = a.cigar + (uint64_t)i * a.cigar_stride;
    const int strand = a.top[i].strand[0];
    if (m == 0 || f < 0 || (uint32_t)f >= a.NF || (strand != 0 && strand != 1)) {
      if (tid == 0) {
        o->score = 0; o->strand = -1; o->flags = MAXSS_ALN_SKIPPED;
        o->_pad[0] = o->_pad[1] = 0;
        o->ref_begin = o->ref_end = -1; o->cigar_len = 0; o->_pad2 = 0;
        cg[0] = 0;
      }
      continue;
    }
    const long long start = (long long)f * a.F;
    long long ra = start - (long long)a.pad;
    if (ra < 0) ra = 0;
    long long rb = start + (long long)a.F + (long long)m - 1 + (long long)a.pad;
    if (rb > (long long)a.G) rb = (long long)a.G;
    const uint32_t ncols = (uint32_t)(rb - ra);
    __syncthreads();  // the previous read's traceback is done with LDS
    const uint8_t* rc = a.rcodes + (uint64_t)i * a.mstride;
    for (uint32_t k = tid; k < m; k += kNwThreads) {
      uint8_t c = strand ? rc[m - 1 - k] : rc[k];
      if (strand) c = c == kN ? kN : (uint8_t)(3 - c);
      lq[k] = c;
    }
    for (uint32_t j = tid; j < ncols; j += kNwThreads) lg[j] = a.gcodes[ra + j];
    for (uint32_t j = tid; j <= ncols; j += kNwThreads)
      rowA[j] = a.global_mode ? (int)j * a.gap : 0;
    __syncthreads();
    int* prev = rowA;
    int* cur = rowB;
    const uint32_t j0 = 1 + tid * a.cw;  // first column of this thread
    for (uint32_t r = 1; r <= m; r++) {
      const uint8_t q = lq[r - 1];
      // this row's match / mismatch: the read base's own pair in quality mode
      // (strand 1 rows run over the read backwards)
      int Mr = a.M, Xr = a.X;
      if (a.qsc) {
        const uint16_t v = a.qsc[(uint64_t)i * a.mstride + (strand ? m - r : r - 1)];
        Mr = (int)(int8_t)(v & 0xFFu);
        Xr = (int)(int8_t)(v >> 8);
      }
      const int col0 = (int)r * a.gap;
      // pass 1: this thread's running max of T[j] + j*g
      long long run = LLONG_MIN;
      for (uint32_t t = 0; t < a.cw; t++) {
        const uint32_t j = j0 + t;
        if (j > ncols) break;
        const uint8_t gc = lg[j - 1];
        const int d = prev[j - 1] + ((q == gc && q != kN) ? Mr : Xr);
        const int u = prev[j] + a.gap;
        const long long tv = (long long)(d > u ? d : u) + (long long)j * g;
        run = tv > run ? tv : run;
      }
      long long carry = block_excl_max(run, scan_sh);
      const long long c0 = (long long)col0;  // column 0: V[0] = D[r][0]
      carry = carry > c0 ? carry : c0;
      // pass 2: D values and moves
      uint8_t* mrow = slab + (uint64_t)(r - 1) * a.rowbytes + tid * (a.cw / 4);
      uint32_t packed = 0;
      for (uint32_t t = 0; t < a.cw; t++) {
        const uint32_t j = j0 + t;
        uint32_t mv = 0;
        if (j <= ncols) {
          const uint8_t gc = lg[j - 1];
          const int d = prev[j - 1] + ((q == gc && q != kN) ? Mr : Xr);
          const int u = prev[j] + a.gap;
          const long long tv = (long long)(d > u ? d : u) + (long long)j * g;
          carry = tv > carry ? tv : carry;
          const int D = (int)(carry - (long long)j * g);
          cur[j] = D;
          mv = (D == d) ? 0u : (D == u ? 1u : 2u);
        }
        packed |= mv << (2 * (t & 3));
        if ((t & 3) == 3) {
          mrow[t >> 2] = (uint8_t)packed;
          packed = 0;
        }
      }
      if (tid == 0) cur[0] = col0;
      __syncthreads();
      int* tmp = prev; prev = cur; cur = tmp;
    }
    // end column: the whole region (global) or the best, smallest column
    long long bestv = LLONG_MIN;
    int bestj = 0;
    if (a.global_mode) {
      bestv = prev[ncols];
      bestj = (int)ncols;
    } else {
      for (uint32_t j = tid; j <= ncols; j += kNwThreads) {
        const long long v = prev[j];
        if (v > bestv) { bestv = v; bestj = (int)j; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        long long v2 = __shfl_xor(bestv, off, 64);
        int j2 = __shfl_xor(bestj, off, 64);
        if (v2 > bestv || (v2 == bestv && j2 < bestj)) { bestv = v2; bestj = j2; }
      }
      if ((tid & 63) == 0) { red_v[tid >> 6] = bestv; red_j[tid >> 6] = bestj; }
      __syncthreads();
      if (tid == 0) {
        for (int w = 1; w < kNwThreads / 64; w++)
          if (red_v[w] > bestv || (red_v[w] == bestv && red_j[w] < bestj)) {
            bestv = red_v[w]; bestj = red_j[w];
          }
      }
    }
    __threadfence_block();
    if (tid == 0) {
      // traceback (moves of row r live in slab row r-1), ops collected backwards
      uint32_t len = 0;
      int ii = (int)m, jj = bestj;
      while (ii > 0 || (a.global_mode && jj > 0)) {
        uint32_t mv;
        if (ii == 0) mv = 2;
        else if (jj == 0) mv = 1;
        else {
          const uint32_t t = (uint32_t)(jj - 1);
          const uint8_t byte = slab[(uint64_t)(ii - 1) * a.rowbytes + (t >> 2)];
          mv = (byte >> (2 * (t & 3))) & 3u;
        }
        if (mv == 0) {
          const uint8_t q = lq[ii - 1], gc = lg[jj - 1];
          ops[len++] = (q == gc && q != kN) ? '=' : 'X';
          ii--; jj--;
        } else if (mv == 1) {
          ops[len++] = 'I';
          ii--;
        } else {
          ops[len++] = 'D';
          jj--;
        }
      }
      // run-length encode forwards
      uint64_t w = 0;
      bool trunc = false;
      for (int p = (int)len - 1; p >= 0;) {
        const char op = ops[p];
        int q2 = p;
        while (q2 >= 0 && ops[q2] == op) q2--;
        uint32_t run = (uint32_t)(p - q2);
        char dig[12];
        int nd = 0;
        do { dig[nd++] = (char)('0' + run % 10); run /= 10; } while (run);
        if (w + (uint64_t)nd + 1 + 1 > a.cigar_stride) { trunc = true; break; }
        while (nd) cg[w++] = dig[--nd];
        cg[w++] = op;
        p = q2;
      }
      cg[w] = 0;
      o->score = (int)bestv;
      o->strand = (int8_t)strand;
      o->flags = trunc ? MAXSS_ALN_TRUNCATED : 0;
      o->_pad[0] = o->_pad[1] = 0;
      o->ref_begin = ra + jj;
      o->ref_end = ra + bestj;
      o->cigar_len = (uint32_t)w;
      o->_pad2 = 0;
    }
  }
}

// The same DP with one wave per read (persistent over reads, 64 threads per
// workgroup, no barrier inside a row).  Lane l owns region columns
// [1 + l*CW, 1 + (l+1)*CW): their previous-row values and genome codes live in
// registers, the left neighbour's last value comes by a lane shuffle, and the
// max-plus prefix across lanes is a 64-lane shuffle scan.  Moves go to the
// slab in the block kernel's layout (column j's two bits at byte (j-1)/4 of
// the row), and lane 0 traces back as there.  Values are int32: the host uses
// this kernel only when every DP value provably fits.
template <int CW>
__global__ __launch_bounds__(64) void nw_wave_kernel(NwArgs a) {
  extern __shared__ uint8_t shw[];
  uint8_t* lq = shw;                                        // m_max read codes
  char* ops = (char*)(shw + ((a.m_max + 15u) & ~15u));     // m_max + 64*CW ops
  const int lane = (int)threadIdx.x;
  uint8_t* slab = a.slab + (uint64_t)blockIdx.x * a.m_max * a.rowbytes;
  const int g = -a.gap;  // >= 0
  for (uint32_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const uint32_t m = a.lens[i];
    const int f = a.top[i].frag[0];
    maxss_aln* o = a.out + i;
    char* cg = a.cigar + (uint64_t)i * a.cigar_stride;
    const int strand = a.top[i].strand[0];
    if (m == 0 || f < 0 || (uint32_t)f >= a.NF || (strand != 0 && strand != 1)) {
      if (lane == 0) {
        o->score = 0; o->strand = -1; o->flags = MAXSS_ALN_SKIPPED;
        o->_pad[0] = o->_pad[1] = 0;
        o->ref_begin = o->ref_end = -1; o->cigar_len = 0; o->_pad2 = 0;
        cg[0] = 0;
      }
      continue;
    }
    const long long start = (long long)f * a.F;
    long long ra = start - (long long)a.pad;
    if (ra < 0) ra = 0;
    long long rb = start + (long long)a.F + (long long)m - 1 + (long long)a.pad;
    if (rb > (long long)a.G) rb = (long long)a.G;
    const int ncols = (int)(rb - ra);
    __syncthreads();  // the previous read's traceback is done with LDS
    const uint8_t* rc = a.rcodes + (uint64_t)i * a.mstride;
    for (uint32_t k = lane; k < m; k += 64) {
      uint8_t c = strand ? rc[m - 1 - k] : rc[k];
      if (strand) c = c == kN ? kN : (uint8_t)(3 - c);
      lq[k] = c;
    }
    const int j0 = 1 + lane * CW;
    uint32_t gv[CW / 4];
#pragma unroll
    for (int w = 0; w < CW / 4; w++) {
      uint32_t v = 0;
#pragma unroll
      for (int b = 0; b < 4; b++) {
        const int j = j0 + 4 * w + b;
        const uint32_t c = j <= ncols ? a.gcodes[ra + j - 1] : (uint32_t)kN;
        v |= c << (8 * b);
      }
      gv[w] = v;
    }
    int prev[CW];
#pragma unroll
    for (int t = 0; t < CW; t++) prev[t] = a.global_mode ? (j0 + t) * a.gap : 0;
    __syncthreads();  // lq written
    for (uint32_t r = 1; r <= m; r++) {
      const uint32_t q = lq[r - 1];
      int Mr = a.M, Xr = a.X;
      if (a.qsc) {
        const uint16_t v = a.qsc[(uint64_t)i * a.mstride + (strand ? m - r : r - 1)];
        Mr = (int)(int8_t)(v & 0xFFu);
        Xr = (int)(int8_t)(v >> 8);
      }
      // Row-invariant per-column values (unpacked genome codes, j*g) are
      // recomputed every row instead of being held in registers across rows:
      // the copies below look row-dependent to the compiler.
      int gg = g;
      asm volatile("" : "+s"(gg));
      uint32_t gw[CW / 4];
#pragma unroll
      for (int w = 0; w < CW / 4; w++) {
        gw[w] = gv[w];
        asm volatile("" : "+v"(gw[w]));
      }
      // D[r-1][j0-1]: the left lane's last column, or column 0
      int pl = __shfl_up(prev[CW - 1], 1, 64);
      if (lane == 0) pl = (int)(r - 1) * a.gap;
      // pass 1: T[j] = max(diag, up) replaces the previous row in place, with
      // one bit per column for "diagonal wins the tie", and this lane's
      // running max of T[j] + j*g
      int run = INT_MIN, old = pl;
      uint32_t dwin[(CW + 31) / 32];
#pragma unroll
      for (int w = 0; w < (CW + 31) / 32; w++) dwin[w] = 0;
#pragma unroll
      for (int t = 0; t < CW; t++) {
        const uint32_t gc = (gw[t >> 2] >> (8 * (t & 3))) & 0xFFu;
        const int d = old + ((q == gc && q != kN) ? Mr : Xr);
        const int u = prev[t] + a.gap;
        old = prev[t];
        prev[t] = max(d, u);
        dwin[t >> 5] |= (d >= u ? 1u : 0u) << (t & 31);
        run = max(run, prev[t] + (j0 + t) * gg);
      }
      // exclusive max-scan across lanes; column 0 (D[r][0] = r*gap) seeds it
      int x = run;
#pragma unroll
      for (int of = 1; of < 64; of <<= 1) {
        const int y = __shfl_up(x, of, 64);
        if (lane >= of) x = max(x, y);
      }
      int carry = __shfl_up(x, 1, 64);
      if (lane == 0) carry = INT_MIN;
      carry = max(carry, (int)r * a.gap);
      // pass 2: D = max(T, left chain); the move is diagonal, then up, then
      // left on ties: T's own winner when D == T, else left
      uint8_t* mrow = slab + (uint64_t)(r - 1) * a.rowbytes + lane * (CW / 4);
      uint32_t packed = 0;
#pragma unroll
      for (int t = 0; t < CW; t++) {
        const int jg = (j0 + t) * gg;
        const int T = prev[t];
        carry = max(carry, T + jg);
        const int D = carry - jg;
        const uint32_t mv = (D == T) ? (((dwin[t >> 5] >> (t & 31)) & 1u) ? 0u : 1u) : 2u;
        prev[t] = D;
        packed |= mv << (2 * (t & 3));
        if ((t & 3) == 3) {
          mrow[t >> 2] = (uint8_t)packed;
          packed = 0;
        }
      }
    }
    // end column: the whole region (global) or the best, smallest column
    int bestv, bestj;
    if (a.global_mode) {
      const int owner = (ncols - 1) / CW, tt = (ncols - 1) - owner * CW;
      int v = 0;
#pragma unroll
      for (int t = 0; t < CW; t++)
        if (t == tt) v = prev[t];
      bestv = __shfl(v, owner, 64);
      bestj = ncols;
    } else {
      int bv = INT_MIN, bj = INT_MAX;
      if (lane == 0) { bv = (int)m * a.gap; bj = 0; }
#pragma unroll
      for (int t = 0; t < CW; t++)
        if (j0 + t <= ncols && prev[t] > bv) { bv = prev[t]; bj = j0 + t; }
#pragma unroll
      for (int of = 32; of > 0; of >>= 1) {
        const int v2 = __shfl_xor(bv, of, 64), j2 = __shfl_xor(bj, of, 64);
        if (v2 > bv || (v2 == bv && j2 < bj)) { bv = v2; bj = j2; }
      }
      bestv = bv;
      bestj = bj;
    }
    __threadfence_block();  // every lane's moves are visible to lane 0
    if (lane == 0) {
      uint32_t len = 0;
      int ii = (int)m, jj = bestj;
      while (ii > 0 || (a.global_mode && jj > 0)) {
        uint32_t mv;
        if (ii == 0) mv = 2;
        else if (jj == 0) mv = 1;
        else {
          const uint32_t t = (uint32_t)(jj - 1);
          const uint8_t byte = slab[(uint64_t)(ii - 1) * a.rowbytes + (t >> 2)];
          mv = (byte >> (2 * (t & 3))) & 3u;
        }
        if (mv == 0) {
          const uint8_t qc = lq[ii - 1], gc = a.gcodes[ra + jj - 1];
          ops[len++] = (qc == gc && qc != kN) ? '=' : 'X';
          ii--; jj--;
        } else if (mv == 1) {
          ops[len++] = 'I';
          ii--;
        } else {
          ops[len++] = 'D';
          jj--;
        }
      }
      uint64_t w = 0;
      bool trunc = false;
      for (int p = (int)len - 1; p >= 0;) {
        const char op = ops[p];
        int q2 = p;
        while (q2 >= 0 && ops[q2] == op) q2--;
        uint32_t run2 = (uint32_t)(p - q2);
        char dig[12];
        int nd = 0;
        do { dig[nd++] = (char)('0' + run2 % 10); run2 /= 10; } while (run2);
        if (w + (uint64_t)nd + 1 + 1 > a.cigar_stride) { trunc = true; break; }
        while (nd) cg[w++] = dig[--nd];
        cg[w++] = op;
        p = q2;
      }
      cg[w] = 0;
      o->score = bestv;
      o->strand = (int8_t)strand;
      o->flags = trunc ? MAXSS_ALN_TRUNCATED : 0;
      o->_pad[0] = o->_pad[1] = 0;
      o->ref_begin = ra + jj;
      o->ref_end = ra + bestj;
      o->cigar_len = (uint32_t)w;
      o->_pad2 = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// Fitting mode in two passes per read (one wave per read, persistent over
// reads), used when every DP value of the region fits in 16 bits (the host
// checks (max_read_len + CW + 2) * max(|M|, |X|, |gap|) <= 32767).
//
// Pass A scores the whole region without moves.  Lane l owns the region
// columns [j0, j0 + CW), j0 = 1 + l*CW, as CW/2 packed pairs: pair t holds
// columns j0 + t (low half) and j0 + CW/2 + t (high half), so the diagonal
// neighbour of pair t is pair t - 1 for both halves.  A row costs per pair
// one v_perm_b32 (both substitution scores from the row's score pool, as in
// the first phase), two packed adds and a packed max for T = max(diag, up),
// a packed add and max for the lane's running max of T + (j - j0) g, and,
// after the 64-lane prefix (DPP row shifts and broadcasts), a packed max
// and subtraction for D = max(T, left chain).  It ends with the best score S
// and its smallest end column.
//
// Pass B recomputes the DP, with moves, only over the window of columns
// (b, jend] with b = jend - m - kmax, where kmax = (sum over rows of the
// largest row score - S) / g bounds the number of genome gaps ('D') of any
// alignment scoring S, so every optimal alignment ending at jend starts at
// or after column b.  In the window the DP starts again from the boundary
// column b (D = i*gap, as column 0); every cell of an optimal alignment keeps
// its value, and a neighbour's value matches the whole-region DP wherever it
// could tie, so the diagonal > up > left choices, hence the traceback, are
// those of the whole-region DP.  The window runs in strips of 256 columns
// (4 per lane); the last column of a strip seeds the next through LDS.
// ---------------------------------------------------------------------------

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

__device__ inline uint32_t pk_add(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}
__device__ inline uint32_t pk_sub(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}
__device__ inline uint32_t pk_max(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(i16x2, a),
                                                                __builtin_bit_cast(i16x2, b)));
}
// a - b per half, saturated: its sign bit is set exactly when a < b
__device__ inline uint32_t pk_sub_sat(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(i16x2, a),
                                                                    __builtin_bit_cast(i16x2, b)));
}
__device__ inline uint32_t pk2(int lo, int hi) {
  return (uint32_t)(uint16_t)lo | ((uint32_t)(uint16_t)hi << 16);
}
__device__ inline int lo16(uint32_t v) { return (int)(short)(v & 0xFFFFu); }
__device__ inline int hi16(uint32_t v) { return (int)(short)(v >> 16); }

// v_perm_b32 selector half of a genome code: the pool byte of its score and
// the byte that sign-extends it (A 1/8, C 3/9, G 5/10, T 7/11; N takes the
// mismatch byte 0 and its sign byte 2).
__device__ inline uint32_t nw_sel16(uint32_t c) {
  return c >= kN ? 0x0200u : ((2u * c + 1u) | ((8u + c) << 8));
}

// Inclusive max-scan over the 64 lanes (DPP row shifts, then the row
// broadcasts of lanes 15 and 31); lanes with no source keep INT_MIN.
__device__ inline int wave_incl_max(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x111, 0xF, 0xF, false));  // row_shr:1
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x112, 0xF, 0xF, false));  // row_shr:2
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x114, 0xF, 0xF, false));  // row_shr:4
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x118, 0xF, 0xF, false));  // row_shr:8
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x142, 0xA, 0xF, false));  // row_bcast:15
  x = max(x, __builtin_amdgcn_update_dpp(INT_MIN, x, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return x;
}
// The value of the lane below (lane 0 gets `none`).
__device__ inline int wave_shr1(int x, int none) {
  return __builtin_amdgcn_update_dpp(none, x, 0x138, 0xF, 0xF, false);  // wave_shr:1
}

// Score pool of a row (read base q, row scores mr / xr): bytes
// [X, X, sign(X), X, 0, X, 0, X] with the byte of q's score flipped to M.
__device__ inline void row_pool(uint32_t q, int mr, int xr, uint32_t& lo, uint32_t& hi) {
  const uint32_t x8 = (uint32_t)xr & 0xFFu, m8 = (uint32_t)mr & 0xFFu;
  const uint32_t sx = xr < 0 ? 0xFFu : 0u;
  uint64_t p = (uint64_t)(x8 | (x8 << 8) | (sx << 16) | (x8 << 24)) |
               ((uint64_t)((x8 << 8) | (x8 << 24)) << 32);
  const uint32_t byte = q >= kN ? 4u : 2u * q + 1u;
  p ^= (uint64_t)(m8 ^ x8) << (8 * byte);
  lo = (uint32_t)p;
  hi = (uint32_t)(p >> 32);
}

static constexpr int kFitStripCw = 4;                  // window columns per lane in pass B
static constexpr int kFitStrip = 64 * kFitStripCw;    // window columns per strip

template <int CW>
__global__ __launch_bounds__(64) void nw_fit_kernel(NwArgs a) {
  constexpr int H = CW / 2;
  constexpr int HB = kFitStripCw / 2;
  extern __shared__ uint8_t shf[];
  const uint32_t mq = (a.m_max + 15u) & ~15u;
  uint8_t* lq = shf;                                            // read codes
  char* ops = (char*)(shf + mq);                                // traceback ops
  const uint32_t ops_bytes = (a.m_max + 64u * CW + 16u + 3u) & ~3u;
  int* lb0 = (int*)(shf + mq + ops_bytes);                      // strip boundaries
  int* lb1 = lb0 + (a.m_max + 1);
  // a one-strip window's moves, [m_max][64] bytes (row r-1, lane = byte)
  uint8_t* lmv = a.lds_moves ? (uint8_t*)(lb1 + (a.m_max + 1)) : nullptr;
  const int lane = (int)threadIdx.x;
  uint8_t* slab = a.slab + (uint64_t)blockIdx.x * a.m_max * a.rowbytes;
  const int g = -a.gap;  // >= 0
  const uint32_t gg = pk2(a.gap, a.gap);
  uint32_t jl[H];        // (j - j0) * g of each pair's columns
#pragma unroll
  for (int t = 0; t < H; t++) jl[t] = pk2(t * g, (t + H) * g);
  uint32_t jlb[HB];
#pragma unroll
  for (int t = 0; t < HB; t++) jlb[t] = pk2(t * g, (t + HB) * g);
  for (uint32_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    const uint32_t m = a.lens[i];
    const int f = a.top[i].frag[0];
    maxss_aln* o = a.out + i;
    char* cg = a.cigar + (uint64_t)i * a.cigar_stride;
    const int strand = a.top[i].strand[0];
    if (m == 0 || f < 0 || (uint32_t)f >= a.NF || (strand != 0 && strand != 1)) {
      if (lane == 0) {
        o->score = 0; o->strand = -1; o->flags = MAXSS_ALN_SKIPPED;
        o->_pad[0] = o->_pad[1] = 0;
        o->ref_begin = o->ref_end = -1; o->cigar_len = 0; o->_pad2 = 0;
        cg[0] = 0;
      }
      continue;
    }
    const long long start = (long long)f * a.F;
    long long ra = start - (long long)a.pad;
    if (ra < 0) ra = 0;
    long long rb = start + (long long)a.F + (long long)m - 1 + (long long)a.pad;
    if (rb > (long long)a.G) rb = (long long)a.G;
    const int ncols = (int)(rb - ra);
    __syncthreads();  // the previous read's traceback is done with LDS
    const uint8_t* rc = a.rcodes + (uint64_t)i * a.mstride;
    for (uint32_t k = lane; k < m; k += 64) {
      uint8_t c = strand ? rc[m - 1 - k] : rc[k];
      if (strand) c = c == kN ? kN : (uint8_t)(3 - c);
      lq[k] = c;
    }
    const uint16_t* qrow = a.qsc ? a.qsc + (uint64_t)i * a.mstride : nullptr;
    // ---- pass A: scores of the whole region
    const int j0 = 1 + lane * CW;
    uint32_t sel[H], D[H];
#pragma unroll
    for (int t = 0; t < H; t++) {
      const int jl0 = j0 + t, jh0 = j0 + H + t;
      const uint32_t cl = jl0 <= ncols ? a.gcodes[ra + jl0 - 1] : (uint32_t)kN;
      const uint32_t ch = jh0 <= ncols ? a.gcodes[ra + jh0 - 1] : (uint32_t)kN;
      sel[t] = nw_sel16(cl) | (nw_sel16(ch) << 16);
      D[t] = 0;  // row 0: D[0][j] = 0 (the alignment may start at any column)
    }
    __syncthreads();  // lq written
    int sum_u = 0;    // sum over rows of the largest score a read base can add
    for (uint32_t r = 1; r <= m; r++) {
      const uint32_t q = __builtin_amdgcn_readfirstlane(lq[r - 1]);
      int mr = a.M, xr = a.X;
      if (qrow) {
        const uint32_t v = __builtin_amdgcn_readfirstlane(qrow[strand ? m - r : r - 1]);
        mr = (int)(int8_t)(v & 0xFFu);
        xr = (int)(int8_t)(v >> 8);
      }
      sum_u += max(mr, max(xr, a.gap));
      uint32_t plo, phi;
      row_pool(q, mr, xr, plo, phi);
      // D[r-1] at the columns left of pair 0: j0 - 1 (the lane below's last
      // column, or column 0) and j0 + H - 1 (this lane's pair H-1, low half)
      const uint32_t last = D[H - 1];
      const int below = wave_shr1((int)last, 0);
      const int dl = lane == 0 ? (int)(r - 1) * a.gap : hi16((uint32_t)below);
      uint32_t old = pk2(dl, lo16(last));
      uint32_t run = 0x80008000u;
#pragma unroll
      for (int t = 0; t < H; t++) {
        const uint32_t cur = D[t];
        const uint32_t s = __builtin_amdgcn_perm(phi, plo, sel[t]);
        const uint32_t T = pk_max(pk_add(old, s), pk_add(cur, gg));
        const uint32_t TJ = pk_add(T, jl[t]);
        run = pk_max(run, TJ);
        D[t] = TJ;
        old = cur;
      }
      // left chain: V[j] = D[r][j] + j g is the running max of T[j] + j g,
      // seeded by column 0 (V[0] = r*gap)
      const int rl = lo16(run);
      const int x = wave_incl_max(max(rl, hi16(run)) + j0 * g);
      const int cin = max(wave_shr1(x, INT_MIN), (int)r * a.gap);
      const int clo = max(cin - j0 * g, -32768);
      uint32_t carry = pk2(clo, max(clo, rl));
#pragma unroll
      for (int t = 0; t < H; t++) {
        carry = pk_max(carry, D[t]);
        D[t] = pk_sub(carry, jl[t]);
      }
    }
    // best end column of the last row (smallest column on ties; column 0 is
    // D[m][0] = m*gap)
    int bv = INT_MIN, bj = INT_MAX;
    if (lane == 0) { bv = (int)m * a.gap; bj = 0; }
#pragma unroll
    for (int t = 0; t < H; t++)
      if (j0 + t <= ncols && lo16(D[t]) > bv) { bv = lo16(D[t]); bj = j0 + t; }
#pragma unroll
    for (int t = 0; t < H; t++)
      if (j0 + H + t <= ncols && hi16(D[t]) > bv) { bv = hi16(D[t]); bj = j0 + H + t; }
#pragma unroll
    for (int of = 32; of > 0; of >>= 1) {
      const int v2 = __shfl_xor(bv, of, 64), j2 = __shfl_xor(bj, of, 64);
      if (v2 > bv || (v2 == bv && j2 < bj)) { bv = v2; bj = j2; }
    }
    const int S = bv, jend = bj;
    // ---- pass B: the window (b, jend] with moves
    int b = 0;
    if (g > 0) {
      const long long kmax = ((long long)sum_u - S) / g;
      const long long lo = (long long)jend - (long long)m - kmax;
      b = lo > 0 ? (int)lo : 0;
    }
    const int W = jend - b;
    // the window fits one strip: its moves stay in LDS, byte lane of row r-1
    // holding columns 4 lane + 1 .. 4 lane + 4
    const bool in_lds = lmv != nullptr && W <= kFitStrip;
    int* lb = lb0;
    int* ln = lb1;
    for (uint32_t r = lane; r <= m; r += 64) lb[r] = (int)r * a.gap;
    if (lane == 0) ln[0] = 0;
    __syncthreads();
    for (int s0 = 0; s0 < W; s0 += kFitStrip) {
      const int jw0 = s0 + 1 + lane * kFitStripCw;  // window column of this lane's first column
      uint32_t selb[HB], Db[HB];
#pragma unroll
      for (int t = 0; t < HB; t++) {
        const int wl = jw0 + t, wh = jw0 + HB + t;
        const uint32_t cl = wl <= W ? a.gcodes[ra + b + wl - 1] : (uint32_t)kN;
        const uint32_t ch = wh <= W ? a.gcodes[ra + b + wh - 1] : (uint32_t)kN;
        selb[t] = nw_sel16(cl) | (nw_sel16(ch) << 16);
        Db[t] = 0;
      }
      const int off = jw0 - s0;  // (jw0 - strip boundary column)
      for (uint32_t r = 1; r <= m; r++) {
        const uint32_t q = __builtin_amdgcn_readfirstlane(lq[r - 1]);
        int mr = a.M, xr = a.X;
        if (qrow) {
          const uint32_t v = __builtin_amdgcn_readfirstlane(qrow[strand ? m - r : r - 1]);
          mr = (int)(int8_t)(v & 0xFFu);
          xr = (int)(int8_t)(v >> 8);
        }
        uint32_t plo, phi;
        row_pool(q, mr, xr, plo, phi);
        const uint32_t last = Db[HB - 1];
        const int below = wave_shr1((int)last, 0);
        const int dl = lane == 0 ? lb[r - 1] : hi16((uint32_t)below);
        uint32_t old = pk2(dl, lo16(last));
        uint32_t run = 0x80008000u;
        uint32_t upw[HB];
#pragma unroll
        for (int t = 0; t < HB; t++) {
          const uint32_t cur = Db[t];
          const uint32_t s = __builtin_amdgcn_perm(phi, plo, selb[t]);
          const uint32_t d = pk_add(old, s), u = pk_add(cur, gg);
          upw[t] = (pk_sub_sat(d, u) >> 15) & 0x00010001u;  // up wins T (d < u)
          const uint32_t TJ = pk_add(pk_max(d, u), jlb[t]);
          run = pk_max(run, TJ);
          Db[t] = TJ;
          old = cur;
        }
        const int rl = lo16(run);
        const int x = wave_incl_max(max(rl, hi16(run)) + off * g);
        const int cin = max(wave_shr1(x, INT_MIN), lb[r]);
        const int clo = max(cin - off * g, -32768);
        uint32_t carry = pk2(clo, max(clo, rl));
        uint32_t mv = 0;
#pragma unroll
        for (int t = 0; t < HB; t++) {
          // left wins when the chain so far exceeds T + (j - jw0) g
          const uint32_t L = (pk_sub_sat(Db[t], carry) >> 15) & 0x00010001u;
          carry = pk_max(carry, Db[t]);
          Db[t] = pk_sub(carry, jlb[t]);
          mv |= ((L << 1) | (upw[t] & ~L)) << (2 * t);  // 0 diagonal, 1 up (I), 2 left (D)
        }
        // columns jw0, jw0+1 in bits 0..3, jw0+2, jw0+3 in bits 16..19
        const uint8_t mb = (uint8_t)((mv & 0xFu) | ((mv >> 12) & 0xF0u));
        if (in_lds) lmv[(r - 1) * 64u + (uint32_t)lane] = mb;
        else slab[(uint64_t)(r - 1) * a.rowbytes + (uint32_t)(jw0 - 1) / 4u] = mb;
        if (lane == 63) ln[r] = hi16(Db[HB - 1]);  // the strip's last column
      }
      __syncthreads();  // ln complete; lb no longer read
      int* tmp = lb; lb = ln; ln = tmp;
      if (lane == 0) ln[0] = 0;
      __syncthreads();
    }
    __threadfence_block();  // every lane's moves are visible to lane 0
    if (lane == 0) {
      uint32_t len = 0;
      int ii = (int)m, jj = W;
      while (ii > 0) {
        uint32_t mv;
        if (jj == 0) mv = 1;
        else {
          const uint32_t t = (uint32_t)(jj - 1);
          const uint8_t byte = in_lds ? lmv[(uint32_t)(ii - 1) * 64u + (t >> 2)]
                                      : slab[(uint64_t)(ii - 1) * a.rowbytes + (t >> 2)];
          mv = (byte >> (2 * (t & 3))) & 3u;
        }
        if (mv == 0) {
          const uint8_t qc = lq[ii - 1], gc = a.gcodes[ra + b + jj - 1];
          ops[len++] = (qc == gc && qc != kN) ? '=' : 'X';
          ii--; jj--;
        } else if (mv == 1) {
          ops[len++] = 'I';
          ii--;
        } else {
          ops[len++] = 'D';
          jj--;
        }
      }
      uint64_t w = 0;
      bool trunc = false;
      for (int p = (int)len - 1; p >= 0;) {
        const char op = ops[p];
        int q2 = p;
        while (q2 >= 0 && ops[q2] == op) q2--;
        uint32_t run2 = (uint32_t)(p - q2);
        char dig[12];
        int nd = 0;
        do { dig[nd++] = (char)('0' + run2 % 10); run2 /= 10; } while (run2);
        if (w + (uint64_t)nd + 1 + 1 > a.cigar_stride) { trunc = true; break; }
        while (nd) cg[w++] = dig[--nd];
        cg[w++] = op;
        p = q2;
      }
      cg[w] = 0;
      o->score = S;
      o->strand = (int8_t)strand;
      o->flags = trunc ? MAXSS_ALN_TRUNCATED : 0;
      o->_pad[0] = o->_pad[1] = 0;
      o->ref_begin = ra + b + jj;
      o->ref_end = ra + jend;
      o->cigar_len = (uint32_t)w;
      o->_pad2 = 0;
    }
  }
}

// Columns per lane of the wave kernel's instantiations.
static constexpr int kWaveCw[] = {8, 16, 24, 32, 40, 48, 56, 64, 72, 80, 88, 96};

template <int CW>
static const void* wave_fn() {
  return (const void*)nw_wave_kernel<CW>;
}

static const void* wave_kernel_for(int cw) {
  switch (cw) {
    case 8: return wave_fn<8>();
    case 16: return wave_fn<16>();
    case 24: return wave_fn<24>();
    case 32: return wave_fn<32>();
    case 40: return wave_fn<40>();
    case 48: return wave_fn<48>();
    case 56: return wave_fn<56>();
    case 64: return wave_fn<64>();
    case 72: return wave_fn<72>();
    case 80: return wave_fn<80>();
    case 88: return wave_fn<88>();
    default: return wave_fn<96>();
  }
}

template <int CW>
static const void* fit_fn() {
  return (const void*)nw_fit_kernel<CW>;
}

static const void* fit_kernel_for(int cw) {
  switch (cw) {
    case 8: return fit_fn<8>();
    case 16: return fit_fn<16>();
    case 24: return fit_fn<24>();
    case 32: return fit_fn<32>();
    case 40: return fit_fn<40>();
    case 48: return fit_fn<48>();
    case 56: return fit_fn<56>();
    case 64: return fit_fn<64>();
    case 72: return fit_fn<72>();
    case 80: return fit_fn<80>();
    case 88: return fit_fn<88>();
    default: return fit_fn<96>();
  }
}

maxss_status nw_shape(const Index* ix, uint32_t n, uint32_t pad, NwShape* sh) {
  const uint32_t m_max = ix->p.max_read_len;
  const uint64_t ncols_need = (uint64_t)ix->F + m_max - 1 + 2ull * pad;
  // the wave kernel: 64 lanes of up to 96 columns, and every DP value (cell
  // scores and gaps along at most m_max + ncols moves, plus the j*g offset of
  // the prefix) within int32
  const int64_t qs = ix->p.qual_scale > 0 ? ix->p.qual_scale : 1;
  const int64_t step_max = std::max<int64_t>({(int64_t)ix->p.match * qs, -(int64_t)ix->p.mismatch * qs,
                                              -(int64_t)ix->p.gap * qs, 1});
  const uint64_t cw64 = (ncols_need + 63) / 64;
  sh->wave_cw = 0;
  if (cw64 <= 96 && (int64_t)(m_max + 2 * ncols_need + 64) * step_max < (1ll << 30)) {
    for (int c : kWaveCw)
      if ((uint64_t)c >= cw64) { sh->wave_cw = (uint32_t)c; break; }
  }
  // fitting mode whose every DP value fits in 16 bits: the two-pass kernel
  sh->fit = false;
  if (sh->wave_cw && !(ix->p.flags & MAXSS_NW_GLOBAL) &&
      (int64_t)(m_max + sh->wave_cw + 2) * step_max <= 32767)
    sh->fit = true;
  if (sh->wave_cw) {
    sh->cw = sh->wave_cw;
    sh->ncols_max = 64 * sh->wave_cw;
    sh->rowbytes = sh->ncols_max / 4;
    sh->lds = ((m_max + 15u) & ~15u) + m_max + sh->ncols_max + 16;
    const void* fn = sh->fit ? fit_kernel_for((int)sh->wave_cw) : wave_kernel_for((int)sh->wave_cw);
    sh->lds_moves = false;
    if (sh->fit) {
      sh->lds = ((m_max + 15u) & ~15u) + ((m_max + sh->ncols_max + 16u + 3u) & ~3u) +
                2 * ((size_t)m_max + 1) * 4;
      // room for a one-strip window's moves when it costs no resident waves
      const size_t with = sh->lds + 64 * (size_t)m_max;
      int occ0 = 0, occ1 = 0;
      if (with <= 65536 &&
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ0, fn, 64, sh->lds) == hipSuccess &&
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ1, fn, 64, with) == hipSuccess &&
          occ1 >= occ0 && occ1 > 0) {
        sh->lds = with;
        sh->lds_moves = true;
      }
    }
    if (sh->lds > 160 * 1024)
      return fail(MAXSS_EINVAL, "NW region too wide for LDS (%zu bytes)", sh->lds);
    maxss_status s;
    if (sh->lds > 65536 &&
        (s = check_hip(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)sh->lds),
                       "hipFuncSetAttribute(nw wave kernel)")))
      return s;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, 64, sh->lds) != hipSuccess || occ < 1)
      occ = 1;
    uint32_t grid = (uint32_t)ix->num_cu * (uint32_t)occ;
    if (n && grid > n) grid = n;
    sh->grid = grid ? grid : 1;
    return MAXSS_OK;
  }
  uint32_t cw = (uint32_t)((ncols_need + kNwThreads - 1) / kNwThreads);
  cw = (cw + 3) & ~3u;
  sh->cw = cw;
  sh->ncols_max = cw * kNwThreads;
  sh->rowbytes = sh->ncols_max / 4;
  sh->lds = (size_t)2 * (sh->ncols_max + 1) * 4 + m_max + sh->ncols_max + (m_max + sh->ncols_max) + 16;
  if (sh->lds > 160 * 1024)
    return fail(MAXSS_EINVAL, "NW region too wide for LDS (%zu bytes)", sh->lds);
  maxss_status s;
  if (sh->lds > 65536 &&
      (s = check_hip(hipFuncSetAttribute((const void*)nw_kernel,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh->lds),
                     "hipFuncSetAttribute(nw_kernel)")))
    return s;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, nw_kernel, kNwThreads, sh->lds) !=
          hipSuccess ||
      occ < 1)
    occ = 1;
  uint32_t grid = (uint32_t)ix->num_cu * (uint32_t)occ;
  if (n && grid > n) grid = n;
  sh->grid = grid ? grid : 1;
  return MAXSS_OK;
}

maxss_status nw_pipeline(const Index* ix, const EncodedReads& er, uint32_t n,
                         const maxss_top2* dtop, uint32_t pad, maxss_aln* dout, char* dcig,
                         uint64_t cigar_stride, uint8_t* slab, const NwShape& sh,
                         hipStream_t st) {
  if (n == 0) return MAXSS_OK;
  NwArgs a{};
  a.gcodes = ix->codes; a.G = ix->G; a.F = ix->F; a.NF = ix->NF;
  a.rcodes = er.codes; a.lens = er.lens; a.mstride = er.mstride;
  a.qsc = qual_mode(ix) ? er.qsc : nullptr;
  if (qual_mode(ix) && !er.qsc) return fail(MAXSS_ESTATE, "quality mode without position scores");
  a.top = dtop; a.n = n; a.pad = pad;
  a.M = ix->p.match; a.X = ix->p.mismatch;
  // in quality mode the gap is in the same 1/qual_scale units as the scores
  a.gap = qual_mode(ix) ? ix->p.gap * (int)ix->p.qual_scale : ix->p.gap;
  a.global_mode = (ix->p.flags & MAXSS_NW_GLOBAL) ? 1 : 0;
  a.cw = sh.cw; a.rowbytes = sh.rowbytes; a.slab = slab; a.m_max = ix->p.max_read_len;
  a.lds_moves = sh.lds_moves ? 1u : 0u;
  a.out = dout; a.cigar = dcig; a.cigar_stride = cigar_stride;
  const uint32_t grid = sh.grid < n ? sh.grid : n;
  if (sh.fit) {
    ProfScope prof("nw", st);
    switch (sh.wave_cw) {
      case 8: nw_fit_kernel<8><<<grid, 64, sh.lds, st>>>(a); break;
      case 16: nw_fit_kernel<16><<<grid, 64, sh.lds, st>>>(a); break;
      case 24: nw_fit_kernel<24><<<grid, 64, sh.lds, st>>>(a); break;
      case 32: nw_fit_kernel<32><<<grid, 64, sh.lds, st>>>(a); break;
      case 40: nw_fit_kernel<40><<<grid, 64, sh.lds, st>>>(a); break;
      case 48: nw_fit_kernel<48><<<grid, 64, sh.lds, st>>>(a); break;
      case 56: nw_fit_kernel<56><<<grid, 64, sh.lds, st>>>(a); break;
      case 64: nw_fit_kernel<64><<<grid, 64, sh.lds, st>>>(a); break;
      case 72: nw_fit_kernel<72><<<grid, 64, sh.lds, st>>>(a); break;
      case 80: nw_fit_kernel<80><<<grid, 64, sh.lds, st>>>(a); break;
      case 88: nw_fit_kernel<88><<<grid, 64, sh.lds, st>>>(a); break;
      default: nw_fit_kernel<96><<<grid, 64, sh.lds, st>>>(a); break;
    }
    return check_hip(hipGetLastError(), "nw_fit_kernel");
  }
  {
    ProfScope prof("nw", st);
    switch (sh.wave_cw) {
      case 0: nw_kernel<<<grid, kNwThreads, sh.lds, st>>>(a); break;
      case 8: nw_wave_kernel<8><<<grid, 64, sh.lds, st>>>(a); break;
      case 16: nw_wave_kernel<16><<<grid, 64, sh.lds, st>>>(a); break;
      case 24: nw_wave_kernel<24><<<grid, 64, sh.lds, st>>>(a); break;
      case 32: nw_wave_kernel<32><<<grid, 64, sh.lds, st>>>(a); break;
      case 40: nw_wave_kernel<40><<<grid, 64, sh.lds, st>>>(a); break;
      case 48: nw_wave_kernel<48><<<grid, 64, sh.lds, st>>>(a); break;
      case 56: nw_wave_kernel<56><<<grid, 64, sh.lds, st>>>(a); break;
      case 64: nw_wave_kernel<64><<<grid, 64, sh.lds, st>>>(a); break;
      case 72: nw_wave_kernel<72><<<grid, 64, sh.lds, st>>>(a); break;
      case 80: nw_wave_kernel<80><<<grid, 64, sh.lds, st>>>(a); break;
      case 88: nw_wave_kernel<88><<<grid, 64, sh.lds, st>>>(a); break;
      default: nw_wave_kernel<96><<<grid, 64, sh.lds, st>>>(a); break;
    }
  }
  return check_hip(hipGetLastError(), "nw_kernel");
}

}  // namespace maxss

using namespace maxss;

extern "C" maxss_status maxss_align_top(const maxss_index* index, const maxss_reads* reads,
                                        const maxss_top2* top, uint32_t pad, maxss_aln* out,
                                        char* cigar, uint64_t cigar_stride, void* stream) {
  clear_error();
  const Index* ix = reinterpret_cast<const Index*>(index);
  if (!ix || !reads || !top || !out || !cigar) return fail(MAXSS_EINVAL, "NULL argument");
  if (cigar_stride < 2) return fail(MAXSS_EINVAL, "cigar_stride must be >= 2");
  if (pad > (1u << 20)) return fail(MAXSS_EINVAL, "pad %u too large", pad);
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
  const uint32_t n = reads->n;
  DeviceReads dr;
  EncodedReads er;
  uint8_t* slab = nullptr;
  maxss_top2* dtop = nullptr;
  maxss_aln* dout = nullptr;
  char* dcig = nullptr;
  do {
    NwShape sh;
    if ((s = nw_shape(ix, n, pad, &sh))) break;
    if ((s = stage_reads(reads, st, &dr))) break;
    if ((s = alloc_encoded(ix, n, st, &er))) break;
    if ((s = encode_reads_into(ix, dr, st, er))) break;
    if ((s = check_hip(dev_malloc_async((void**)&slab, (size_t)sh.grid * ix->p.max_read_len * sh.rowbytes,
                                      st),
                       "alloc NW slab")))
      break;
    if (reads->on_device) {
      dtop = const_cast<maxss_top2*>(top);
      dout = out;
      dcig = cigar;
    } else {
      if ((s = check_hip(dev_malloc_async((void**)&dtop, sizeof(maxss_top2) * n, st), "alloc top")) ||
          (s = check_hip(dev_malloc_async((void**)&dout, sizeof(maxss_aln) * n, st), "alloc aln")) ||
          (s = check_hip(dev_malloc_async((void**)&dcig, (size_t)n * cigar_stride, st), "alloc cigar")) ||
          (s = check_hip(hipMemcpyAsync(dtop, top, sizeof(maxss_top2) * n, hipMemcpyHostToDevice, st),
                         "copy top")))
        break;
    }
    if ((s = nw_pipeline(ix, er, n, dtop, pad, dout, dcig, cigar_stride, slab, sh, st))) break;
    if (!reads->on_device) {
      if ((s = check_hip(hipMemcpyAsync(out, dout, sizeof(maxss_aln) * n, hipMemcpyDeviceToHost, st),
                         "copy aln")) ||
          (s = check_hip(hipMemcpyAsync(cigar, dcig, (size_t)n * cigar_stride, hipMemcpyDeviceToHost, st),
                         "copy cigar")))
        break;
    }
  } while (0);
  if (slab) (void)hipFreeAsync(slab, st);
  if (!reads->on_device) {
    if (dtop) (void)hipFreeAsync(dtop, st);
    if (dout) (void)hipFreeAsync(dout, st);
    if (dcig) (void)hipFreeAsync(dcig, st);
  }
  release_encoded(&er, st);
  release_reads(&dr, st);
  if (!reads->on_device && s == MAXSS_OK) s = check_hip(hipStreamSynchronize(st), "sync");
  return s;
}
