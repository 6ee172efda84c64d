// Learned fragment proposal: 4-mer profiles, a 512-256-1 MLP in bf16 with
// fp32 accumulation (MFMA GEMMs + a VALU pair stage), per-read top-K with a
// margin test, and the MLP's training step (forward, backward, Adam).  HIP,
// gfx950.  Not in the paper: the proposal only ranks fragments; every
// fragment that is scanned is scored by the exact MaxSS scan.
//
// Network: z = [v_read ; v_frag] (two L2-normalised 256-bin 4-mer count
// profiles), h = ReLU(W1 z + b1), y = w2 . h + b2.  Inference uses
// W1 z = W1a v_read + W1b v_frag: A = V_read W1a^T (+ b1) and B = V_frag W1b^T
// are two bf16 MFMA GEMMs; the pair stage computes sum_k w2[k] ReLU(A + B)
// for every (read strand, fragment) on the fp32 VALU.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace maxss {

static constexpr int kD = 256;                       // profile bins (4^4)
static constexpr int kH = 256;                       // hidden units
static constexpr uint32_t kW1 = kH * 2 * kD;         // 131,072
static constexpr uint32_t kParams = kW1 + kH + kH + 1;  // 131,585
static constexpr int kCand = 64;                     // candidates per training read

// SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) in counter mode, for the random numbers the
// library draws itself (initial weights, read order and negatives of
// training): draw k (k = 0, 1, ...) of stream s under `seed` is
// mix64(key + (k + 1) * gamma) with key = mix64(seed * gamma + s), mix64
// being the generator's output function.  A unit double takes the top 53
// bits; an integer in [0, n) is floor(unit * n).
static constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm_key(uint64_t seed, uint64_t stream) {
  return mix64(seed * kGamma + stream);
}
__host__ __device__ inline uint64_t sm_draw(uint64_t key, uint64_t k) {
  return mix64(key + (k + 1) * kGamma);
}
__host__ __device__ inline double sm_unit(uint64_t x) {
  return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}
// streams: initial weights, negatives, read order of epoch e (kStreamOrder + e)
static constexpr uint64_t kStreamInit = 1, kStreamNeg = 2, kStreamOrder = 16;

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __host__ inline uint16_t f2bf(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}

__device__ __host__ inline float bf2f(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float x;
  memcpy(&x, &u, 4);
  return x;
}

// ------------------------------------------------------------- profiles

// One wave per profile: counts of the 4-mers without N of a code sequence,
// normalised in float64 (exact integer sum of squares, correctly rounded
// sqrt and divide), rounded to float32 and then to bf16.
// Reads: row = 2*i + s (s = 1: reverse complement of read i).
// Fragments: row = f, 4-mers starting in [fF, fF+F) of the genome codes.
__global__ __launch_bounds__(256) void profile_kernel(
    const uint8_t* __restrict__ rcodes, const uint32_t* __restrict__ lens, uint32_t mstride,
    uint32_t nreads, const uint8_t* __restrict__ gcodes, uint32_t F, uint32_t NF,
    uint16_t* __restrict__ out_bf, float* __restrict__ out_f32) {
  __shared__ int cnt[4][kD];
  const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t row = blockIdx.x * 4 + wv;
  const uint32_t nrows = rcodes ? 2 * nreads : NF;
  int* c = cnt[wv];
  for (int b = lane; b < kD; b += 64) c[b] = 0;
  __syncthreads();
  if (row < nrows) {
    if (rcodes) {
      const uint32_t i = row >> 1, s = row & 1;
      const uint32_t m = lens[i];
      const uint8_t* q = rcodes + (uint64_t)i * mstride;
      for (uint32_t t = lane; t + 3 < m; t += 64) {
        uint32_t x0, x1, x2, x3;
        if (!s) {
          x0 = q[t]; x1 = q[t + 1]; x2 = q[t + 2]; x3 = q[t + 3];
        } else {  // reverse complement position t = complement of m-1-t
          x0 = q[m - 1 - t]; x1 = q[m - 2 - t]; x2 = q[m - 3 - t]; x3 = q[m - 4 - t];
          x0 = x0 == kN ? kN : 3 - x0; x1 = x1 == kN ? kN : 3 - x1;
          x2 = x2 == kN ? kN : 3 - x2; x3 = x3 == kN ? kN : 3 - x3;
        }
        if (x0 < 4 && x1 < 4 && x2 < 4 && x3 < 4) atomicAdd(&c[64 * x0 + 16 * x1 + 4 * x2 + x3], 1);
      }
    } else {
      const uint64_t base = (uint64_t)row * F;
      for (uint32_t t = lane; t < F; t += 64) {
        const uint8_t* g = gcodes + base + t;  // codes past the genome end are N
        const uint32_t x0 = g[0], x1 = g[1], x2 = g[2], x3 = g[3];
        if (x0 < 4 && x1 < 4 && x2 < 4 && x3 < 4) atomicAdd(&c[64 * x0 + 16 * x1 + 4 * x2 + x3], 1);
      }
    }
  }
  __syncthreads();
  if (row >= nrows) return;
  long long ss = 0;
  for (int b = lane; b < kD; b += 64) ss += (long long)c[b] * c[b];
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o, 64);
  const double nrm = sqrt((double)ss);
  for (int b = lane; b < kD; b += 64) {
    const float v = ss > 0 ? (float)((double)c[b] / nrm) : 0.0f;
    out_bf[(uint64_t)row * kD + b] = f2bf(v);
    if (out_f32) out_f32[(uint64_t)row * kD + b] = v;
  }
}

// ---------------------------------------------------------- MFMA GEMM

// Operand view: element (r, k) = p[(ri ? ri[r] : r) * sr + (ki ? ki[k] : k) * sk]
// (bf16), with optional row / reduction-index gathers.
struct Opnd {
  const uint16_t* p;
  long long sr, sk;
  const int32_t* ri;
  const int32_t* ki;
};

__device__ inline uint16_t opnd_at(const Opnd& o, int r, int k) {
  const long long rr = o.ri ? o.ri[r] : r;
  const long long kk = o.ki ? o.ki[k] : k;
  return o.p[rr * o.sr + kk * o.sk];
}

// LDS row of a staged slab: 32 k values plus 8 halfwords of padding (80
// bytes, so 16-byte reads stay aligned and rows start on different banks).
static constexpr int kLdsRow = 40;

// One operand's 64 x 32 slab (rows base.., k k0..) into LDS, zero outside
// [0, lim) x [k0, kend).  When the operand's k values are contiguous (row
// gathers allowed), a thread moves 8 of them of one row with one 16-byte
// load and store; when its rows are contiguous (reduction-index gathers
// allowed), a thread loads 8 rows of one k value with one 16-byte load and
// spreads them over the slab's rows; any other view, a ragged edge or an
// unaligned address takes the element-wise path.
__device__ inline void stage_opnd(uint16_t (*S)[kLdsRow], const Opnd& o, int base, int lim, int k0,
                                  int kend, int tid) {
  if (o.sk == 1 && !o.ki) {
    const int r = tid >> 2, c = (tid & 3) * 8;
    const int gr = base + r, gk = k0 + c;
    uint4 v = {0u, 0u, 0u, 0u};
    if (gr < lim) {
      const long long rr = o.ri ? o.ri[gr] : gr;
      const uint16_t* p = o.p + rr * o.sr + gk;
      if (gk + 8 <= kend && (reinterpret_cast<uintptr_t>(p) & 15u) == 0) {
        v = *reinterpret_cast<const uint4*>(p);
      } else {
        uint16_t h[8];
#pragma unroll
        for (int j = 0; j < 8; j++) h[j] = gk + j < kend ? p[j] : (uint16_t)0;
        memcpy(&v, h, 16);
      }
    }
    *reinterpret_cast<uint4*>(&S[r][c]) = v;
  } else if (o.sr == 1 && !o.ri) {
    const int kk = tid >> 3, r = (tid & 7) * 8;
    const int gk = k0 + kk, gr = base + r;
    uint16_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (gk < kend) {
      const long long kx = o.ki ? o.ki[gk] : gk;
      const uint16_t* p = o.p + gr + kx * o.sk;
      if (gr + 8 <= lim && (reinterpret_cast<uintptr_t>(p) & 15u) == 0) {
        const uint4 v = *reinterpret_cast<const uint4*>(p);
        memcpy(h, &v, 16);
      } else {
#pragma unroll
        for (int j = 0; j < 8; j++) h[j] = gr + j < lim ? p[j] : (uint16_t)0;
      }
    }
#pragma unroll
    for (int j = 0; j < 8; j++) S[r + j][kk] = h[j];
  } else {
    for (int e = tid; e < 64 * 32; e += 256) {
      const int r = e >> 5, kk = e & 31;
      const int gr = base + r, gk = k0 + kk;
      S[r][kk] = (gr < lim && gk < kend) ? opnd_at(o, gr, gk) : (uint16_t)0;
    }
  }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// C[i][j] (+)= sum_k A(i,k) B(j,k) (+ bias[j]), fp32 out (ldc), bf16 in.
// 256 threads, 64x64 output tile, each wave a 32x32 quarter of 2x2
// v_mfma_f32_16x16x32_bf16 tiles (gfx950: lane l holds 8 consecutive k of
// row l % 16 at k offset 8 (l / 16), one 16-byte LDS read per operand
// tile); K staged through LDS 32 at a time.  blockIdx.z takes the k range
// [z*kchunk, (z+1)*kchunk) and writes its partial product at C + z*zstride
// (split K).
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, int kchunk, Opnd A,
                                                        Opnd B, float* __restrict__ C,
                                                        long long ldc, long long zstride,
                                                        const float* __restrict__ bias,
                                                        int accumulate) {
  __shared__ __attribute__((aligned(16))) uint16_t As[64][kLdsRow];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[64][kLdsRow];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  C += blockIdx.z * zstride;
  f32x4 acc[2][2];
  for (int a = 0; a < 2; a++)
    for (int b = 0; b < 2; b++) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int ak = (lane >> 4) * 8;
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
    stage_opnd(As, A, i0, M, k0, kend, tid);
    stage_opnd(Bs, B, j0, N, k0, kend, tid);
    __syncthreads();
    bf16x8 a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; t++) {
      a[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&As[wi + t * 16 + (lane & 15)][ak]));
      b[t] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bs[wj + t * 16 + (lane & 15)][ak]));
    }
#pragma unroll
    for (int ti = 0; ti < 2; ti++)
#pragma unroll
      for (int tj = 0; tj < 2; tj++)
        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int ti = 0; ti < 2; ti++)
#pragma unroll
    for (int tj = 0; tj < 2; tj++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int gi = i0 + wi + ti * 16 + (lane >> 4) * 4 + r;
        const int gj = j0 + wj + tj * 16 + (lane & 15);
        if (gi < M && gj < N) {
          float v = acc[ti][tj][r];
          if (bias) v += bias[gj];
          float* cp = C + (long long)gi * ldc + gj;
          *cp = accumulate ? *cp + v : v;
        }
      }
}

// out[i] = sum over z of part[z][i], z in increasing order (deterministic).
__global__ void sum_splits_kernel(const float* __restrict__ part, int S, long long n,
                                  float* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < S; z++) s += part[z * n + i];
  out[i] = s;
}

constexpr int kSplitMax = 32;  // partial products a split-K GEMM may keep

// C = A B^T (+ bias, or += when accumulating).  With `part` (kSplitMax * M * N
// floats) and a long K against few output tiles, K is split so that the
// launch has about 512 workgroups, then the partials are summed in a fixed
// order; split GEMMs write a dense C (ldc = N) without bias or accumulation.
static maxss_status gemm(int M, int N, int K, const Opnd& A, const Opnd& B, float* C, long long ldc,
                         const float* bias, bool accumulate, hipStream_t st,
                         float* part = nullptr) {
  if (M <= 0 || N <= 0) return MAXSS_OK;
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int S = 1, kchunk = K;
  if (part && !bias && !accumulate && ldc == N && K > 0) {
    const int want = std::min(kSplitMax, std::max(1, (512 + tiles - 1) / tiles));
    const int kblocks = (K + 31) / 32;
    const int per = (kblocks + want - 1) / want;       // 32-wide k blocks per split
    kchunk = per * 32;
    S = (K + kchunk - 1) / kchunk;
  }
  ProfScope prof("gemm", st);
  if (S <= 1) {
    dim3 grid((N + 63) / 64, (M + 63) / 64, 1);
    gemm_bf16_kernel<<<grid, 256, 0, st>>>(M, N, K, std::max(K, 1), A, B, C, ldc, 0, bias,
                                           accumulate ? 1 : 0);
    return check_hip(hipGetLastError(), "gemm_bf16_kernel");
  }
  const long long n = (long long)M * N;
  dim3 grid((N + 63) / 64, (M + 63) / 64, S);
  gemm_bf16_kernel<<<grid, 256, 0, st>>>(M, N, K, kchunk, A, B, part, N, n, nullptr, 0);
  sum_splits_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(part, S, n, C);
  return check_hip(hipGetLastError(), "gemm_bf16_kernel (split K)");
}

// ------------------------------------------------------------ pair stage

// S[r][f] = max over strands s of  sum_k w2[k] ReLU(A[2r+s][k] + B[f][k]) + b2
// for reads [0, n) and fragments [0, NF).  A holds b1 already.  Tile: 32
// reads (64 A rows) x 64 fragments per 256-thread block; each thread owns
// 2 reads x 2 strands x 4 fragments.  K staged through LDS, transposed so
// that every thread reads 4 consecutive words.
__global__ __launch_bounds__(256) void pair_kernel(const float* __restrict__ A,
                                                   const float* __restrict__ B,
                                                   const float* __restrict__ w2, float b2, uint32_t n,
                                                   uint32_t NF, float* __restrict__ S,
                                                   uint32_t ldS) {
  __shared__ float At[32][64];
  __shared__ float Bt[32][64];
  __shared__ float ws[32];
  const uint32_t tid = threadIdx.x;
  const uint32_t rg = tid >> 4, fg = tid & 15;
  const uint32_t arow0 = blockIdx.y * 64;   // first A row (= 2 * first read)
  const uint32_t f0 = blockIdx.x * 64;
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = 0.f;
  for (int k0 = 0; k0 < kH; k0 += 32) {
    for (uint32_t e = tid; e < 64 * 32; e += 256) {
      const uint32_t r = e >> 5, kk = e & 31;
      const uint32_t ar = arow0 + r, fr = f0 + r;
      At[kk][r] = ar < 2 * n ? A[(uint64_t)ar * kH + k0 + kk] : 0.f;
      Bt[kk][r] = fr < NF ? B[(uint64_t)fr * kH + k0 + kk] : 0.f;
    }
    if (tid < 32) ws[tid] = w2[k0 + tid];
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 32; kk++) {
      const float w = ws[kk];
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = At[kk][rg * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; j++) b[j] = Bt[kk][fg * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = fmaf(w, fmaxf(a[i] + b[j], 0.f), acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 2; q++) {
    const uint32_t r = (arow0 >> 1) + rg * 2 + q;
    if (r >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const uint32_t f = f0 + fg * 4 + j;
      if (f < NF) S[(uint64_t)r * ldS + f] = fmaxf(acc[2 * q][j], acc[2 * q + 1][j]) + b2;
    }
  }
}

// ------------------------------------------------------------- top-K

__device__ inline uint64_t score_key(float s, uint32_t f) {
  uint32_t u = __float_as_uint(s);
  u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);  // order-preserving
  return ((uint64_t)u << 32) | (0xFFFFFFFFu - f);
}

// Per read (one 256-thread block): the K largest (score desc, fragment asc)
// keys by an 8-pass, 8-bit radix select, written as fragment ids in
// ascending order; margin = best score - second best; fell_back = margin < tau.
// Reads with lens == 0 (invalid) get no candidates and do not fall back.
__global__ __launch_bounds__(256) void topk_kernel(const float* __restrict__ S, uint32_t ldS,
                                                   uint32_t NF, uint32_t K, float tau,
                                                   const uint32_t* __restrict__ lens,
                                                   uint32_t r0, int32_t* __restrict__ cand,
                                                   float* __restrict__ margin,
                                                   uint8_t* __restrict__ fb) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_need;
  __shared__ uint64_t red[4][2];
  __shared__ uint32_t s_base;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t rl = blockIdx.x, r = r0 + rl;
  const float* row = S + (uint64_t)rl * ldS;
  const uint32_t Ke = K < NF ? K : NF;
  // best and second-best keys
  uint64_t b1 = 0, b2 = 0;
  for (uint32_t f = tid; f < NF; f += 256) {
    const uint64_t k = score_key(row[f], f);
    if (k > b1) { b2 = b1; b1 = k; } else if (k > b2) { b2 = k; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t o1 = __shfl_xor(b1, o, 64), o2 = __shfl_xor(b2, o, 64);
    const uint64_t n1 = b1 > o1 ? b1 : o1;
    const uint64_t lo = b1 > o1 ? o1 : b1;
    const uint64_t m2 = b2 > o2 ? b2 : o2;
    b2 = lo > m2 ? lo : m2;
    b1 = n1;
  }
  if (lane == 0) { red[wv][0] = b1; red[wv][1] = b2; }
  if (tid == 0) { s_prefix = 0; s_need = Ke; }
  __syncthreads();
  if (tid == 0) {
    uint64_t x1 = 0, x2 = 0;
    for (int w = 0; w < 4; w++) {
      for (int t = 0; t < 2; t++) {
        const uint64_t k = red[w][t];
        if (k > x1) { x2 = x1; x1 = k; } else if (k > x2) { x2 = k; }
      }
    }
    const bool valid = lens[r] != 0;
    float mg = INFINITY;
    if (NF > 1) {
      const float s1 = row[0xFFFFFFFFu - (uint32_t)(x1 & 0xFFFFFFFFu)];
      const float s2 = row[0xFFFFFFFFu - (uint32_t)(x2 & 0xFFFFFFFFu)];
      mg = s1 - s2;
    }
    margin[r] = mg;
    fb[r] = (valid && mg < tau) ? 1 : 0;
  }
  // radix select of the Ke-th largest key
  for (int pass = 0; pass < 8; pass++) {
    const int sh = 56 - 8 * pass;
    const uint64_t pmask = pass ? (~0ull << (64 - 8 * pass)) : 0ull;
    hist[tid] = 0;
    __syncthreads();
    const uint64_t pre = s_prefix;
    for (uint32_t f = tid; f < NF; f += 256) {
      const uint64_t k = score_key(row[f], f);
      if ((k & pmask) == pre) atomicAdd(&hist[(k >> sh) & 0xFF], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t need = s_need;
      int b = 255;
      for (; b > 0; b--) {
        if (hist[b] >= need) break;
        need -= hist[b];
      }
      s_need = need;
      s_prefix = pre | ((uint64_t)b << sh);
    }
    __syncthreads();
  }
  const uint64_t T = s_prefix;  // the Ke-th largest key
  // keys >= T, compacted in increasing fragment order
  if (tid == 0) s_base = 0;
  __syncthreads();
  int32_t* out = cand + (uint64_t)r * K;
  for (uint32_t f0 = 0; f0 < NF; f0 += 256) {
    const uint32_t f = f0 + tid;
    const bool take = f < NF && score_key(row[f], f) >= T;
    const uint64_t bal = __ballot(take);
    if (lane == 0) hist[wv] = (uint32_t)__builtin_popcountll(bal);
    __syncthreads();
    uint32_t pos = s_base;
    for (uint32_t w = 0; w < wv; w++) pos += hist[w];
    pos += (uint32_t)__builtin_popcountll(bal & ((1ull << lane) - 1ull));
    if (take && pos < Ke) out[pos] = (int32_t)f;
    __syncthreads();
    if (tid == 0) s_base += hist[0] + hist[1] + hist[2] + hist[3];
    __syncthreads();
  }
  for (uint32_t c = Ke + tid; c < K; c += 256) out[c] = -1;
}

// fb[i] = 0 (keep the candidate scan's record) when the network's margin
// reaches tau or the best candidate's exact score reaches min_score, else 1
// (full scan); invalid reads keep fb = 0.
__global__ void guard_kernel(const float* __restrict__ margin, const maxss_top2* __restrict__ oc,
                             const uint32_t* __restrict__ lens, float tau, int32_t min_score,
                             uint32_t n, uint8_t* __restrict__ fb) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool accept = margin[i] >= tau || oc[i].score[0] >= min_score;
  fb[i] = (lens[i] != 0 && !accept) ? 1 : 0;
}

// lens_out[i] = (fb[i] == want) ? lens[i] : 0
__global__ void mask_lens_kernel(const uint32_t* __restrict__ lens, const uint8_t* __restrict__ fb,
                                 uint8_t want, uint32_t n, uint32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (fb[i] == want) ? lens[i] : 0u;
}

// out[i] = fb[i] ? full[i] : cand[i]; invalid reads keep the invalid record
__global__ void select_kernel(const maxss_top2* __restrict__ rc, const maxss_top2* __restrict__ rf,
                              const uint8_t* __restrict__ fb, const uint32_t* __restrict__ lens,
                              uint32_t n, maxss_top2* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = (lens[i] != 0 && fb[i]) ? rf[i] : rc[i];
}

// --------------------------------------------------------------- model

struct Model {
  int device = 0;
  float* master = nullptr;     // [kParams] fp32
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  uint16_t* W1a = nullptr;     // [kH][kD] bf16 (W1[:, :256])
  uint16_t* W1b = nullptr;     // [kH][kD] bf16 (W1[:, 256:])
  float* w2f = nullptr;        // [kH] w2 rounded to bf16, as fp32
  uint32_t step = 0;
  // training scratch, grown on demand
  uint32_t cap_reads = 0;
  EncodedReads er;
  uint16_t* rprof = nullptr;   // [cap][2][kD]
  float* Ar = nullptr;         // [cap][kH]
  float* Bc = nullptr;         // [cap*kCand][kH]
  float* dy = nullptr;         // [cap*kCand]
  float* lossv = nullptr;      // [cap]
  uint16_t* dH = nullptr;      // [cap*kCand][kH] bf16
  uint16_t* dA = nullptr;      // [cap][kH] bf16
  float* part = nullptr;       // [cap][2*kH + 1] per-read dw2, db1, db2
  float* grad = nullptr;       // [kParams]
  int32_t* rsel = nullptr;     // [cap] profile row per read (2*b + strand)
  // fragment profiles of the last index used (bf16, [NF][kD])
  const Index* fp_ix = nullptr;
  uint16_t* fprof = nullptr;
};

// bf16 shadows of W1 (split) and w2 from the fp32 master.
__global__ void shadow_kernel(const float* __restrict__ master, uint16_t* __restrict__ W1a,
                              uint16_t* __restrict__ W1b, float* __restrict__ w2f) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kW1) {
    const uint32_t k = i / (2 * kD), j = i - k * 2 * kD;
    const uint16_t b = f2bf(master[i]);
    if (j < kD) W1a[k * kD + j] = b; else W1b[k * kD + (j - kD)] = b;
  } else if (i < kW1 + kH) {
    // b1 stays fp32 in the master
  } else if (i < kW1 + 2 * kH) {
    w2f[i - kW1 - kH] = bf2f(f2bf(master[i]));
  }
}

static maxss_status refresh_shadow(Model* m, hipStream_t st) {
  shadow_kernel<<<(kParams + 255) / 256, 256, 0, st>>>(m->master, m->W1a, m->W1b, m->w2f);
  return check_hip(hipGetLastError(), "shadow_kernel");
}

static maxss_status ensure_fprof(Model* m, const Index* ix, hipStream_t st) {
  if (m->fp_ix == ix && m->fprof) return MAXSS_OK;
  if (m->fprof) (void)hipFree(m->fprof);
  m->fprof = nullptr;
  m->fp_ix = nullptr;
  maxss_status s;
  if ((s = check_hip(dev_malloc((void**)&m->fprof, sizeof(uint16_t) * (size_t)ix->NF * kD),
                     "alloc fragment profiles")))
    return s;
  profile_kernel<<<(ix->NF + 3) / 4, 256, 0, st>>>(nullptr, nullptr, 0, 0, ix->codes, ix->F, ix->NF,
                                                    m->fprof, nullptr);
  if ((s = check_hip(hipGetLastError(), "profile_kernel"))) return s;
  m->fp_ix = ix;
  return MAXSS_OK;
}

// ---------------------------------------------------------- training

// Forward + loss per read (one 256-thread block): 4 threads per candidate
// compute y_c = w2 . ReLU(A[b] + Bc[b,c]) + b2; one wave takes the softmax
// over the 64 candidates (label at 0): loss_b and dy = (p - onehot) / nb.
__global__ __launch_bounds__(256) void train_fwd_kernel(const float* __restrict__ Ar,
                                                        const float* __restrict__ Bc,
                                                        const float* __restrict__ w2, float b2,
                                                        uint32_t nb, float* __restrict__ dy,
                                                        float* __restrict__ lossv) {
  __shared__ float ys[kCand];
  const uint32_t b = blockIdx.x, tid = threadIdx.x;
  const uint32_t c = tid >> 2, q = tid & 3;
  const float* a = Ar + (uint64_t)b * kH;
  const float* bc = Bc + ((uint64_t)b * kCand + c) * kH;
  float s = 0.f;
  for (int k = q * 64; k < q * 64 + 64; k++) s = fmaf(w2[k], fmaxf(a[k] + bc[k], 0.f), s);
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  if (q == 0) ys[c] = s + b2;
  __syncthreads();
  if (tid < 64) {
    const float y = ys[tid];
    float mx = y;
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    float e = expf(y - mx), se = e;
    for (int o = 32; o > 0; o >>= 1) se += __shfl_xor(se, o, 64);
    const float lse = mx + logf(se);
    dy[(uint64_t)b * kCand + tid] = (e / se - (tid == 0 ? 1.f : 0.f)) / (float)nb;
    if (tid == 0) lossv[b] = lse - y;
  }
}

// Backward per read (one block, thread = hidden unit k): dH[b,c,k] =
// dy_c w2[k] [pre > 0] (bf16, for dW1b), dA[b,k] = sum_c dH (bf16, for dW1a),
// and this read's partial sums of dw2 (sum_c dy_c h_c), db1 and db2.
__global__ __launch_bounds__(256) void train_bwd_kernel(const float* __restrict__ Ar,
                                                        const float* __restrict__ Bc,
                                                        const float* __restrict__ w2,
                                                        const float* __restrict__ dy,
                                                        uint16_t* __restrict__ dH,
                                                        uint16_t* __restrict__ dA,
                                                        float* __restrict__ part) {
  const uint32_t b = blockIdx.x, k = threadIdx.x;
  const float a = Ar[(uint64_t)b * kH + k];
  const float wk = w2[k];
  float sa = 0.f, sw = 0.f;
  for (int c = 0; c < kCand; c++) {
    const uint64_t p = (uint64_t)b * kCand + c;
    const float pre = a + Bc[p * kH + k];
    const float d = dy[p];
    const float g = pre > 0.f ? d * wk : 0.f;
    dH[p * kH + k] = f2bf(g);
    sa += g;
    sw = fmaf(d, fmaxf(pre, 0.f), sw);
  }
  dA[(uint64_t)b * kH + k] = f2bf(sa);
  float* pr = part + (uint64_t)b * (2 * kH + 1);
  pr[k] = sw;
  pr[kH + k] = sa;
  if (k == 0) {
    float d = 0.f;
    for (int c = 0; c < kCand; c++) d += dy[(uint64_t)b * kCand + c];
    pr[2 * kH] = d;
  }
}

// Deterministic reduction of the per-read partials into the gradient
// (dw2, db1, db2) and of the per-read losses into the mean loss.  A block
// takes 64 consecutive sums (the last block the loss); thread group g of 4
// adds the partials of reads b = g, g + 4, ... in increasing b, and the four
// group sums are added in group order.
__global__ __launch_bounds__(256) void train_reduce_kernel(const float* __restrict__ part,
                                                           const float* __restrict__ lossv,
                                                           uint32_t nb, float* __restrict__ grad,
                                                           float* __restrict__ loss) {
  __shared__ float acc[4][64];
  constexpr uint32_t kSums = 2 * kH + 1;
  const uint32_t j = threadIdx.x & 63, g = threadIdx.x >> 6;
  const bool loss_block = blockIdx.x == (kSums + 63) / 64;
  const uint32_t k = blockIdx.x * 64 + j;  // 0 .. 2*kH
  float s = 0.f;
  if (loss_block) {
    if (j == 0)
      for (uint32_t b = g; b < nb; b += 4) s += lossv[b];
  } else if (k < kSums) {
    for (uint32_t b = g; b < nb; b += 4) s += part[(uint64_t)b * kSums + k];
  }
  acc[g][j] = s;
  __syncthreads();
  if (g != 0) return;
  const float t = ((acc[0][j] + acc[1][j]) + acc[2][j]) + acc[3][j];
  if (loss_block) {
    if (j == 0 && loss) *loss = t / (float)nb;
  } else if (k < kH) {
    grad[kW1 + kH + k] = t;          // dw2
  } else if (k < 2 * kH) {
    grad[kW1 + (k - kH)] = t;        // db1
  } else if (k < kSums) {
    grad[kParams - 1] = t;           // db2
  }
}

// dW1 assembly: grad[k*512 + j] from dW1a (j < 256) and dW1b (j >= 256),
// both [kH][kD] fp32 in `tmp`.
__global__ void assemble_w1_kernel(const float* __restrict__ tmp, float* __restrict__ grad) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kW1) return;
  const uint32_t k = i / (2 * kD), j = i - k * 2 * kD;
  grad[i] = j < kD ? tmp[k * kD + j] : tmp[kH * kD + k * kD + (j - kD)];
}

// Adam (Kingma & Ba, 2015) on the fp32 master weights.
__global__ void adam_kernel(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, uint32_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void fill_flag_kernel(uint32_t* flag) { *flag = 0u; }

// flag |= 1 if any of the n fragment ids is outside [0, NF)
__global__ void check_ids_kernel(const int32_t* __restrict__ ids, uint32_t n, uint32_t NF,
                                 uint32_t* __restrict__ flag) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (ids[i] < 0 || (uint32_t)ids[i] >= NF)) atomicOr(flag, 1u);
}

// row index of each read's label-strand profile: 2*b + strand[b]
__global__ void rsel_kernel(const int8_t* __restrict__ strand, uint32_t nb, int32_t* __restrict__ rs) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) rs[b] = (int32_t)(2 * b + (strand[b] ? 1 : 0));
}

static void free_train_scratch(Model* m) {
  void* ps[] = {m->er.sel4, m->er.codes, m->er.lens, m->rprof, m->Ar, m->Bc, m->dy, m->lossv,
                m->dH, m->dA, m->part, m->grad, m->rsel};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  m->er = EncodedReads{};
  m->rprof = nullptr; m->Ar = nullptr; m->Bc = nullptr; m->dy = nullptr; m->lossv = nullptr;
  m->dH = nullptr; m->dA = nullptr; m->part = nullptr; m->grad = nullptr; m->rsel = nullptr;
  m->cap_reads = 0;
}

static maxss_status ensure_train_scratch(Model* m, const Index* ix, uint32_t nb) {
  if (nb <= m->cap_reads && m->er.mstride == read_stride(ix)) return MAXSS_OK;
  free_train_scratch(m);
  const uint32_t cap = nb;
  maxss_status s;
  m->er.mstride = read_stride(ix);
  const uint64_t P = (uint64_t)cap * kCand;
  if ((s = check_hip(dev_malloc((void**)&m->er.sel4, 4ull * (cap * 2ull * (m->er.mstride / 8) + 64)),
                     "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->er.codes, (uint64_t)cap * m->er.mstride + 64), "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->er.lens, 4ull * (cap + 1)), "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->rprof, 2ull * cap * 2 * kD), "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->Ar, 4ull * cap * kH), "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->Bc, 4ull * P * kH), "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->dy, 4ull * P), "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->lossv, 4ull * cap), "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->dH, 2ull * P * kH), "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->dA, 2ull * cap * kH), "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->part, 4ull * cap * (2 * kH + 1)), "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->grad,
                                4ull * (kParams + 2 * kH * kD + (size_t)kSplitMax * kH * kD)),
                      "alloc")) ||
      (s = check_hip(dev_malloc((void**)&m->rsel, 4ull * cap), "alloc"))) {
    free_train_scratch(m);
    return s;
  }
  m->cap_reads = cap;
  return MAXSS_OK;
}

}  // namespace maxss

using namespace maxss;

extern "C" void maxss_model_free(maxss_model* model) {
  Model* m = reinterpret_cast<Model*>(model);
  if (!m) return;
  free_train_scratch(m);
  void* ps[] = {m->master, m->adam_m, m->adam_v, m->W1a, m->W1b, m->w2f, m->fprof};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  delete m;
}

extern "C" maxss_status maxss_model_get_params(const maxss_model* model, float* out) {
  clear_error();
  const Model* m = reinterpret_cast<const Model*>(model);
  if (!m || !out) return fail(MAXSS_EINVAL, "NULL argument");
  return check_hip(hipMemcpy(out, m->master, 4ull * kParams, hipMemcpyDeviceToHost), "copy params");
}

static const char kMagic[8] = {'M', 'A', 'X', 'S', 'S', 'M', 'L', 'P'};

extern "C" maxss_status maxss_model_save(const maxss_model* model, const char* path) {
  clear_error();
  const Model* m = reinterpret_cast<const Model*>(model);
  if (!m || !path) return fail(MAXSS_EINVAL, "NULL argument");
  std::vector<float> buf(3ull * kParams);
  maxss_status s;
  if ((s = check_hip(hipMemcpy(buf.data(), m->master, 4ull * kParams, hipMemcpyDeviceToHost), "copy")) ||
      (s = check_hip(hipMemcpy(buf.data() + kParams, m->adam_m, 4ull * kParams, hipMemcpyDeviceToHost),
                     "copy")) ||
      (s = check_hip(hipMemcpy(buf.data() + 2 * kParams, m->adam_v, 4ull * kParams,
                               hipMemcpyDeviceToHost),
                     "copy")))
    return s;
  FILE* f = fopen(path, "wb");
  if (!f) return fail(MAXSS_EINVAL, "cannot open %s for writing", path);
  const uint32_t hdr[3] = {1u, m->step, kParams};  // format version, step, parameter count
  bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(hdr, 4, 3, f) == 3 &&
            fwrite(buf.data(), 4, buf.size(), f) == buf.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? MAXSS_OK : fail(MAXSS_EINVAL, "short write to %s", path);
}

extern "C" maxss_status maxss_model_load(const char* path, maxss_model** out) {
  clear_error();
  if (!path || !out) return fail(MAXSS_EINVAL, "NULL argument");
  FILE* f = fopen(path, "rb");
  if (!f) return fail(MAXSS_EINVAL, "cannot open %s", path);
  char mg[8];
  uint32_t hdr[3];
  std::vector<float> buf(3ull * kParams);
  const bool ok = fread(mg, 1, 8, f) == 8 && memcmp(mg, kMagic, 8) == 0 && fread(hdr, 4, 3, f) == 3 &&
                  hdr[0] == 1u && hdr[2] == kParams && fread(buf.data(), 4, buf.size(), f) == buf.size();
  fclose(f);
  if (!ok) return fail(MAXSS_EINVAL, "%s is not a version-1 model file", path);
  maxss_status s = maxss_model_from_params(buf.data(), out);
  if (s) return s;
  Model* m = reinterpret_cast<Model*>(*out);
  m->step = hdr[1];
  if ((s = check_hip(hipMemcpy(m->adam_m, buf.data() + kParams, 4ull * kParams, hipMemcpyHostToDevice),
                     "copy")) ||
      (s = check_hip(hipMemcpy(m->adam_v, buf.data() + 2 * kParams, 4ull * kParams,
                               hipMemcpyHostToDevice),
                     "copy"))) {
    maxss_model_free(*out);
    *out = nullptr;
    return s;
  }
  return MAXSS_OK;
}

extern "C" maxss_status maxss_profiles(const maxss_index* index, const maxss_reads* reads,
                                       float* read_prof, float* frag_prof, void* stream) {
  clear_error();
  const Index* ix = reinterpret_cast<const Index*>(index);
  if (!ix || (!read_prof && !frag_prof)) return fail(MAXSS_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  maxss_status s = MAXSS_OK;
  uint16_t* tmp = nullptr;
  DeviceReads dr;
  EncodedReads er;
  const uint32_t n = (reads && read_prof) ? reads->n : 0;
  do {
    if (reads && read_prof) {
      if (!reads->on_device) { s = fail(MAXSS_EINVAL, "profiles take device reads"); break; }
      if (n) {
        if ((s = stage_reads(reads, st, &dr))) break;
        if ((s = alloc_encoded(ix, n, st, &er))) break;
        if ((s = encode_reads_into(ix, dr, st, er))) break;
        if ((s = check_hip(dev_malloc_async((void**)&tmp, 2ull * n * 2 * kD, st), "alloc"))) break;
        profile_kernel<<<(2 * n + 3) / 4, 256, 0, st>>>(er.codes, er.lens, er.mstride, n, nullptr,
                                                         0, 0, tmp, read_prof);
        if ((s = check_hip(hipGetLastError(), "profile_kernel"))) break;
        (void)hipFreeAsync(tmp, st);
        tmp = nullptr;
      }
    }
    if (frag_prof) {
      if ((s = check_hip(dev_malloc_async((void**)&tmp, 2ull * ix->NF * kD, st), "alloc"))) break;
      profile_kernel<<<(ix->NF + 3) / 4, 256, 0, st>>>(nullptr, nullptr, 0, 0, ix->codes, ix->F,
                                                        ix->NF, tmp, frag_prof);
      if ((s = check_hip(hipGetLastError(), "profile_kernel"))) break;
    }
  } while (0);
  if (tmp) (void)hipFreeAsync(tmp, st);
  release_encoded(&er, st);
  release_reads(&dr, st);
  return s;
}

// A = V_read W1a^T + b1 for rows [0, 2n): rprof [2n][kD] bf16 -> A [2n][kH]
static maxss_status read_side(const Model* m, const uint16_t* rprof, uint32_t rows, float* A,
                              hipStream_t st) {
  Opnd a{rprof, kD, 1, nullptr, nullptr};
  Opnd b{m->W1a, kD, 1, nullptr, nullptr};
  return gemm((int)rows, kH, kD, a, b, A, kH, m->master + kW1, false, st);
}

static maxss_status frag_side(const Model* m, const uint16_t* fprof, uint32_t NF, float* B,
                              hipStream_t st) {
  Opnd a{fprof, kD, 1, nullptr, nullptr};
  Opnd b{m->W1b, kD, 1, nullptr, nullptr};
  return gemm((int)NF, kH, kD, a, b, B, kH, nullptr, false, st);
}

static float host_b2(const Model* m) {
  float b2 = 0.f;
  (void)hipMemcpy(&b2, m->master + kParams - 1, 4, hipMemcpyDeviceToHost);
  return b2;
}

extern "C" maxss_status maxss_proposal_scores(const maxss_index* index, maxss_model* model,
                                              const maxss_reads* reads, float* scores,
                                              void* stream) {
  clear_error();
  const Index* ix = reinterpret_cast<const Index*>(index);
  Model* m = reinterpret_cast<Model*>(model);
  if (!ix || !m || !reads || !scores) return fail(MAXSS_EINVAL, "NULL argument");
  if (!reads->on_device) return fail(MAXSS_EINVAL, "scores take device reads");
  const uint32_t n = reads->n;
  if (n == 0) return MAXSS_OK;
  hipStream_t st = (hipStream_t)stream;
  maxss_status s;
  DeviceReads dr;
  EncodedReads er;
  uint16_t* rprof = nullptr;
  float *A = nullptr, *B = nullptr;
  do {
    if ((s = ensure_fprof(m, ix, st))) break;
    if ((s = stage_reads(reads, st, &dr))) break;
    if ((s = alloc_encoded(ix, n, st, &er))) break;
    if ((s = encode_reads_into(ix, dr, st, er))) break;
    if ((s = check_hip(dev_malloc_async((void**)&rprof, 2ull * n * 2 * kD, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&A, 4ull * n * 2 * kH, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&B, 4ull * ix->NF * kH, st), "alloc")))
      break;
    profile_kernel<<<(2 * n + 3) / 4, 256, 0, st>>>(er.codes, er.lens, er.mstride, n, nullptr, 0, 0,
                                                     rprof, nullptr);
    if ((s = check_hip(hipGetLastError(), "profile_kernel"))) break;
    if ((s = read_side(m, rprof, 2 * n, A, st))) break;
    if ((s = frag_side(m, m->fprof, ix->NF, B, st))) break;
    const float b2 = host_b2(m);
    dim3 grid((ix->NF + 63) / 64, (n + 31) / 32);
    {
      ProfScope prof("pair", st);
      pair_kernel<<<grid, 256, 0, st>>>(A, B, m->w2f, b2, n, ix->NF, scores, ix->NF);
    }
    s = check_hip(hipGetLastError(), "pair_kernel");
  } while (0);
  if (rprof) (void)hipFreeAsync(rprof, st);
  if (A) (void)hipFreeAsync(A, st);
  if (B) (void)hipFreeAsync(B, st);
  release_encoded(&er, st);
  release_reads(&dr, st);
  return s;
}

// Bytes of the per-batch score matrix of the proposal.
static constexpr uint64_t kScoreBudget = 512ull << 20;

// Scores, top-K candidates (cand [n][K], ascending), margins and fall-back
// flags for n encoded reads (er).  Scratch is stream-ordered.
static maxss_status propose_impl(const Index* ix, Model* m, const EncodedReads& er, uint32_t n,
                                 uint32_t K, float tau, int32_t* cand, float* mg, uint8_t* fb,
                                 hipStream_t st) {
  maxss_status s;
  uint16_t* rprof = nullptr;
  float *A = nullptr, *B = nullptr, *S = nullptr;
  do {
    if ((s = ensure_fprof(m, ix, st))) break;
    if ((s = check_hip(dev_malloc_async((void**)&rprof, 2ull * n * 2 * kD, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&A, 4ull * n * 2 * kH, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&B, 4ull * ix->NF * kH, st), "alloc")))
      break;
    {
      ProfScope prof("profile", st);
      profile_kernel<<<(2 * n + 3) / 4, 256, 0, st>>>(er.codes, er.lens, er.mstride, n, nullptr, 0,
                                                       0, rprof, nullptr);
    }
    if ((s = check_hip(hipGetLastError(), "profile_kernel"))) break;
    if ((s = read_side(m, rprof, 2 * n, A, st))) break;
    if ((s = frag_side(m, m->fprof, ix->NF, B, st))) break;
    const float b2 = host_b2(m);
    uint64_t batch = kScoreBudget / (4ull * ix->NF);
    if (batch < 1) batch = 1;
    if (batch > n) batch = n;
    if ((s = check_hip(dev_malloc_async((void**)&S, 4ull * batch * ix->NF, st), "alloc scores"))) break;
    for (uint32_t r0 = 0; r0 < n && !s; r0 += (uint32_t)batch) {
      const uint32_t nb = (uint32_t)((n - r0) < batch ? (n - r0) : batch);
      dim3 grid((ix->NF + 63) / 64, (nb + 31) / 32);
      {
        ProfScope prof("pair", st);
        pair_kernel<<<grid, 256, 0, st>>>(A + (uint64_t)r0 * 2 * kH, B, m->w2f, b2, nb, ix->NF, S,
                                          ix->NF);
      }
      if ((s = check_hip(hipGetLastError(), "pair_kernel"))) break;
      {
        ProfScope prof("topk", st);
        topk_kernel<<<nb, 256, 0, st>>>(S, ix->NF, ix->NF, K, tau, er.lens, r0, cand, mg, fb);
      }
      s = check_hip(hipGetLastError(), "topk_kernel");
    }
  } while (0);
  void* ps[] = {rprof, A, B, S};
  for (void* p : ps)
    if (p) (void)hipFreeAsync(p, st);
  return s;
}

extern "C" maxss_status maxss_proposal_candidates(const maxss_index* index, maxss_model* model,
                                                  const maxss_reads* reads, uint32_t K, float margin,
                                                  int32_t* cand, float* margins, uint8_t* fell_back,
                                                  void* stream) {
  clear_error();
  const Index* ix = reinterpret_cast<const Index*>(index);
  Model* m = reinterpret_cast<Model*>(model);
  if (!ix || !m || !reads || !cand || !margins || !fell_back)
    return fail(MAXSS_EINVAL, "NULL argument");
  if (!reads->on_device) return fail(MAXSS_EINVAL, "the proposal path takes device reads");
  if (K == 0 || K > 4096) return fail(MAXSS_EINVAL, "K must be in 1..4096");
  const uint32_t n = reads->n;
  if (n == 0) return MAXSS_OK;
  hipStream_t st = (hipStream_t)stream;
  DeviceReads dr;
  dr.seq = reads->seq;
  dr.off = reads->offsets;
  dr.n = n;
  EncodedReads er;
  maxss_status s;
  do {
    if ((s = alloc_encoded(ix, n, st, &er))) break;
    if ((s = encode_reads_into(ix, dr, st, er))) break;
    s = propose_impl(ix, m, er, n, K, margin, cand, margins, fell_back, st);
  } while (0);
  release_encoded(&er, st);
  return s;
}

extern "C" maxss_status maxss_scan_reads_proposed(const maxss_index* index, maxss_model* model,
                                                  const maxss_reads* reads, uint32_t K,
                                                  float margin_tau, int32_t min_score,
                                                  maxss_top2* out, uint8_t* fell_back,
                                                  void* stream) {
  clear_error();
  const Index* ix = reinterpret_cast<const Index*>(index);
  Model* m = reinterpret_cast<Model*>(model);
  if (!ix || !m || !reads || !out) return fail(MAXSS_EINVAL, "NULL argument");
  if (!reads->on_device) return fail(MAXSS_EINVAL, "the proposal path takes device reads");
  if (K == 0 || K > 4096) return fail(MAXSS_EINVAL, "K must be in 1..4096");
  if (maxss_status q = require_quals(ix, reads)) return q;
  const uint32_t n = reads->n;
  if (n == 0) return MAXSS_OK;
  if (!reads->seq || !reads->offsets) return fail(MAXSS_EINVAL, "NULL reads");
  hipStream_t st = (hipStream_t)stream;
  maxss_status s;
  DeviceReads dr;
  dr.seq = reads->seq;
  dr.off = reads->offsets;
  dr.qual = reads->qual;
  dr.n = n;
  ScanWork wc, wf;
  float* mg = nullptr;
  int32_t* cand = nullptr;
  uint8_t* fb = nullptr;
  uint32_t *lens_c = nullptr, *lens_f = nullptr;
  maxss_top2 *oc = nullptr, *of = nullptr;
  const uint32_t Kc = K < ix->NF ? K : ix->NF;
  do {
    if ((s = alloc_scan_work(ix, n, scan_partial_entries(ix, n, nullptr), true, st, &wf))) break;
    if ((s = encode_reads_into(ix, dr, st, wf.er))) break;
    if ((s = check_hip(dev_malloc_async((void**)&cand, 4ull * n * K, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&mg, 4ull * n, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&fb, n, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&lens_c, 4ull * n, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&lens_f, 4ull * n, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&oc, sizeof(maxss_top2) * n, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&of, sizeof(maxss_top2) * n, st), "alloc")))
      break;
    if ((s = propose_impl(ix, m, wf.er, n, K, margin_tau, cand, mg, fb, st))) break;
    if ((s = alloc_scan_work(ix, n, (uint64_t)n * (Kc < 16 ? Kc : 16), true, st, &wc))) break;
    if (min_score >= 0) {
      // exact-score guard: every read's candidates are scanned, and a read
      // keeps that record when its margin reaches tau or its best
      // candidate's exact score reaches min_score
      if ((s = candidate_scan(ix, wf.er, wf.er.lens, n, cand, K, Kc, oc, wc, st))) break;
      guard_kernel<<<(n + 255) / 256, 256, 0, st>>>(mg, oc, wf.er.lens, margin_tau, min_score, n, fb);
      mask_lens_kernel<<<(n + 255) / 256, 256, 0, st>>>(wf.er.lens, fb, 1, n, lens_f);
      if ((s = check_hip(hipGetLastError(), "guard_kernel"))) break;
    } else {
      mask_lens_kernel<<<(n + 255) / 256, 256, 0, st>>>(wf.er.lens, fb, 0, n, lens_c);
      mask_lens_kernel<<<(n + 255) / 256, 256, 0, st>>>(wf.er.lens, fb, 1, n, lens_f);
      if ((s = check_hip(hipGetLastError(), "mask_lens_kernel"))) break;
      // candidate scan of the reads that kept their proposal
      if ((s = candidate_scan(ix, wf.er, lens_c, n, cand, K, Kc, oc, wc, st))) break;
    }
    // full scan of the reads that fell back
    if ((s = scan_pipeline_lens(ix, wf.er, lens_f, n, of, wf, st))) break;
    select_kernel<<<(n + 255) / 256, 256, 0, st>>>(oc, of, fb, wf.er.lens, n, out);
    if ((s = check_hip(hipGetLastError(), "select_kernel"))) break;
    if (fell_back &&
        (s = check_hip(hipMemcpyAsync(fell_back, fb, n, hipMemcpyDeviceToDevice, st), "copy fb")))
      break;
  } while (0);
  void* ps[] = {mg, cand, fb, lens_c, lens_f, oc, of};
  for (void* p : ps)
    if (p) (void)hipFreeAsync(p, st);
  release_scan_work(&wc, true, st);
  release_scan_work(&wf, true, st);
  return s;
}

namespace maxss {

// One step on nb reads whose label-strand profiles are rows rsel[b] of
// `rprof` (bf16, [rows][kD]) and whose 64 candidates (label first) are
// cand[b*64 ..]: forward, loss, backward, and with lr > 0 an Adam step.
// loss (device float, may be NULL) gets the batch mean, grad_out (device,
// may be NULL) the gradient.
static maxss_status train_step_impl(Model* m, const Index* ix, const uint16_t* rprof,
                                    const int32_t* rsel, const int32_t* cand, uint32_t nb,
                                    float lr, float* loss, float* grad_out, hipStream_t st) {
  maxss_status s;
  const uint32_t P = nb * kCand;
  // forward: A = Vr W1a^T + b1 (label strand rows), Bc = Vc W1b^T
  {
    Opnd a{rprof, kD, 1, rsel, nullptr};
    Opnd b{m->W1a, kD, 1, nullptr, nullptr};
    if ((s = gemm((int)nb, kH, kD, a, b, m->Ar, kH, m->master + kW1, false, st))) return s;
  }
  {
    Opnd a{m->fprof, kD, 1, cand, nullptr};
    Opnd b{m->W1b, kD, 1, nullptr, nullptr};
    if ((s = gemm((int)P, kH, kD, a, b, m->Bc, kH, nullptr, false, st))) return s;
  }
  const float b2 = host_b2(m);
  train_fwd_kernel<<<nb, 256, 0, st>>>(m->Ar, m->Bc, m->w2f, b2, nb, m->dy, m->lossv);
  train_bwd_kernel<<<nb, kH, 0, st>>>(m->Ar, m->Bc, m->w2f, m->dy, m->dH, m->dA, m->part);
  if ((s = check_hip(hipGetLastError(), "train fwd/bwd"))) return s;
  float* tmp = m->grad + kParams;  // [2][kH][kD] fp32 for dW1a, dW1b
  float* split = tmp + 2 * kH * kD;  // split-K partials, [kSplitMax][kH][kD]
  {
    // dW1a[k][j] = sum_b dA[b][k] Vr[rsel[b]][j]
    Opnd a{m->dA, 1, kH, nullptr, nullptr};
    Opnd b{rprof, 1, kD, nullptr, rsel};
    if ((s = gemm(kH, kD, (int)nb, a, b, tmp, kD, nullptr, false, st, split))) return s;
  }
  {
    // dW1b[k][j] = sum_p dH[p][k] Vf[cand[p]][j]
    Opnd a{m->dH, 1, kH, nullptr, nullptr};
    Opnd b{m->fprof, 1, kD, nullptr, cand};
    if ((s = gemm(kH, kD, (int)P, a, b, tmp + kH * kD, kD, nullptr, false, st, split)))
      return s;
  }
  assemble_w1_kernel<<<(kW1 + 255) / 256, 256, 0, st>>>(tmp, m->grad);
  train_reduce_kernel<<<(2 * kH + 1 + 63) / 64 + 1, 256, 0, st>>>(m->part, m->lossv, nb, m->grad, loss);
  if ((s = check_hip(hipGetLastError(), "train reduce"))) return s;
  if (grad_out &&
      (s = check_hip(hipMemcpyAsync(grad_out, m->grad, 4ull * kParams, hipMemcpyDeviceToDevice, st),
                     "copy grad")))
    return s;
  if (lr > 0.f) {
    m->step++;
    const float b1c = 1.f - powf(0.9f, (float)m->step), b2c = 1.f - powf(0.999f, (float)m->step);
    adam_kernel<<<(kParams + 255) / 256, 256, 0, st>>>(m->master, m->adam_m, m->adam_v, m->grad,
                                                       kParams, lr, 0.9f, 0.999f, 1e-8f, b1c, b2c);
    if ((s = check_hip(hipGetLastError(), "adam_kernel"))) return s;
    if ((s = refresh_shadow(m, st))) return s;
  }
  return MAXSS_OK;
}

}  // namespace maxss

extern "C" maxss_status maxss_model_train_step(maxss_model* model, const maxss_index* index,
                                               const maxss_reads* batch, const int32_t* cand,
                                               const int8_t* strand, float lr, float* loss,
                                               float* grad_out, void* stream) {
  clear_error();
  Model* m = reinterpret_cast<Model*>(model);
  const Index* ix = reinterpret_cast<const Index*>(index);
  if (!m || !ix || !batch || !cand || !strand) return fail(MAXSS_EINVAL, "NULL argument");
  if (!batch->on_device) return fail(MAXSS_EINVAL, "training takes device reads");
  const uint32_t nb = batch->n;
  if (nb == 0) return fail(MAXSS_EINVAL, "empty batch");
  hipStream_t st = (hipStream_t)stream;
  maxss_status s;
  DeviceReads dr;
  dr.seq = batch->seq;
  dr.off = batch->offsets;
  dr.n = nb;
  if ((s = ensure_fprof(m, ix, st))) return s;
  if ((s = ensure_train_scratch(m, ix, nb))) return s;
  {
    // every candidate must name a fragment of the index (they are gathered)
    uint32_t* flag = m->rsel ? reinterpret_cast<uint32_t*>(m->lossv) : nullptr;
    fill_flag_kernel<<<1, 1, 0, st>>>(flag);
    check_ids_kernel<<<(nb * kCand + 255) / 256, 256, 0, st>>>(cand, nb * kCand, ix->NF, flag);
    uint32_t h = 0;
    if ((s = check_hip(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, st), "copy flag")) ||
        (s = check_hip(hipStreamSynchronize(st), "sync")))
      return s;
    if (h) return fail(MAXSS_EINVAL, "candidate fragment ids must lie in [0, %u)", ix->NF);
  }
  if ((s = encode_reads_into(ix, dr, st, m->er))) return s;
  profile_kernel<<<(2 * nb + 3) / 4, 256, 0, st>>>(m->er.codes, m->er.lens, m->er.mstride, nb,
                                                    nullptr, 0, 0, m->rprof, nullptr);
  rsel_kernel<<<(nb + 255) / 256, 256, 0, st>>>(strand, nb, m->rsel);
  if ((s = check_hip(hipGetLastError(), "profile/rsel"))) return s;
  return train_step_impl(m, ix, m->rprof, m->rsel, cand, nb, lr, loss, grad_out, st);
}

// ------------------------------------------------- training loop, thresholds

namespace maxss {

// Initial parameters (fp32): MAXSS_INIT_GLOROT draws W1 and w2 uniformly in
// +-sqrt(6 / (fan_in + fan_out)) (Glorot & Bengio, 2010) from stream
// kStreamInit (W1 element i is draw i, w2 element k draw kW1 + k), biases 0.
// MAXSS_INIT_PROFILE_MATCH sets hidden unit k to compare bin k of the two
// profiles: W1[k][k] = 8 (read), W1[k][256 + k] = 1 (fragment), every other
// weight 0, b1 = -0.2, w2 = 1, b2 = 0, so that a read's 4-mers present in
// the fragment add the fragment's share of them (the score then ranks
// fragments much like the cosine of the profiles) and training starts there.
static void init_params(uint32_t seed, uint32_t kind, std::vector<float>& p) {
  p.assign(kParams, 0.0f);
  if (kind == MAXSS_INIT_PROFILE_MATCH) {
    for (int k = 0; k < kH; k++) {
      p[(size_t)k * 2 * kD + k] = 8.0f;
      p[(size_t)k * 2 * kD + kD + k] = 1.0f;
      p[kW1 + k] = -0.2f;
      p[kW1 + kH + k] = 1.0f;
    }
    return;
  }
  const uint64_t key = sm_key(seed, kStreamInit);
  const double a1 = sqrt(6.0 / (2 * kD + kH)), a2 = sqrt(6.0 / (kH + 1));
  for (uint32_t i = 0; i < kW1; i++) p[i] = (float)((2.0 * sm_unit(sm_draw(key, i)) - 1.0) * a1);
  for (uint32_t k = 0; k < (uint32_t)kH; k++)
    p[kW1 + kH + k] = (float)((2.0 * sm_unit(sm_draw(key, kW1 + k)) - 1.0) * a2);
}

// Candidate rows of a training batch: row b = [label, second (if it is a
// fragment other than the label), hard negatives (the model's best
// fragments other than the label, ascending ids, at most `hard`), distinct
// uniform draws over the fragments other than the label (draw c = (t*B + b)
// * 512 + k of stream kStreamNeg for k = 0, 1, ..., 511; f = floor(u *
// (NF - 1)), then f + 1 if f >= label)], and, when fewer than 63 negatives
// were found, the remaining fragments other than the label in increasing id
// order, repeated as needed.  rsel[b] = 2 * read + label strand.
// One wave per row, the row in LDS.  Each phase takes its entries in the
// rule's order: lane l holds entry k0 + l of a chunk of 64, which is kept
// when it is not in the row and equals no earlier entry of the chunk (an
// earlier equal entry was either kept, or dropped because its value was
// already in the row); the first free slots go to the kept lanes in lane
// order.
// Orders the wave's LDS accesses: what a lane wrote before is visible to
// every lane after.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline bool row_has(const int32_t* row, int n, int32_t f) {
  bool hit = false;
  for (int j = 0; j < n; j++) hit |= row[j] == f;
  return hit;
}

// Appends the kept candidates of a chunk (lane value f, ok = eligible),
// at most `room`; returns how many were appended.
__device__ inline int row_append(int32_t* row, int n, int room, int32_t f, bool ok) {
  const uint32_t lane = threadIdx.x & 63;
  bool dup = false;
  for (uint32_t i = 0; i < 63; i++) {
    const int32_t g = __shfl(f, (int)i, 64);
    dup |= i < lane && g == f;
  }
  const bool keep = ok && !dup && !row_has(row, n, f);
  const uint64_t m = __ballot(keep);
  const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  if (keep && (int)pos < room) row[n + pos] = f;
  const int cnt = __popcll(m);
  return cnt < room ? cnt : room;
}

__global__ __launch_bounds__(256) void negatives_kernel(
    const int32_t* __restrict__ bidx, const maxss_top2* __restrict__ labels,
    const int32_t* __restrict__ hardc, uint32_t hard_k, uint32_t hard, uint64_t key, uint64_t t,
    uint32_t B, uint32_t NF, int32_t* __restrict__ cand, int32_t* __restrict__ rsel) {
  __shared__ int32_t rows[4][kCand];
  const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t b = blockIdx.x * 4 + wv;
  if (b >= B) return;  // whole waves: the rest of the block never syncs
  int32_t* row = rows[wv];
  const int32_t r = bidx[b];
  const int32_t L = labels[r].frag[0], S2 = labels[r].frag[1];
  if (lane == 0) {
    rsel[b] = 2 * r + (labels[r].strand[0] ? 1 : 0);
    row[0] = L;
  }
  int n = 1;
  if (S2 >= 0 && (uint32_t)S2 < NF && S2 != L) {
    if (lane == 0) row[1] = S2;
    n = 2;
  }
  wave_sync();
  if (hardc) {
    // the model's best fragments in its order, at most `hard` of them
    const int32_t f = lane < hard_k ? hardc[(uint64_t)b * hard_k + lane] : -1;
    const int room = (int)hard < kCand - n ? (int)hard : kCand - n;
    n += row_append(row, n, room, f, f >= 0 && f != L);
    wave_sync();
  }
  if (NF > 1) {
    const uint64_t c0 = (t * B + b) * 512ull;
    for (uint32_t k0 = 0; k0 < 512 && n < kCand; k0 += 64) {
      int32_t f = (int32_t)(sm_unit(sm_draw(key, c0 + k0 + lane)) * (double)(NF - 1));
      if (f >= L) f++;
      n += row_append(row, n, kCand - n, f, true);
      wave_sync();
    }
  }
  for (uint32_t f0 = 0; f0 < NF && n < kCand; f0 += 64) {
    const uint32_t f = f0 + lane;
    n += row_append(row, n, kCand - n, (int32_t)f, f < NF && (int32_t)f != L);
    wave_sync();
  }
  // fewer than 64 fragments: the negatives found so far again (the label
  // itself when it is the only fragment)
  wave_sync();
  int32_t* out = cand + (uint64_t)b * kCand;
  const int j = (int)lane;
  out[j] = j < n ? row[j] : (n > 1 ? row[1 + (j - n) % (n - 1)] : L);
}

__global__ void fill_words_kernel(uint32_t* __restrict__ p, uint32_t v, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Profile rows of both strands of the batch reads: rows[2b + s] = 2 bidx[b] + s.
__global__ void batch_rows_kernel(const int32_t* __restrict__ bidx, uint32_t B,
                                  int32_t* __restrict__ rows) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2 * B) rows[i] = 2 * bidx[i >> 1] + (int32_t)(i & 1);
}

// hits += number of reads r (lens > 0) whose label fragment is among its K
// candidates.
__global__ void count_hits_kernel(const int32_t* __restrict__ cand, uint32_t K,
                                  const maxss_top2* __restrict__ labels,
                                  const uint32_t* __restrict__ lens, uint32_t n,
                                  uint32_t* __restrict__ hits) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || lens[i] == 0) return;
  const int32_t L = labels[i].frag[0];
  if (L < 0) return;
  for (uint32_t k = 0; k < K; k++)
    if (cand[(uint64_t)i * K + k] == L) {
      atomicAdd(hits, 1u);
      return;
    }
}

}  // namespace maxss

static maxss_status model_from_host(const float* params, maxss_model** out) {
  Model* m = new (std::nothrow) Model();
  if (!m) return fail(MAXSS_ENOMEM, "host allocation");
  maxss_status s;
  do {
    if ((s = check_hip(hipGetDevice(&m->device), "hipGetDevice"))) break;
    if ((s = check_hip(dev_malloc((void**)&m->master, 4ull * kParams), "alloc")) ||
        (s = check_hip(dev_malloc((void**)&m->adam_m, 4ull * kParams), "alloc")) ||
        (s = check_hip(dev_malloc((void**)&m->adam_v, 4ull * kParams), "alloc")) ||
        (s = check_hip(dev_malloc((void**)&m->W1a, 2ull * kH * kD), "alloc")) ||
        (s = check_hip(dev_malloc((void**)&m->W1b, 2ull * kH * kD), "alloc")) ||
        (s = check_hip(dev_malloc((void**)&m->w2f, 4ull * kH), "alloc")))
      break;
    if ((s = check_hip(hipMemcpy(m->master, params, 4ull * kParams, hipMemcpyHostToDevice), "copy")) ||
        (s = check_hip(hipMemset(m->adam_m, 0, 4ull * kParams), "memset")) ||
        (s = check_hip(hipMemset(m->adam_v, 0, 4ull * kParams), "memset")))
      break;
    if ((s = refresh_shadow(m, nullptr))) break;
    if ((s = check_hip(hipDeviceSynchronize(), "sync"))) break;
  } while (0);
  if (s) {
    maxss_model_free(reinterpret_cast<maxss_model*>(m));
    return s;
  }
  *out = reinterpret_cast<maxss_model*>(m);
  return MAXSS_OK;
}

extern "C" maxss_status maxss_model_create(uint32_t seed, uint32_t init, maxss_model** out) {
  clear_error();
  if (!out) return fail(MAXSS_EINVAL, "NULL argument");
  if (init != MAXSS_INIT_GLOROT && init != MAXSS_INIT_PROFILE_MATCH)
    return fail(MAXSS_EINVAL, "unknown initialisation %u", init);
  std::vector<float> p;
  init_params(seed, init, p);
  return model_from_host(p.data(), out);
}

extern "C" maxss_status maxss_model_from_params(const float* params, maxss_model** out) {
  clear_error();
  if (!params || !out) return fail(MAXSS_EINVAL, "NULL argument");
  return model_from_host(params, out);
}

extern "C" maxss_status maxss_choose_acceptance(uint32_t n, const float* margin,
                                                const int32_t* best_score, const uint8_t* correct,
                                                float target, float* tau, int32_t* min_score,
                                                float* accept_frac, float* agreement) {
  clear_error();
  if (!tau || !min_score || (n && (!margin || !best_score || !correct)))
    return fail(MAXSS_EINVAL, "NULL argument");
  if (!(target >= 0.0f && target <= 1.0f)) return fail(MAXSS_EINVAL, "target must lie in [0, 1]");
  // misses allowed among the n reads (a fallen-back read always agrees); the
  // slack of 1e-6 n absorbs the float rounding of `target` (0.8f < 0.8)
  const double budget = (1.0 - (double)target) * (double)n * (1.0 + 1e-6) + 1e-6 * (double)n + 1e-9;
  std::vector<uint32_t> idx(n);
  for (uint32_t i = 0; i < n; i++) idx[i] = i;
  // score rule alone: accept every read whose best exact score reaches the
  // threshold; the smallest threshold within the budget (ties accept together)
  std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
    return best_score[a] != best_score[b] ? best_score[a] > best_score[b] : a < b;
  });
  int32_t ms = -1;
  double miss = 0;
  for (uint32_t p = 0; p < n;) {
    uint32_t q = p;
    double add = 0;
    while (q < n && best_score[idx[q]] == best_score[idx[p]]) add += correct[idx[q++]] ? 0 : 1;
    if (best_score[idx[p]] < 0 || miss + add > budget) break;
    miss += add;
    ms = best_score[idx[p]];
    p = q;
  }
  // margin rule on the reads the score rule leaves: the smallest tau within
  // what is left of the budget
  std::vector<uint32_t> rest;
  for (uint32_t i = 0; i < n; i++)
    if (ms < 0 || best_score[i] < ms) rest.push_back(i);
  std::sort(rest.begin(), rest.end(), [&](uint32_t a, uint32_t b) {
    return margin[a] != margin[b] ? margin[a] > margin[b] : a < b;
  });
  float t = INFINITY;
  for (size_t p = 0; p < rest.size();) {
    size_t q = p;
    double add = 0;
    while (q < rest.size() && margin[rest[q]] == margin[rest[p]]) add += correct[rest[q++]] ? 0 : 1;
    if (!(margin[rest[p]] > -INFINITY) || miss + add > budget) break;
    miss += add;
    t = margin[rest[p]];
    p = q;
  }
  uint32_t acc = 0;
  for (uint32_t i = 0; i < n; i++)
    if (margin[i] >= t || (ms >= 0 && best_score[i] >= ms)) acc++;
  *tau = t;
  *min_score = ms;
  if (accept_frac) *accept_frac = n ? (float)acc / (float)n : 0.0f;
  if (agreement) *agreement = n ? (float)(1.0 - miss / (double)n) : 1.0f;
  return MAXSS_OK;
}

namespace maxss {

// The read order of epoch e: the valid training reads sorted by (draw r of
// stream kStreamOrder + e, r).
static void epoch_order(uint64_t seed, uint64_t e, const std::vector<int32_t>& valid,
                        std::vector<int32_t>& out) {
  const uint64_t key = sm_key(seed, kStreamOrder + e);
  std::vector<std::pair<uint64_t, int32_t>> kv(valid.size());
  for (size_t j = 0; j < valid.size(); j++) kv[j] = {sm_draw(key, (uint64_t)valid[j]), valid[j]};
  std::sort(kv.begin(), kv.end());
  out.resize(valid.size());
  for (size_t j = 0; j < kv.size(); j++) out[j] = kv[j].second;
}

// Encoded reads [a, n) of `er` (rows are contiguous per read).
static EncodedReads encoded_tail(const EncodedReads& er, uint32_t a) {
  EncodedReads t = er;
  t.sel4 = er.sel4 + (uint64_t)a * 2 * (er.mstride / 8);
  t.codes = er.codes + (uint64_t)a * er.mstride;
  t.lens = er.lens + a;
  if (er.qsc) t.qsc = er.qsc + (uint64_t)a * er.mstride;
  return t;
}

}  // namespace maxss

extern "C" maxss_status maxss_model_train(maxss_model* model, const maxss_index* index,
                                          const maxss_reads* reads, const maxss_top2* labels,
                                          const maxss_train_opts* opts, maxss_train_stats* stats,
                                          void* stream) {
  clear_error();
  Model* m = reinterpret_cast<Model*>(model);
  const Index* ix = reinterpret_cast<const Index*>(index);
  if (!m || !ix || !reads || !labels || !opts || !stats) return fail(MAXSS_EINVAL, "NULL argument");
  if (!reads->on_device) return fail(MAXSS_EINVAL, "training takes device reads");
  if (reads->n == 0 || !reads->seq || !reads->offsets) return fail(MAXSS_EINVAL, "no reads");
  const maxss_train_opts o = *opts;
  if (o.batch == 0 || o.batch > 65536) return fail(MAXSS_EINVAL, "batch must be in 1..65536");
  if (o.K == 0 || o.K > 4096) return fail(MAXSS_EINVAL, "K must be in 1..4096");
  if (o.hard_negatives > kCand - 2) return fail(MAXSS_EINVAL, "hard_negatives must be <= 62");
  if (!(o.val_fraction >= 0.0f && o.val_fraction <= 0.9f))
    return fail(MAXSS_EINVAL, "val_fraction must lie in [0, 0.9]");
  if (!(o.target_agreement >= 0.0f && o.target_agreement <= 1.0f))
    return fail(MAXSS_EINVAL, "target_agreement must lie in [0, 1]");
  if (!(o.lr >= 0.0f)) return fail(MAXSS_EINVAL, "lr must be >= 0");
  maxss_status s;
  if ((s = require_quals(ix, reads))) return s;
  int cur = 0;
  if ((s = check_hip(hipGetDevice(&cur), "hipGetDevice"))) return s;
  if (cur != ix->device || cur != m->device)
    return fail(MAXSS_ESTATE, "index, model and current device differ");
  hipStream_t st = (hipStream_t)stream;
  const uint32_t n = reads->n, NF = ix->NF, B = o.batch;
  const uint32_t n_val = (uint32_t)((double)n * (double)o.val_fraction);
  const uint32_t n_train = n - n_val;
  const uint32_t Kc = o.K < NF ? o.K : NF;
  memset(stats, 0, sizeof(*stats));
  stats->n_train = n_train;
  stats->n_val = n_val;
  std::vector<maxss_top2> hl(n);
  if ((s = check_hip(hipMemcpyAsync(hl.data(), labels, sizeof(maxss_top2) * n, hipMemcpyDeviceToHost, st),
                     "copy labels")) ||
      (s = check_hip(hipStreamSynchronize(st), "sync")))
    return s;
  auto labelled = [&](uint32_t i) {
    return hl[i].frag[0] >= 0 && (uint32_t)hl[i].frag[0] < NF &&
           (hl[i].strand[0] == 0 || hl[i].strand[0] == 1);
  };
  std::vector<int32_t> valid;
  for (uint32_t i = 0; i < n_train; i++)
    if (labelled(i)) valid.push_back((int32_t)i);
  uint32_t nv_val = 0;
  for (uint32_t i = n_train; i < n; i++) nv_val += labelled(i) ? 1u : 0u;
  if (o.steps > 0 && valid.empty()) return fail(MAXSS_EINVAL, "no labelled training reads");
  DeviceReads dr;
  dr.seq = reads->seq;
  dr.off = reads->offsets;
  dr.qual = reads->qual;
  dr.n = n;
  EncodedReads er;
  ScanWork wc;
  uint16_t* rprof = nullptr;
  int32_t *bidx = nullptr, *cand = nullptr, *rows2 = nullptr, *hardc = nullptr, *cand_v = nullptr;
  float *trace = nullptr, *best = nullptr, *Ah = nullptr, *Bf = nullptr, *Sh = nullptr;
  float *mg = nullptr, *mg_v = nullptr;
  uint32_t *hits = nullptr, *ones = nullptr;
  uint8_t *fb = nullptr, *fb_v = nullptr;
  maxss_top2* oc = nullptr;
  const uint32_t hk = o.hard_negatives ? o.hard_negatives + 1 : 0;
  std::vector<float> trace_h(o.steps ? o.steps : 1);
  do {
    if ((s = ensure_fprof(m, ix, st))) break;
    if ((s = ensure_train_scratch(m, ix, B))) break;
    if ((s = alloc_encoded(ix, n, st, &er))) break;
    if ((s = encode_reads_into(ix, dr, st, er))) break;
    if ((s = check_hip(dev_malloc_async((void**)&rprof, 2ull * n * 2 * kD, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&bidx, 4ull * B, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&cand, 4ull * B * kCand, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&trace, 4ull * (o.steps ? o.steps : 1), st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&best, 4ull * kParams, st), "alloc")) ||
        (s = check_hip(dev_malloc_async((void**)&hits, 4, st), "alloc")))
      break;
    profile_kernel<<<(2 * n + 3) / 4, 256, 0, st>>>(er.codes, er.lens, er.mstride, n, nullptr, 0, 0,
                                                     rprof, nullptr);
    if ((s = check_hip(hipGetLastError(), "profile_kernel"))) break;
    if (hk) {
      if ((s = check_hip(dev_malloc_async((void**)&rows2, 8ull * B, st), "alloc")) ||
          (s = check_hip(dev_malloc_async((void**)&hardc, 4ull * B * hk, st), "alloc")) ||
          (s = check_hip(dev_malloc_async((void**)&Ah, 4ull * 2 * B * kH, st), "alloc")) ||
          (s = check_hip(dev_malloc_async((void**)&Bf, 4ull * NF * kH, st), "alloc")) ||
          (s = check_hip(dev_malloc_async((void**)&Sh, 4ull * B * NF, st), "alloc")) ||
          (s = check_hip(dev_malloc_async((void**)&mg, 4ull * B, st), "alloc")) ||
          (s = check_hip(dev_malloc_async((void**)&fb, B, st), "alloc")) ||
          (s = check_hip(dev_malloc_async((void**)&ones, 4ull * B, st), "alloc")))
        break;
      fill_words_kernel<<<(B + 255) / 256, 256, 0, st>>>(ones, 1u, B);
    }
    if (n_val &&
        ((s = check_hip(dev_malloc_async((void**)&cand_v, 4ull * n_val * o.K, st), "alloc")) ||
         (s = check_hip(dev_malloc_async((void**)&mg_v, 4ull * n_val, st), "alloc")) ||
         (s = check_hip(dev_malloc_async((void**)&fb_v, n_val, st), "alloc")) ||
         (s = check_hip(dev_malloc_async((void**)&oc, sizeof(maxss_top2) * n_val, st), "alloc"))))
      break;
    const EncodedReads er_val = encoded_tail(er, n_train);
    // held-out recall@K of the current parameters (-1 without held-out reads)
    auto evaluate = [&](float* r) -> maxss_status {
      *r = -1.0f;
      if (!nv_val) return MAXSS_OK;
      maxss_status q;
      if ((q = propose_impl(ix, m, er_val, n_val, o.K, 0.0f, cand_v, mg_v, fb_v, st))) return q;
      fill_words_kernel<<<1, 64, 0, st>>>(hits, 0u, 1u);
      count_hits_kernel<<<(n_val + 255) / 256, 256, 0, st>>>(cand_v, o.K, labels + n_train,
                                                             er_val.lens, n_val, hits);
      uint32_t h = 0;
      if ((q = check_hip(hipGetLastError(), "count_hits_kernel")) ||
          (q = check_hip(hipMemcpyAsync(&h, hits, 4, hipMemcpyDeviceToHost, st), "copy hits")) ||
          (q = check_hip(hipStreamSynchronize(st), "sync")))
        return q;
      *r = (float)h / (float)nv_val;
      return MAXSS_OK;
    };
    float rec = 0;
    if ((s = evaluate(&rec))) break;
    stats->val_recall_init = stats->val_recall_best = rec;
    if ((s = check_hip(hipMemcpyAsync(best, m->master, 4ull * kParams, hipMemcpyDeviceToDevice, st),
                       "copy params")))
      break;
    const uint64_t nkey = sm_key(o.seed, kStreamNeg);
    const uint64_t nvalid = valid.size();
    std::vector<int32_t> order, hb(B);
    uint64_t order_epoch = ~0ull;
    bool evaluated_last = true;
    for (uint32_t t = 0; t < o.steps && !s; t++) {
      for (uint32_t b = 0; b < B; b++) {
        const uint64_t p = (uint64_t)t * B + b, e = p / nvalid;
        if (e != order_epoch) {
          epoch_order(o.seed, e, valid, order);
          order_epoch = e;
        }
        hb[b] = order[p % nvalid];
      }
      if ((s = check_hip(hipMemcpyAsync(bidx, hb.data(), 4ull * B, hipMemcpyHostToDevice, st),
                         "copy batch")))
        break;
      if (hk) {
        // the model's best fragments for the batch reads (both strands)
        batch_rows_kernel<<<(2 * B + 255) / 256, 256, 0, st>>>(bidx, B, rows2);
        Opnd a{rprof, kD, 1, rows2, nullptr};
        Opnd w{m->W1a, kD, 1, nullptr, nullptr};
        if ((s = gemm((int)(2 * B), kH, kD, a, w, Ah, kH, m->master + kW1, false, st))) break;
        if ((s = frag_side(m, m->fprof, NF, Bf, st))) break;
        dim3 grid((NF + 63) / 64, (B + 31) / 32);
        pair_kernel<<<grid, 256, 0, st>>>(Ah, Bf, m->w2f, host_b2(m), B, NF, Sh, NF);
        topk_kernel<<<B, 256, 0, st>>>(Sh, NF, NF, hk, 0.0f, ones, 0, hardc, mg, fb);
        if ((s = check_hip(hipGetLastError(), "hard negatives"))) break;
      }
      negatives_kernel<<<(B + 3) / 4, 256, 0, st>>>(bidx, labels, hk ? hardc : nullptr, hk,
                                                      o.hard_negatives, nkey, t, B, NF, cand, m->rsel);
      if ((s = check_hip(hipGetLastError(), "negatives_kernel"))) break;
      if (o.cand_trace &&
          (s = check_hip(hipMemcpyAsync(o.cand_trace + (uint64_t)t * B * kCand, cand,
                                        4ull * B * kCand, hipMemcpyDeviceToHost, st),
                         "copy candidates")))
        break;
      if ((s = train_step_impl(m, ix, rprof, m->rsel, cand, B, o.lr, trace + t, nullptr, st))) break;
      stats->steps_run = t + 1;
      evaluated_last = false;
      if (o.eval_every && (t + 1) % o.eval_every == 0) {
        if ((s = evaluate(&rec))) break;
        evaluated_last = true;
        if (rec > stats->val_recall_best) {
          stats->val_recall_best = rec;
          stats->best_step = t + 1;
          if ((s = check_hip(hipMemcpyAsync(best, m->master, 4ull * kParams, hipMemcpyDeviceToDevice,
                                            st),
                             "copy params")))
            break;
        }
      }
    }
    if (s) break;
    if (!evaluated_last) {
      if ((s = evaluate(&rec))) break;
      if (rec > stats->val_recall_best) {
        stats->val_recall_best = rec;
        stats->best_step = stats->steps_run;
        if ((s = check_hip(hipMemcpyAsync(best, m->master, 4ull * kParams, hipMemcpyDeviceToDevice, st),
                           "copy params")))
          break;
      }
    }
    if (stats->best_step != stats->steps_run || !nv_val) {
      // keep the parameters of the best held-out recall (the initial ones
      // when no step improved it); without held-out reads, the last ones
      if (nv_val &&
          ((s = check_hip(hipMemcpyAsync(m->master, best, 4ull * kParams, hipMemcpyDeviceToDevice, st),
                          "copy params")) ||
           (s = refresh_shadow(m, st))))
        break;
      if (!nv_val) stats->best_step = stats->steps_run;
    }
    if (o.steps) {
      if ((s = check_hip(hipMemcpyAsync(trace_h.data(), trace, 4ull * o.steps, hipMemcpyDeviceToHost, st),
                         "copy losses")) ||
          (s = check_hip(hipStreamSynchronize(st), "sync")))
        break;
      stats->loss_first = trace_h[0];
      stats->loss_last = trace_h[stats->steps_run ? stats->steps_run - 1 : 0];
      if (o.loss_trace) memcpy(o.loss_trace, trace_h.data(), 4ull * o.steps);
    }
    // thresholds on the held-out reads: the network's margins and the exact
    // best score among the candidates against the full scan's best fragment
    stats->tau = INFINITY;
    stats->min_score = -1;
    if (nv_val) {
      if ((s = propose_impl(ix, m, er_val, n_val, o.K, 0.0f, cand_v, mg_v, fb_v, st))) break;
      if ((s = alloc_scan_work(ix, n_val, (uint64_t)n_val * (Kc < 16 ? Kc : 16), true, st, &wc))) break;
      if ((s = candidate_scan(ix, er_val, er_val.lens, n_val, cand_v, o.K, Kc, oc, wc, st))) break;
      std::vector<float> hm(n_val);
      std::vector<maxss_top2> ho(n_val);
      if ((s = check_hip(hipMemcpyAsync(hm.data(), mg_v, 4ull * n_val, hipMemcpyDeviceToHost, st),
                         "copy margins")) ||
          (s = check_hip(hipMemcpyAsync(ho.data(), oc, sizeof(maxss_top2) * n_val, hipMemcpyDeviceToHost,
                                        st),
                         "copy records")) ||
          (s = check_hip(hipStreamSynchronize(st), "sync")))
        break;
      std::vector<float> vm;
      std::vector<int32_t> vs;
      std::vector<uint8_t> vc;
      for (uint32_t j = 0; j < n_val; j++) {
        if (!labelled(n_train + j)) continue;
        vm.push_back(hm[j]);
        vs.push_back(ho[j].frag[0] >= 0 ? ho[j].score[0] : -1);
        vc.push_back(ho[j].frag[0] == hl[n_train + j].frag[0] ? 1 : 0);
      }
      if ((s = maxss_choose_acceptance((uint32_t)vm.size(), vm.data(), vs.data(), vc.data(),
                                       o.target_agreement, &stats->tau, &stats->min_score,
                                       &stats->val_accept, &stats->val_agreement)))
        break;
    }
  } while (0);
  void* ps[] = {rprof, bidx, cand, trace, best, hits, rows2, hardc, Ah, Bf, Sh, mg, fb, ones,
                cand_v, mg_v, fb_v, oc};
  for (void* p : ps)
    if (p) (void)hipFreeAsync(p, st);
  release_scan_work(&wc, true, st);
  release_encoded(&er, st);
  const maxss_status s2 = check_hip(hipStreamSynchronize(st), "sync");
  return s ? s : s2;
}
