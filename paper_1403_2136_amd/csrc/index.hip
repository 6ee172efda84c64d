// Genome index, read staging and read encoding (HIP, gfx950).
//
// The genome is cut into NF = ceil(G/F) disjoint fragments of F bases; the
// last one, and everything past the genome end, is padded with N (Methods,
// "Coalescent global memory access" and Figure 2; "Byte packing for faster
// global memory access").  On the device the genome is kept 2-bit packed with
// a separate N mask (the scan stages it into LDS) and as one code byte per
// position (the second phase and the winners' re-scan read it).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace maxss {

static thread_local std::string g_err;

maxss_status fail(maxss_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

void clear_error() { g_err.clear(); }

maxss_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return MAXSS_OK;
  if (e == hipErrorOutOfMemory)
    return fail(MAXSS_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(MAXSS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Countdown of maxss_fail_alloc_after: the allocation that brings it from 1
// to 0 fails; 0 = off.
static std::atomic<uint32_t> g_fail_alloc{0};

static bool alloc_should_fail() {
  uint32_t v = g_fail_alloc.load();
  while (v != 0) {
    if (g_fail_alloc.compare_exchange_weak(v, v - 1)) return v == 1;
  }
  return false;
}

hipError_t dev_malloc(void** p, size_t bytes) {
  if (alloc_should_fail()) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

hipError_t dev_malloc_async(void** p, size_t bytes, hipStream_t st) {
  if (alloc_should_fail()) return hipErrorOutOfMemory;
  return hipMallocAsync(p, bytes, st);
}

uint8_t host_code(char c) {
  switch (c) {
    case 'A': case 'a': return kA;
    case 'C': case 'c': return kC;
    case 'G': case 'g': return kG;
    case 'T': case 't': return kT;
    case 'N': case 'n': return kN;
    default: return 0xFF;
  }
}

maxss_status validate_host_reads(const Index* ix, const maxss_reads* r) {
  for (uint32_t i = 0; i < r->n; i++) {
    uint64_t a = r->offsets[i], b = r->offsets[i + 1];
    if (b <= a) return fail(MAXSS_ETOOLONG, "read %u is empty", i);
    if (b - a > ix->p.max_read_len)
      return fail(MAXSS_ETOOLONG, "read %u has length %llu > max_read_len %u", i,
                  (unsigned long long)(b - a), ix->p.max_read_len);
    for (uint64_t k = a; k < b; k++)
      if (host_code(r->seq[k]) == 0xFF)
        return fail(MAXSS_EINVAL, "read %u: invalid character 0x%02x at %llu", i,
                    (unsigned)(unsigned char)r->seq[k], (unsigned long long)(k - a));
    if (qual_mode(ix) && r->qual)
      for (uint64_t k = a; k < b; k++) {
        const int c = (unsigned char)r->qual[k];
        if (c < 33 || c > 126)
          return fail(MAXSS_EINVAL, "read %u: quality 0x%02x at %llu outside '!'..'~'", i,
                      (unsigned)c, (unsigned long long)(k - a));
      }
  }
  return MAXSS_OK;
}

maxss_status require_quals(const Index* ix, const maxss_reads* r) {
  if (qual_mode(ix) && r->n && !r->qual)
    return fail(MAXSS_EINVAL, "the index scores with base qualities: reads need `qual`");
  return MAXSS_OK;
}

maxss_status stage_reads(const maxss_reads* r, hipStream_t st, DeviceReads* d) {
  d->n = r->n;
  if (r->on_device) {
    d->seq = r->seq;
    d->off = r->offsets;
    d->qual = r->qual;
    return MAXSS_OK;
  }
  uint64_t a = r->offsets[0], b = r->offsets[r->n];
  uint64_t bytes = b - a;
  maxss_status s;
  if ((s = check_hip(dev_malloc_async((void**)&d->own_seq, bytes ? bytes : 1, st),
                     "hipMallocAsync(reads)")))
    return s;
  if ((s = check_hip(dev_malloc_async((void**)&d->own_off, sizeof(uint64_t) * (r->n + 1), st),
                     "hipMallocAsync(offsets)")))
    return s;
  std::vector<uint64_t> off(r->n + 1);
  for (uint32_t i = 0; i <= r->n; i++) off[i] = r->offsets[i] - a;
  if ((s = check_hip(hipMemcpyAsync(d->own_seq, r->seq + a, bytes, hipMemcpyHostToDevice, st),
                     "copy reads")))
    return s;
  if ((s = check_hip(hipMemcpyAsync(d->own_off, off.data(), sizeof(uint64_t) * (r->n + 1),
                                    hipMemcpyHostToDevice, st),
                     "copy offsets")))
    return s;
  if (r->qual) {
    if ((s = check_hip(dev_malloc_async((void**)&d->own_qual, bytes ? bytes : 1, st),
                       "hipMallocAsync(qualities)")) ||
        (s = check_hip(hipMemcpyAsync(d->own_qual, r->qual + a, bytes, hipMemcpyHostToDevice, st),
                       "copy qualities")))
      return s;
    d->qual = d->own_qual;
  }
  // the host vector dies at return: make the copy complete first
  if ((s = check_hip(hipStreamSynchronize(st), "sync after read upload"))) return s;
  d->seq = d->own_seq;
  d->off = d->own_off;
  return MAXSS_OK;
}

void release_reads(DeviceReads* d, hipStream_t st) {
  if (d->own_seq) (void)hipFreeAsync(d->own_seq, st);
  if (d->own_off) (void)hipFreeAsync(d->own_off, st);
  if (d->own_qual) (void)hipFreeAsync(d->own_qual, st);
  d->own_seq = nullptr;
  d->own_off = nullptr;
  d->own_qual = nullptr;
}

// ----------------------------------------------------------- kernel timing

struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static std::vector<ProfRec> g_prof;
static std::atomic<int> g_prof_on{0};

bool stream_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
  return cs != hipStreamCaptureStatusNone;
}

ProfScope::ProfScope(const char* n, hipStream_t s) : name(n), st(s) {
  if (!g_prof_on.load() || stream_capturing(st)) return;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    a = b = nullptr;
    return;
  }
  (void)hipEventRecord(a, st);
}

ProfScope::~ProfScope() {
  if (!a) return;
  (void)hipEventRecord(b, st);
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof.push_back(ProfRec{name, a, b});
}

// ------------------------------------------------------------ read encoding

__device__ inline uint8_t dev_code(char c) {
  switch (c) {
    case 'A': case 'a': return kA;
    case 'C': case 'c': return kC;
    case 'G': case 'g': return kG;
    case 'T': case 't': return kT;
    case 'N': case 'n': return kN;
    default: return 0xFF;
  }
}

// Pool-shift code of a read base: which byte of the scan's 8-byte score pool
// holds the score against the genome base equal to it (A 1, C 3, G 5, T 7);
// N gets byte 4, which no genome selector reads, so it mismatches everything.
__device__ inline uint32_t pool_shift_code(uint8_t q) { return q == kN ? 4u : 2u * q + 1u; }

// One wave per read: validity (length and characters), forward base codes,
// and the 4-bit pool-shift codes of both strands for positions [0, mstride)
// (N past the end).
__global__ __launch_bounds__(256) void encode_reads_kernel(
    const char* __restrict__ seq, const uint64_t* __restrict__ off, uint32_t n,
    uint32_t max_len, uint32_t mstride, uint32_t step, uint32_t* __restrict__ sel4,
    uint8_t* __restrict__ codes, uint32_t* __restrict__ lens, const char* __restrict__ qual,
    QualTable qt, uint16_t* __restrict__ qsc) {
  const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint32_t lane = threadIdx.x & 63;
  if (wave >= n) return;
  const uint64_t a = off[wave], b = off[wave + 1];
  const uint64_t len64 = b > a ? b - a : 0;
  bool ok = len64 >= 1 && len64 <= max_len;
  const uint32_t m = ok ? (uint32_t)len64 : 0;
  bool bad = false;
  for (uint32_t k = lane; k < m; k += 64) bad |= dev_code(seq[a + k]) == 0xFF;
  if (qsc)
    for (uint32_t k = lane; k < m; k += 64) {
      const int c = (unsigned char)qual[a + k];
      bad |= c < 33 || c > 126;
    }
  ok = ok && !__any(bad);
  if (qsc) {
    // per position: (match, mismatch) of its quality, in read order
    uint16_t* qr = qsc + (uint64_t)wave * mstride;
    for (uint32_t k = lane; k < mstride; k += 64) {
      uint16_t v = 0;
      if (ok && k < m) {
        const int q = (unsigned char)qual[a + k] - 33;
        v = (uint16_t)((uint8_t)qt.sm[q] | ((uint16_t)(uint8_t)qt.sx[q] << 8));
      }
      qr[k] = v;
    }
  }
  const uint32_t nw = mstride / 8;
  uint32_t* sf = sel4 + (uint64_t)wave * 2 * nw;
  uint32_t* sr = sf + nw;
  uint8_t* cf = codes + (uint64_t)wave * mstride;
  for (uint32_t w = lane; w < nw; w += 64) {
    uint32_t wf = 0, wr = 0;
    for (uint32_t t = 0; t < 8; t++) {
      const uint32_t k = 8 * w + t;
      // the read as given (second phase, re-scan)
      cf[k] = (ok && k < m) ? dev_code(seq[a + k]) : kN;
      // first-phase codes: position step*k of each strand (every other
      // base with step 2)
      const uint32_t kk = step * k;
      uint8_t qf = kN, qr = kN;
      if (ok && kk < m) {
        qf = dev_code(seq[a + kk]);
        const uint8_t c = dev_code(seq[a + (m - 1 - kk)]);
        qr = c == kN ? kN : (uint8_t)(3 - c);  // complement: A<->T, C<->G
      }
      wf |= pool_shift_code(qf) << (4 * t);
      wr |= pool_shift_code(qr) << (4 * t);
    }
    sf[w] = wf;
    sr[w] = wr;
  }
  if (lane == 0) lens[wave] = ok ? m : 0;
}

static constexpr uint32_t kSlack = 64;

maxss_status alloc_encoded(const Index* ix, uint32_t n, hipStream_t st, EncodedReads* e) {
  e->mstride = read_stride(ix);
  maxss_status s;
  if (qual_mode(ix) &&
      (s = check_hip(dev_malloc_async((void**)&e->qsc, sizeof(uint16_t) * ((uint64_t)n * e->mstride +
                                                                         kSlack), st),
                     "hipMallocAsync(position scores)")))
    return s;
  if ((s = check_hip(dev_malloc_async((void**)&e->sel4,
                                    sizeof(uint32_t) * ((uint64_t)n * 2 * (e->mstride / 8) + kSlack),
                                    st),
                     "hipMallocAsync(read codes)")))
    return s;
  if ((s = check_hip(dev_malloc_async((void**)&e->codes, (uint64_t)n * e->mstride + kSlack, st),
                     "hipMallocAsync(read bases)")))
    return s;
  return check_hip(dev_malloc_async((void**)&e->lens, sizeof(uint32_t) * ((uint64_t)n + 1), st),
                   "hipMallocAsync(lens)");
}

maxss_status encode_reads_into(const Index* ix, const DeviceReads& r, hipStream_t st,
                               const EncodedReads& e) {
  const uint64_t n = r.n;
  const uint32_t blocks = (uint32_t)((n * 64 + 255) / 256);
  ProfScope prof("encode", st);
  const uint32_t step = (ix->p.flags & MAXSS_FAST) ? 2u : 1u;
  QualTable qt;
  memcpy(qt.sm, ix->qsm, sizeof(qt.sm));
  memcpy(qt.sx, ix->qsx, sizeof(qt.sx));
  // position scores only where both the buffer and the qualities exist (a
  // proposal-only call encodes reads without qualities)
  uint16_t* qsc = (qual_mode(ix) && r.qual) ? e.qsc : nullptr;
  encode_reads_kernel<<<blocks, 256, 0, st>>>(r.seq, r.off, r.n, ix->p.max_read_len, e.mstride,
                                              step, e.sel4, e.codes, e.lens, r.qual, qt, qsc);
  return check_hip(hipGetLastError(), "encode_reads_kernel");
}

void release_encoded(EncodedReads* e, hipStream_t st) {
  if (e->sel4) (void)hipFreeAsync(e->sel4, st);
  if (e->codes) (void)hipFreeAsync(e->codes, st);
  if (e->lens) (void)hipFreeAsync(e->lens, st);
  if (e->qsc) (void)hipFreeAsync(e->qsc, st);
  e->sel4 = nullptr;
  e->codes = nullptr;
  e->lens = nullptr;
  e->qsc = nullptr;
}

}  // namespace maxss

using namespace maxss;

extern "C" maxss_status maxss_index_genome(const char* seq, uint64_t len,
                                           const maxss_params* params, maxss_index** out) {
  clear_error();
  if (!seq || !params || !out) return fail(MAXSS_EINVAL, "NULL argument");
  const maxss_params& p = *params;
  if (len == 0) return fail(MAXSS_EINVAL, "empty genome");
  if (p.frag_len == 0 || p.frag_len % 16 != 0)
    return fail(MAXSS_EINVAL, "frag_len %u must be a positive multiple of 16", p.frag_len);
  if (p.match < 1 || p.match > 127) return fail(MAXSS_EINVAL, "match %d not in 1..127", p.match);
  if (p.mismatch < -127 || p.mismatch > 0)
    return fail(MAXSS_EINVAL, "mismatch %d not in -127..0", p.mismatch);
  if (p.gap < -1000000 || p.gap > 0) return fail(MAXSS_EINVAL, "gap %d not in -1e6..0", p.gap);
  if (p.max_read_len < 1 || p.max_read_len > 8192)
    return fail(MAXSS_EINVAL, "max_read_len %u not in 1..8192", p.max_read_len);
  if ((uint64_t)p.max_read_len * (uint64_t)p.match > 65535u)
    return fail(MAXSS_EINVAL, "max_read_len * match = %llu exceeds 65535",
                (unsigned long long)p.max_read_len * p.match);
  if (p.flags & ~(MAXSS_ONE_STRAND | MAXSS_NW_GLOBAL | MAXSS_FAST | MAXSS_EXCLUDE_ADJACENT))
    return fail(MAXSS_EINVAL, "unknown flags 0x%x", p.flags);
  if (p.qual_scale > 0) {
    // every position score must fit the scan's int8 score pool, and a whole
    // read its 16-bit exact range
    if ((int64_t)p.match * p.qual_scale > 127 || -(int64_t)p.mismatch * p.qual_scale > 381)
      return fail(MAXSS_EINVAL, "match*qual_scale <= 127 and -mismatch*qual_scale <= 381 needed");
    if ((uint64_t)p.max_read_len * (uint64_t)p.match * p.qual_scale > 65535u)
      return fail(MAXSS_EINVAL, "max_read_len * match * qual_scale exceeds 65535");
    if ((int64_t)p.gap * p.qual_scale < -1000000000ll)
      return fail(MAXSS_EINVAL, "gap * qual_scale too large");
  }
  const uint64_t F = p.frag_len;
  const uint64_t NF64 = (len + F - 1) / F;
  if (NF64 >= (1ull << 31) || F >= (1u << 30))
    return fail(MAXSS_EINVAL, "genome too large for 31-bit fragment ids");
  for (uint64_t i = 0; i < len; i++)
    if (host_code(seq[i]) == 0xFF)
      return fail(MAXSS_EINVAL, "genome: invalid character 0x%02x at %llu",
                  (unsigned)(unsigned char)seq[i], (unsigned long long)i);

  Index* ix = new (std::nothrow) Index();
  if (!ix) return fail(MAXSS_ENOMEM, "host allocation");
  ix->G = len;
  ix->F = (uint32_t)F;
  ix->NF = (uint32_t)NF64;
  ix->p = p;
  if (p.qual_scale > 0)
    for (int q = 0; q < 94; q++) {
      // x = 1 - 10^(-q/10), the probability that the base is right
      const double x = 1.0 - pow(10.0, -(double)q / 10.0);
      ix->qsm[q] = (int8_t)lround((double)p.match * x * (double)p.qual_scale);
      ix->qsx[q] = (int8_t)lround((double)p.mismatch * x * (double)p.qual_scale / 3.0);
    }
  // Room past the last fragment: a full window (max_read_len-1), the widest
  // scan tile's second half and staging tail, and the NW padding.
  uint64_t tail = 2ull * 128 * 32 + ((p.max_read_len + 63u) & ~63u) + 1024;
  ix->Lpad = ((NF64 * F + tail) + 31) & ~31ull;
  maxss_status s;
  if ((s = check_hip(hipGetDevice(&ix->device), "hipGetDevice"))) { delete ix; return s; }
  if ((s = check_hip(hipDeviceGetAttribute(&ix->num_cu, hipDeviceAttributeMultiprocessorCount,
                                           ix->device),
                     "hipDeviceGetAttribute"))) {
    delete ix;
    return s;
  }
  int lds_cu = 0;
  if ((s = check_hip(hipDeviceGetAttribute(&lds_cu,
                                           hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                           ix->device),
                     "hipDeviceGetAttribute"))) {
    delete ix;
    return s;
  }
  ix->lds_per_cu = lds_cu > 0 ? (size_t)lds_cu : 0;
  std::vector<uint32_t> g2(ix->Lpad / 16, 0), nm(ix->Lpad / 32, 0);
  std::vector<uint8_t> codes(ix->Lpad, kN);
  for (uint64_t i = 0; i < ix->Lpad; i++) {
    uint8_t c = i < len ? host_code(seq[i]) : (uint8_t)kN;
    codes[i] = c;
    if (c == kN)
      nm[i >> 5] |= 1u << (i & 31);
    else
      g2[i >> 4] |= (uint32_t)c << (2 * (i & 15));
  }
  if ((s = check_hip(dev_malloc((void**)&ix->g2, g2.size() * 4), "hipMalloc(genome)")) ||
      (s = check_hip(dev_malloc((void**)&ix->nmask, nm.size() * 4), "hipMalloc(N mask)")) ||
      (s = check_hip(dev_malloc((void**)&ix->codes, codes.size()), "hipMalloc(codes)")) ||
      (s = check_hip(hipMemcpy(ix->g2, g2.data(), g2.size() * 4, hipMemcpyHostToDevice),
                     "copy genome")) ||
      (s = check_hip(hipMemcpy(ix->nmask, nm.data(), nm.size() * 4, hipMemcpyHostToDevice),
                     "copy N mask")) ||
      (s = check_hip(hipMemcpy(ix->codes, codes.data(), codes.size(), hipMemcpyHostToDevice),
                     "copy codes"))) {
    maxss_index_free(reinterpret_cast<maxss_index*>(ix));
    return s;
  }
  *out = reinterpret_cast<maxss_index*>(ix);
  return MAXSS_OK;
}

extern "C" void maxss_index_free(maxss_index* index) {
  Index* ix = reinterpret_cast<Index*>(index);
  if (!ix) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(ix->device);
  if (ix->g2) (void)hipFree(ix->g2);
  if (ix->nmask) (void)hipFree(ix->nmask);
  if (ix->codes) (void)hipFree(ix->codes);
  (void)hipSetDevice(cur);
  delete ix;
}

extern "C" maxss_status maxss_index_info(const maxss_index* index, uint64_t* genome_len,
                                         uint32_t* num_fragments, uint32_t* frag_len) {
  clear_error();
  const Index* ix = reinterpret_cast<const Index*>(index);
  if (!ix) return fail(MAXSS_EINVAL, "NULL index");
  if (genome_len) *genome_len = ix->G;
  if (num_fragments) *num_fragments = ix->NF;
  if (frag_len) *frag_len = ix->F;
  return MAXSS_OK;
}

extern "C" maxss_status maxss_profile_enable(int on) {
  clear_error();
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (auto& r : g_prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.clear();
  g_prof_on.store(on ? 1 : 0);
  return MAXSS_OK;
}

extern "C" maxss_status maxss_profile_read(const char* name, double* total_ms,
                                           uint32_t* launches) {
  clear_error();
  if (!name || !total_ms || !launches) return fail(MAXSS_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(g_prof_mu);
  double t = 0;
  uint32_t k = 0;
  for (auto& r : g_prof) {
    if (r.name != name) continue;
    maxss_status s;
    if ((s = check_hip(hipEventSynchronize(r.b), "hipEventSynchronize"))) return s;
    float ms = 0;
    if ((s = check_hip(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime"))) return s;
    t += ms;
    k++;
  }
  *total_ms = t;
  *launches = k;
  return MAXSS_OK;
}

extern "C" const char* maxss_last_error(void) { return g_err.c_str(); }

extern "C" const char* maxss_version(void) { return "maxss-gfx950 0.1"; }

extern "C" maxss_status maxss_fail_alloc_after(uint32_t n) {
  clear_error();
  g_fail_alloc.store(n);
  return MAXSS_OK;
}
