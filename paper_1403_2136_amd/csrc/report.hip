// Mapping quality and SAM records (Methods, paragraph on mapping qualities,
// read lengths, SAM output and source code).
//
// MAPQ = -100 log2 p with p = second-best / best fragment score, as the
// integer part, capped at 254 (SAM keeps 255 for "unavailable"); no second
// fragment or a second score of 0 gives the cap, a best score of 0 gives 0.
// A read is mapped when the ratio is below num/den (0.9 in the first-phase
// paragraph), decided exactly in integers, and its MAPQ exceeds min_mapq
// (62 for the ancient-DNA runs of the Results).  The MAPQ kernel runs on
// the device next to the scan's records; SAM text is formatted on the host.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "internal.h"

namespace maxss {

constexpr int kMapqCap = 254;

__global__ void mapq_kernel(const maxss_top2* __restrict__ top, uint32_t n, uint32_t num,
                            uint32_t den, int32_t min_mapq, uint8_t* __restrict__ mapq,
                            uint8_t* __restrict__ mapped) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const maxss_top2 t = top[i];
  int q = 0;
  bool ok = false;
  if (t.frag[0] >= 0 && t.score[0] > 0) {
    const int s1 = t.score[0];
    const int s2 = t.frag[1] >= 0 ? t.score[1] : -1;
    if (s2 <= 0) {
      q = kMapqCap;
    } else {
      const double v = floor(-100.0 * log2((double)s2 / (double)s1));
      q = v < 0.0 ? 0 : (v > (double)kMapqCap ? kMapqCap : (int)v);
    }
    ok = (uint64_t)(s2 > 0 ? s2 : 0) * den < (uint64_t)s1 * num && q > min_mapq;
  }
  mapq[i] = (uint8_t)q;
  if (mapped) mapped[i] = ok ? 1 : 0;
}

static void put_rc(std::string& out, const char* s, uint64_t m) {
  for (uint64_t k = m; k-- > 0;) {
    switch (s[k] & 0xDF) {
      case 'A': out.push_back('T'); break;
      case 'C': out.push_back('G'); break;
      case 'G': out.push_back('C'); break;
      case 'T': out.push_back('A'); break;
      default: out.push_back('N'); break;
    }
  }
}

static void put_upper(std::string& out, const char* s, uint64_t m) {
  for (uint64_t k = 0; k < m; k++) {
    const char c = s[k];
    out.push_back(c >= 'a' && c <= 'z' ? (char)(c - 32) : c);
  }
}

// QUAL of a read: the Phred+33 string as given, or reversed for a record on
// the reverse strand (SAM stores QUAL in the order of SEQ); "*" without
// qualities.
static void put_qual(std::string& out, const char* q, uint64_t m, bool reverse) {
  if (!q || m == 0) {
    out.push_back('*');
  } else if (reverse) {
    for (uint64_t k = m; k-- > 0;) out.push_back(q[k]);
  } else {
    out.append(q, m);
  }
}

static bool valid_name(const char* s) {
  if (!s || !*s) return false;
  for (const char* p = s; *p; p++)
    if (*p < '!' || *p > '~' || *p == '\t') return false;
  return true;
}

}  // namespace maxss

using namespace maxss;

extern "C" maxss_status maxss_mapq(const maxss_top2* top, uint32_t n, uint32_t ratio_num,
                                   uint32_t ratio_den, int32_t min_mapq, uint8_t* mapq,
                                   uint8_t* mapped, void* stream) {
  clear_error();
  if (n == 0) return MAXSS_OK;
  if (!top || !mapq) return fail(MAXSS_EINVAL, "NULL argument");
  if (ratio_den == 0) return fail(MAXSS_EINVAL, "ratio_den must be > 0");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  mapq_kernel<<<(n + 255) / 256, 256, 0, st>>>(top, n, ratio_num, ratio_den, min_mapq, mapq,
                                               mapped);
  return check_hip(hipGetLastError(), "mapq_kernel");
}

extern "C" maxss_status maxss_sam_header(const maxss_index* index, const char* rname, char* buf,
                                         uint64_t cap, uint64_t* len) {
  clear_error();
  const Index* ix = reinterpret_cast<const Index*>(index);
  if (!ix || !len) return fail(MAXSS_EINVAL, "NULL argument");
  if (!valid_name(rname)) return fail(MAXSS_EINVAL, "reference name must be printable, no spaces");
  std::string h = "@HD\tVN:1.6\tSO:unsorted\n@SQ\tSN:";
  h += rname;
  h += "\tLN:" + std::to_string((unsigned long long)ix->G) + "\n@PG\tID:maxss\tPN:maxss\n";
  *len = h.size();
  if (!buf || cap < h.size()) return fail(MAXSS_EINVAL, "buffer holds %llu bytes, %llu needed",
                                          (unsigned long long)cap,
                                          (unsigned long long)h.size());
  memcpy(buf, h.data(), h.size());
  return MAXSS_OK;
}

extern "C" maxss_status maxss_sam_records(const maxss_reads* reads, const maxss_top2* top,
                                          const maxss_aln* aln, const char* cigar,
                                          uint64_t cigar_stride, const uint8_t* mapq,
                                          const uint8_t* mapped, const char* rname,
                                          const char* const* names, char* buf, uint64_t cap,
                                          uint64_t* len) {
  clear_error();
  if (!reads || !len) return fail(MAXSS_EINVAL, "NULL argument");
  if (reads->on_device) return fail(MAXSS_EINVAL, "SAM records take host reads");
  const uint32_t n = reads->n;
  if (n && (!reads->seq || !reads->offsets || !top || !aln || !mapq || !mapped))
    return fail(MAXSS_EINVAL, "NULL argument");
  if (n && (!cigar || cigar_stride < 2)) return fail(MAXSS_EINVAL, "CIGAR buffer missing");
  if (!valid_name(rname)) return fail(MAXSS_EINVAL, "reference name must be printable, no spaces");
  std::string out;
  out.reserve((size_t)n * 64);
  for (uint32_t i = 0; i < n; i++) {
    const uint64_t a = reads->offsets[i], b = reads->offsets[i + 1];
    if (b < a) return fail(MAXSS_EINVAL, "offsets decrease at read %u", i);
    const char* s = reads->seq + a;
    const uint64_t m = b - a;
    const char* q = reads->qual ? reads->qual + a : nullptr;
    if (q)
      for (uint64_t k = 0; k < m; k++)
        if (q[k] < '!' || q[k] > '~')
          return fail(MAXSS_EINVAL, "read %u: quality 0x%02x at %llu outside '!'..'~'", i,
                      (unsigned)(unsigned char)q[k], (unsigned long long)k);
    if (names) {
      if (!valid_name(names[i])) return fail(MAXSS_EINVAL, "read name %u is not printable", i);
      out += names[i];
    } else {
      out += "r" + std::to_string(i);
    }
    if (top[i].frag[0] < 0) {  // read marked invalid by the scan
      out += "\t4\t*\t0\t0\t*\t*\t0\t0\t*\t*\n";
      continue;
    }
    if (!mapped[i]) {
      out += "\t4\t*\t0\t0\t*\t*\t0\t0\t";
      put_upper(out, s, m);
      out += "\t";
      put_qual(out, q, m, false);
      out += "\n";
      continue;
    }
    const maxss_aln& al = aln[i];
    out += al.strand ? "\t16\t" : "\t0\t";
    out += rname;
    out += "\t" + std::to_string((long long)al.ref_begin + 1) + "\t" + std::to_string(mapq[i]) +
           "\t";
    if (al.flags & MAXSS_ALN_TRUNCATED) {
      out += "*";
    } else {
      const char* c = cigar + (uint64_t)i * cigar_stride;
      out.append(c, strnlen(c, cigar_stride));
    }
    out += "\t*\t0\t0\t";
    if (al.strand) put_rc(out, s, m);
    else put_upper(out, s, m);
    out += "\t";
    put_qual(out, q, m, al.strand != 0);
    out += "\tAS:i:" + std::to_string(al.score) + "\n";
  }
  *len = out.size();
  if (!buf || cap < out.size())
    return fail(MAXSS_EINVAL, "buffer holds %llu bytes, %llu needed", (unsigned long long)cap,
                (unsigned long long)out.size());
  memcpy(buf, out.data(), out.size());
  return MAXSS_OK;
}
