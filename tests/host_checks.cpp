// Host-only entry points of libmaxss (SAM formatting, MAPQ argument checks,
// index parameter validation, error text) driven with edge-case inputs.  The
// test builds this with the library's index and report sources under the
// host address and undefined-behaviour sanitizers; it needs no GPU.
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "maxss.h"

static int bad = 0;
#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      bad++;                                                  \
    }                                                         \
  } while (0)

int main() {
  // four reads: mapped forward, mapped reverse with a truncated CIGAR,
  // unmapped, invalid; all with qualities
  const char* seq = "ACGTACGTAAcgtacgNNACGTTTTT";
  uint64_t off[5] = {0, 8, 16, 20, 26};
  const char* qual = "IIIIIIII#####!!!~~~~ABCDEF";
  maxss_reads r{};
  r.seq = seq; r.offsets = off; r.n = 4; r.on_device = 0; r.qual = qual;
  maxss_top2 top[4];
  memset(top, 0, sizeof top);
  top[0].frag[0] = 1; top[0].score[0] = 8; top[0].frag[1] = 3; top[0].score[1] = 2;
  top[1].frag[0] = 2; top[1].score[0] = 7; top[1].frag[1] = -1; top[1].score[1] = -1;
  top[2].frag[0] = 0; top[2].score[0] = 4; top[2].frag[1] = 1; top[2].score[1] = 4;
  top[3].frag[0] = MAXSS_READ_INVALID;
  maxss_aln aln[4];
  memset(aln, 0, sizeof aln);
  aln[0].score = 8;
  aln[1].strand = 1; aln[1].ref_begin = 99; aln[1].flags = MAXSS_ALN_TRUNCATED;
  std::vector<char> cig(4 * 8, 0);
  memcpy(&cig[0], "8=", 2);
  memcpy(&cig[8], "12345678", 8);  // a full row without its NUL
  uint8_t mq[4] = {60, 254, 0, 0}, mp[4] = {1, 1, 0, 0};
  const char* names[4] = {"a", "b", "c", "d"};
  uint64_t len = 0;
  CHECK(maxss_sam_records(&r, top, aln, cig.data(), 8, mq, mp, "chr", names, nullptr, 0, &len) ==
        MAXSS_EINVAL);
  std::vector<char> buf(len);
  CHECK(maxss_sam_records(&r, top, aln, cig.data(), 8, mq, mp, "chr", names, buf.data(), len,
                          &len) == MAXSS_OK);
  const std::string want =
      "a\t0\tchr\t1\t60\t8=\t*\t0\t0\tACGTACGT\tIIIIIIII\tAS:i:8\n"
      "b\t16\tchr\t100\t254\t*\t*\t0\t0\tCGTACGTT\t!!!#####\tAS:i:0\n"
      "c\t4\t*\t0\t0\t*\t*\t0\t0\tNNAC\t~~~~\n"
      "d\t4\t*\t0\t0\t*\t*\t0\t0\t*\t*\n";
  CHECK(std::string(buf.data(), len) == want);
  std::vector<char> small(len - 1);
  CHECK(maxss_sam_records(&r, top, aln, cig.data(), 8, mq, mp, "chr", names, small.data(),
                          len - 1, &len) == MAXSS_EINVAL);
  const char* badq = "IIIIIIII#####!!!~~~~ABC EF";
  r.qual = badq;
  CHECK(maxss_sam_records(&r, top, aln, cig.data(), 8, mq, mp, "chr", names, buf.data(),
                          buf.size(), &len) == MAXSS_EINVAL);
  // without qualities QUAL is "*"; default names r<i>
  r.qual = nullptr;
  CHECK(maxss_sam_records(&r, top, aln, cig.data(), 8, mq, mp, "chr", nullptr, buf.data(),
                          buf.size(), &len) == MAXSS_OK);
  const std::string first = "r0\t0\tchr\t1\t60\t8=\t*\t0\t0\tACGTACGT\t*\tAS:i:8\n";
  CHECK(std::string(buf.data(), len).compare(0, first.size(), first) == 0);
  r.qual = qual;
  const char* badn[4] = {"a", "b c", "c", "d"};
  CHECK(maxss_sam_records(&r, top, aln, cig.data(), 8, mq, mp, "chr", badn, buf.data(),
                          buf.size(), &len) == MAXSS_EINVAL);
  CHECK(maxss_sam_records(&r, top, aln, cig.data(), 8, mq, mp, "c h", names, buf.data(),
                          buf.size(), &len) == MAXSS_EINVAL);
  CHECK(maxss_sam_records(nullptr, top, aln, cig.data(), 8, mq, mp, "chr", names, buf.data(),
                          buf.size(), &len) == MAXSS_EINVAL);
  uint64_t dec[3] = {0, 5, 3};
  maxss_reads rd{};
  rd.seq = seq; rd.offsets = dec; rd.n = 2;
  CHECK(maxss_sam_records(&rd, top, aln, cig.data(), 8, mq, mp, "chr", names, buf.data(),
                          buf.size(), &len) == MAXSS_EINVAL);
  CHECK(maxss_sam_header(nullptr, "chr", buf.data(), buf.size(), &len) == MAXSS_EINVAL);
  // MAPQ: nothing to do for n = 0; bad ratio
  CHECK(maxss_mapq(nullptr, 0, 9, 10, -1, nullptr, nullptr, nullptr) == MAXSS_OK);
  CHECK(maxss_mapq(top, 4, 9, 0, -1, mq, mp, nullptr) == MAXSS_EINVAL);
  // index parameters rejected before any device call
  maxss_params p{};
  p.match = 1; p.mismatch = -1; p.gap = -2; p.frag_len = 40; p.max_read_len = 100;
  maxss_index* ix = nullptr;
  CHECK(maxss_index_genome("ACGT", 4, &p, &ix) == MAXSS_EINVAL);
  p.frag_len = 64; p.flags = 64;
  CHECK(maxss_index_genome("ACGT", 4, &p, &ix) == MAXSS_EINVAL);
  p.flags = MAXSS_EXCLUDE_ADJACENT; p.qual_scale = 1000;
  CHECK(maxss_index_genome("ACGT", 4, &p, &ix) == MAXSS_EINVAL);
  p.qual_scale = 0; p.max_read_len = 9000;
  CHECK(maxss_index_genome("ACGT", 4, &p, &ix) == MAXSS_EINVAL);
  p.max_read_len = 100;
  CHECK(maxss_index_genome("ACGU", 4, &p, &ix) == MAXSS_EINVAL);
  CHECK(strstr(maxss_last_error(), "0x55") != nullptr);
  CHECK(maxss_index_genome(nullptr, 4, &p, &ix) == MAXSS_EINVAL);
  CHECK(ix == nullptr);
  printf("host checks: %s\n", bad ? "FAIL" : "ok");
  return bad;
}
