// Internal declarations of libmaxss (HIP, gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/maxss.h"

namespace maxss {

// Base codes used on the device: A C G T, and N (also the padding).
enum : uint8_t { kA = 0, kC = 1, kG = 2, kT = 3, kN = 4 };

// Genome index (library-owned, immutable after maxss_index_genome).
//   g2    : 2-bit base codes, 16 per 32-bit word (base p at bits 2*(p%16)).
//   nmask : 1 bit per position (p%32 of word p/32), set where the base is N.
//   codes : 1 byte per position (kA..kN), used by the second phase and by the
//           exact re-scan of the two winning fragments.
// All three cover positions [0, Lpad); positions >= G are N.  Lpad leaves room
// for the longest window of the last fragment plus every tile's staging tail.
struct Index {
  int device = 0;
  int num_cu = 0;
  uint64_t G = 0;
  uint32_t F = 0, NF = 0;
  maxss_params p{};
  uint64_t Lpad = 0;
  uint32_t* g2 = nullptr;
  uint32_t* nmask = nullptr;
  uint8_t* codes = nullptr;
};

// Thread-local error message + status helper.
maxss_status fail(maxss_status st, const char* fmt, ...);
void clear_error();

// Returns MAXSS_EDEVICE (and records the message) when e != hipSuccess.
maxss_status check_hip(hipError_t e, const char* what);

// Host-side ASCII -> code, 0xFF for a character outside ACGTN/acgtn.
uint8_t host_code(char c);

// Padded read-profile stride (positions per read per strand) for an index.
inline uint32_t read_stride(const Index* ix) { return (ix->p.max_read_len + 63u) & ~63u; }

// Reads resident on the device for the duration of one call.
struct DeviceReads {
  const char* seq = nullptr;
  const uint64_t* off = nullptr;
  uint32_t n = 0;
  char* own_seq = nullptr;       // set when the library uploaded host reads
  uint64_t* own_off = nullptr;
};

// Validate host reads (length and characters).  MAXSS_OK or an error status.
maxss_status validate_host_reads(const Index* ix, const maxss_reads* r);

// Upload host reads (stream-ordered allocation) or wrap device reads.
maxss_status stage_reads(const maxss_reads* r, hipStream_t st, DeviceReads* out);
void release_reads(DeviceReads* d, hipStream_t st);

// Encoded reads for one call.
//   sel4  : per read and strand, mstride/8 words of 4-bit pool-shift codes,
//           8 positions per word (position k at bits 4*(k%8)): the byte of the
//           scan's score pool that the read base turns into a match score
//           (A 1, C 3, G 5, T 7; N and the padding past the read 4, a byte no
//           genome selector reads).
//   codes : forward-strand base codes (kA..kN), kN past the end.
//   lens  : read lengths, 0 for an invalid read.
struct EncodedReads {
  uint32_t* sel4 = nullptr;  // [n][2][mstride/8]
  uint8_t* codes = nullptr;  // [n][mstride]
  uint32_t* lens = nullptr;  // [n]
  uint32_t mstride = 0;
};

maxss_status encode_reads(const Index* ix, const DeviceReads& r, hipStream_t st,
                          EncodedReads* out);
void release_encoded(EncodedReads* e, hipStream_t st);

// Event bracket of one kernel launch when profiling is on (see
// maxss_profile_enable); a no-op otherwise.
struct ProfScope {
  ProfScope(const char* name, hipStream_t st);
  ~ProfScope();
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace maxss
