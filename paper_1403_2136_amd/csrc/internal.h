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
// Tile shape forced by the autotuner (0 fields = the built-in choice).
struct TileOverride {
  int NP = 0;            // packed offset pairs per lane: 8, 16 or 32
  uint32_t R = 0;        // reads per tile
  uint32_t rounds = 0;   // minimum rounds of work items per resident wave
};

struct Index {
  int device = 0;
  int num_cu = 0;
  size_t lds_per_cu = 0;  // bytes of LDS per compute unit
  TileOverride tune;     // set only by maxss_autotune
  uint64_t G = 0;
  uint32_t F = 0, NF = 0;
  maxss_params p{};
  uint64_t Lpad = 0;
  uint32_t* g2 = nullptr;
  uint32_t* nmask = nullptr;
  uint8_t* codes = nullptr;
  // position-specific scores by Phred quality (qual_scale > 0): match, mismatch
  int8_t qsm[94] = {};
  int8_t qsx[94] = {};
};

// The per-quality score pairs as a kernel argument.
struct QualTable {
  int8_t sm[94];
  int8_t sx[94];
};

inline bool qual_mode(const Index* ix) { return ix->p.qual_scale > 0; }

// Thread-local error message + status helper.
maxss_status fail(maxss_status st, const char* fmt, ...);
void clear_error();

// Returns MAXSS_EDEVICE (and records the message) when e != hipSuccess.
maxss_status check_hip(hipError_t e, const char* what);

// Every device allocation of the library goes through these: hipMalloc and
// hipMallocAsync, except that the allocation maxss_fail_alloc_after armed
// returns hipErrorOutOfMemory without allocating (a test hook for the
// out-of-memory paths).
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t dev_malloc_async(void** p, size_t bytes, hipStream_t st);

// Host-side ASCII -> code, 0xFF for a character outside ACGTN/acgtn.
uint8_t host_code(char c);

// Read positions advanced per first-phase Kadane step: 2 when every other
// base is scored (MAXSS_FAST), else 1.
inline uint32_t scan_step(const Index* ix) { return (ix->p.flags & MAXSS_FAST) ? 2u : 1u; }

// Padded read-profile stride (positions per read per strand) for an index.
inline uint32_t read_stride(const Index* ix) { return (ix->p.max_read_len + 63u) & ~63u; }

// Reads resident on the device for the duration of one call.
struct DeviceReads {
  const char* seq = nullptr;
  const uint64_t* off = nullptr;
  const char* qual = nullptr;    // Phred+33 qualities laid out as seq, or null
  uint32_t n = 0;
  char* own_seq = nullptr;       // set when the library uploaded host reads
  uint64_t* own_off = nullptr;
  char* own_qual = nullptr;
};

// EINVAL when the index scores with base qualities and the reads carry none.
maxss_status require_quals(const Index* ix, const maxss_reads* r);

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
  // [n][mstride] per read position (forward orientation): match score in the
  // low byte, mismatch score in the high byte (int8 each); quality mode only
  uint16_t* qsc = nullptr;
  uint32_t mstride = 0;
};

// Allocation (stream-ordered) and release of encoded reads for n reads.
maxss_status alloc_encoded(const Index* ix, uint32_t n, hipStream_t st, EncodedReads* e);
void release_encoded(EncodedReads* e, hipStream_t st);
// Encode n device reads into preallocated buffers (no allocation).
maxss_status encode_reads_into(const Index* ix, const DeviceReads& r, hipStream_t st,
                               const EncodedReads& e);

// Scratch of the first phase for up to `cap` reads (library-allocated).
struct ScanWork {
  EncodedReads er;
  uint32_t* order = nullptr;   // [cap]
  uint32_t* hist = nullptr;    // [max_read_len + 1]
  uint32_t* ctr = nullptr;     // [1]
  int4* partial = nullptr;     // [partial_cap]
  uint64_t partial_cap = 0;    // entries (read x fragment chunk)
  // MAXSS_EXCLUDE_ADJACENT only: the second pass's fragment left out, read
  // lengths (0 = not scanned again) and records, per read
  int32_t* excl = nullptr;     // [cap]
  uint32_t* lens2 = nullptr;   // [cap]
  maxss_top2* again = nullptr; // [cap]
};

// Entries the partial buffer needs for n reads (built-in or forced tiles).
uint64_t scan_partial_entries(const Index* ix, uint32_t n, const TileOverride* force);
maxss_status alloc_scan_work(const Index* ix, uint32_t n, uint64_t partial_cap, bool stream_ordered,
                             hipStream_t st, ScanWork* w);
void release_scan_work(ScanWork* w, bool stream_ordered, hipStream_t st);

// First phase on n device reads with the given scratch: encode, length sort,
// scan, merge, exact re-scan of the winners.  No allocation, no host sync, so
// it may be captured into a graph.  `force` (may be NULL) overrides tiles.
maxss_status scan_pipeline(const Index* ix, const DeviceReads& r, maxss_top2* dout,
                           const ScanWork& w, const TileOverride* force, hipStream_t st);

// First phase on encoded reads with per-read lengths `lens` (0 = skip):
// the full scan, or (candidate_scan) only each read's Kc first candidates of
// `cand` (K per read, ascending fragment ids).  Records of skipped reads are
// invalid.  No allocation.
maxss_status scan_pipeline_lens(const Index* ix, const EncodedReads& er, const uint32_t* lens,
                                uint32_t n, maxss_top2* dout, const ScanWork& w, hipStream_t st);
maxss_status candidate_scan(const Index* ix, const EncodedReads& er, const uint32_t* lens,
                            uint32_t n, const int32_t* cand, uint32_t K, uint32_t Kc,
                            maxss_top2* dout, const ScanWork& w, hipStream_t st);

// Second phase scratch and launch (reads already encoded in `er`).
struct NwShape {
  uint32_t cw = 0, ncols_max = 0, rowbytes = 0, grid = 0;
  uint32_t wave_cw = 0;  // columns per lane of the wave kernel, 0 = block kernel
  bool fit = false;       // fitting mode in 16 bits: the two-pass kernel (wave_cw columns per lane)
  bool lds_moves = false; // the two-pass kernel keeps a one-strip window's moves in LDS
  size_t lds = 0;
};
maxss_status nw_shape(const Index* ix, uint32_t n, uint32_t pad, NwShape* sh);
maxss_status nw_pipeline(const Index* ix, const EncodedReads& er, uint32_t n,
                         const maxss_top2* dtop, uint32_t pad, maxss_aln* dout, char* dcig,
                         uint64_t cigar_stride, uint8_t* slab, const NwShape& sh,
                         hipStream_t st);

// Event bracket of one kernel launch when profiling is on (see
// maxss_profile_enable); a no-op otherwise.
// True while `st` is being captured into a graph.
bool stream_capturing(hipStream_t st);

struct ProfScope {
  ProfScope(const char* name, hipStream_t st);
  ~ProfScope();
  const char* name;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace maxss
