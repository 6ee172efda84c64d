// First phase without allocation: maxss_scan_reads for device-resident reads,
// with every scratch buffer carved from one file-scope device array.
//
// The array (kScratchBytes per device) is part of the library's code object:
// each device the library runs on holds its own copy until the process ends.
// Host code never passes the array's name to a kernel (on the host that name
// is only a stand-in, not a device address): the first call on a device looks
// up that device's address with hipGetSymbolAddress, and every later call on
// it uses the cached address.
//
// The scratch is shared by every call on a device and keeps the last call's
// contents; the kernels clear what must start at zero (length histogram, work
// counter) and overwrite the rest before reading it.  Calls that overlap on
// one device (two streams, two host threads) race on it.
#include <mutex>

#include "internal.h"

namespace maxss {

static constexpr size_t kScratchBytes = 64ull << 20;
static constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static uint8_t* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device `dev` (looked up once).
static maxss_status scratch_base(int dev, uint8_t** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MAXSS_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    maxss_status s = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                               "hipGetSymbolAddress(scratch)");
    if (s) return s;
    if (!p) return fail(MAXSS_EDEVICE, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_ptr[dev] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return MAXSS_OK;
}

// Bump carving of the scratch in 256-byte aligned pieces.
// Offsets are computed as integers, so a layout too large for the scratch
// forms no out-of-range pointer before it is rejected.
struct Carver {
  uintptr_t base;
  size_t used = 0;
  template <typename T>
  T* take(size_t bytes) {
    used = (used + 255) & ~(size_t)255;
    T* p = reinterpret_cast<T*>(base + used);
    used += bytes;
    return p;
  }
};

// Lay out the first phase's buffers for n reads in the scratch; the per-chunk
// partial top-2 buffer takes whatever is left (the tile chooser caps the
// fragment chunks per read to fit it).
static maxss_status carve(const Index* ix, uint32_t n, uint8_t* base, ScanWork* w) {
  Carver c{reinterpret_cast<uintptr_t>(base)};
  EncodedReads& e = w->er;
  e.mstride = read_stride(ix);
  const uint64_t mst = e.mstride;
  e.sel4 = c.take<uint32_t>(sizeof(uint32_t) * ((uint64_t)n * 2 * (mst / 8) + 64));
  e.codes = c.take<uint8_t>((uint64_t)n * mst + 64);
  e.lens = c.take<uint32_t>(sizeof(uint32_t) * ((uint64_t)n + 1));
  if (qual_mode(ix)) e.qsc = c.take<uint16_t>(sizeof(uint16_t) * ((uint64_t)n * mst + 64));
  w->order = c.take<uint32_t>(sizeof(uint32_t) * (uint64_t)n);
  w->hist = c.take<uint32_t>(sizeof(uint32_t) * ((uint64_t)ix->p.max_read_len + 1));
  w->ctr = c.take<uint32_t>(sizeof(uint32_t));
  if (ix->p.flags & MAXSS_EXCLUDE_ADJACENT) {
    w->excl = c.take<int32_t>(sizeof(int32_t) * (uint64_t)n);
    w->lens2 = c.take<uint32_t>(sizeof(uint32_t) * (uint64_t)n);
    w->again = c.take<maxss_top2>(sizeof(maxss_top2) * (uint64_t)n);
  }
  // at least one fragment chunk per read
  w->partial = c.take<int4>(0);
  const size_t need = c.used + sizeof(int4) * (uint64_t)n;
  if (need > kScratchBytes) {
    *w = ScanWork{};
    return fail(MAXSS_EINVAL,
                "%u reads of stride %u need at least %llu bytes of scratch; it holds %llu", n,
                (unsigned)mst, (unsigned long long)need, (unsigned long long)kScratchBytes);
  }
  w->partial_cap = (kScratchBytes - c.used) / sizeof(int4);
  return MAXSS_OK;
}

}  // namespace maxss

using namespace maxss;

extern "C" maxss_status maxss_scan_reads_noalloc(const maxss_index* index,
                                                 const maxss_reads* reads, maxss_top2* out,
                                                 void* stream) {
  clear_error();
  const Index* ix = reinterpret_cast<const Index*>(index);
  if (!ix || !reads || !out) return fail(MAXSS_EINVAL, "NULL argument");
  if (!reads->on_device) return fail(MAXSS_EINVAL, "device-resident reads only");
  if (reads->n == 0) return MAXSS_OK;
  if (!reads->seq || !reads->offsets) return fail(MAXSS_EINVAL, "NULL reads");
  maxss_status s;
  if ((s = require_quals(ix, reads))) return s;
  int cur = 0;
  if ((s = check_hip(hipGetDevice(&cur), "hipGetDevice"))) return s;
  if (cur != ix->device) return fail(MAXSS_ESTATE, "index lives on device %d, current is %d",
                                     ix->device, cur);
  uint8_t* base = nullptr;
  if ((s = scratch_base(cur, &base))) return s;
  ScanWork w;
  if ((s = carve(ix, reads->n, base, &w))) return s;
  DeviceReads dr;
  dr.seq = reads->seq;
  dr.off = reads->offsets;
  dr.qual = reads->qual;
  dr.n = reads->n;
  return scan_pipeline(ix, dr, out, w, nullptr, (hipStream_t)stream);
}
