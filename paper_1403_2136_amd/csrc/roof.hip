// Measured issue rate of packed 16-bit integer adds on this GPU: the
// instruction class of the scan's inner loop (saturating v_pk_add_i16), used
// as the measured counterpart of the nominal roof (CUs x 64 lanes x clock x 2
// halves).
//
// Every lane runs kChains independent chains of clamped packed adds, so no
// instruction waits on the one before it; the grid keeps 8 waves on every
// SIMD.  Operations counted: lanes x adds x 2 halves.
#include "internal.h"

namespace maxss {

static constexpr int kChains = 8;
static constexpr int kUnroll = 16;
static constexpr int kRoofThreads = 256;

__global__ __launch_bounds__(kRoofThreads) void roof_pk_add_kernel(uint32_t iters, uint32_t seed,
                                                                   uint32_t* sink) {
  uint32_t v[kChains];
#pragma unroll
  for (int c = 0; c < kChains; c++) v[c] = seed ^ (threadIdx.x * 2654435761u + (uint32_t)c);
  uint32_t d = seed | 0x00010001u;
  asm volatile("" : "+v"(d));
  for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
    for (int u = 0; u < kUnroll; u++)
#pragma unroll
      for (int c = 0; c < kChains; c++)
        asm volatile("v_pk_add_i16 %0, %0, %1 clamp" : "+v"(v[c]) : "v"(d));
  }
  uint32_t x = 0;
#pragma unroll
  for (int c = 0; c < kChains; c++) x ^= v[c];
  if (x == 0x12345678u) sink[blockIdx.x] = x;  // keeps the chains live
}

}  // namespace maxss

using namespace maxss;

extern "C" maxss_status maxss_roof_int16(double* ops_per_s, void* stream) {
  clear_error();
  if (!ops_per_s) return fail(MAXSS_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, ncu = 0;
  maxss_status s;
  if ((s = check_hip(hipGetDevice(&dev), "hipGetDevice")) ||
      (s = check_hip(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev),
                     "hipDeviceGetAttribute")))
    return s;
  const uint32_t grid = (uint32_t)ncu * 8u;  // 8 blocks of 4 waves: 8 waves per SIMD
  const uint32_t iters = 16384;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  uint32_t* sink = nullptr;
  double best = 0.0;
  do {
    if ((s = check_hip(dev_malloc((void**)&sink, sizeof(uint32_t) * grid), "hipMalloc")) ||
        (s = check_hip(hipEventCreate(&e0), "hipEventCreate")) ||
        (s = check_hip(hipEventCreate(&e1), "hipEventCreate")))
      break;
    for (int rep = 0; rep < 4 && !s; rep++) {  // the first launch is a warm-up
      if ((s = check_hip(hipEventRecord(e0, st), "hipEventRecord"))) break;
      roof_pk_add_kernel<<<grid, kRoofThreads, 0, st>>>(iters, 0x9E3779B9u + (uint32_t)rep, sink);
      if ((s = check_hip(hipGetLastError(), "roof_pk_add_kernel")) ||
          (s = check_hip(hipEventRecord(e1, st), "hipEventRecord")) ||
          (s = check_hip(hipEventSynchronize(e1), "hipEventSynchronize")))
        break;
      float ms = 0;
      if ((s = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime"))) break;
      const double ops = (double)grid * kRoofThreads * iters * kUnroll * kChains * 2.0;
      if (rep > 0 && ms > 0 && ops / (ms * 1e-3) > best) best = ops / (ms * 1e-3);
    }
  } while (0);
  if (sink) (void)hipFree(sink);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) return s;
  *ops_per_s = best;
  return MAXSS_OK;
}
