// Device-wide exclusive prefix sum of uint32 counts (in place), used by the
// counting sort that keeps particles ordered by grid cell.
#include "scan.h"

namespace sbx {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

// Exclusive scan of each tile of kScanTile items; tile totals to sums.
__global__ void __launch_bounds__(kScanThreads)
    k_scan_tiles(uint32_t* __restrict__ d, size_t n, uint32_t* __restrict__ sums) {
  __shared__ uint32_t wtot[kScanThreads / 64];
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  // whole 16-item runs of an aligned array load as four 16-byte vectors
  const bool vec = ((uintptr_t)d & 15u) == 0 && base + kScanItems <= n;
  if (vec) {
#pragma unroll
    for (int k = 0; k < kScanItems / 4; ++k) {
      const uint4 q = *(const uint4*)(d + base + 4 * k);
      v[4 * k] = q.x;
      v[4 * k + 1] = q.y;
      v[4 * k + 2] = q.z;
      v[4 * k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = base + k < n ? d[base + k] : 0u;
  }
  uint32_t t = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t c = v[k];
    v[k] = t;
    t += c;
  }
  const uint32_t incl = wave_incl_scan(t);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 63) wtot[wave] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (int w = 0; w < wave; ++w) woff += wtot[w];
  const uint32_t off = woff + incl - t;
  if (vec) {
#pragma unroll
    for (int k = 0; k < kScanItems / 4; ++k)
      *(uint4*)(d + base + 4 * k) =
          make_uint4(v[4 * k] + off, v[4 * k + 1] + off, v[4 * k + 2] + off, v[4 * k + 3] + off);
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
      if (base + k < n) d[base + k] = v[k] + off;
  }
  if (threadIdx.x == kScanThreads - 1) {
    uint32_t tot = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) tot += wtot[w];
    sums[blockIdx.x] = tot;
  }
}

__global__ void __launch_bounds__(kScanThreads)
    k_scan_add(uint32_t* __restrict__ d, size_t n, const uint32_t* __restrict__ offs) {
  const uint32_t o = offs[blockIdx.x];
  const size_t base = (size_t)blockIdx.x * kScanTile;
  for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
    if (base + k < n) d[base + k] += o;
}

size_t scan_tmp_elems(size_t n) {
  size_t t = 0;
  while (n > 1) {
    n = (n + kScanTile - 1) / kScanTile;
    t += n;
  }
  return t + 1;
}

sbx_status exclusive_scan_u32(uint32_t* d, size_t n, uint32_t* tmp, hipStream_t s) {
  if (n == 0) return SBX_OK;
  const size_t tiles = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, d, n, tmp);
  SBX_HIP(hipGetLastError());
  if (tiles > 1) {
    SBX_TRY(exclusive_scan_u32(tmp, tiles, tmp + tiles, s));
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, d, n, tmp);
    SBX_HIP(hipGetLastError());
  }
  return SBX_OK;
}

}  // namespace sbx
