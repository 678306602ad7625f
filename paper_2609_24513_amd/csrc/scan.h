// Block- and device-wide prefix sums for the ordered compactions of the
// filter, the pair compaction and the serving batch assembly (the result
// materialisation of Section 3.5): a wave scans with lane shuffles, the
// waves of a block combine through LDS, and a device-wide scan runs in
// three launches over tiles of kScanTile items (tile sums, one block
// scanning the tile sums, each tile scanned again from its offset).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pr {
namespace {  // each translation unit keeps its own copy of the kernels

constexpr int kTileThreads = 256;
constexpr int kTileItems = 16;
constexpr int64_t kScanTile = (int64_t)kTileThreads * kTileItems;  // items per tile
constexpr int kTopThreads = 1024;                                  // threads of the tile-sum scan

// Inclusive scan of v over the wave's lanes.
template <typename T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(v, o);
    if (lane >= o) v += y;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Exclusive prefix of v over the block (threads in index order) and the
// block total.  s has one entry per wave; every thread of the block calls
// this (it synchronises twice, so s can be reused right after).
template <int BLOCK, typename T>
__device__ __forceinline__ T block_exclusive_sum(T v, T* s, T& total) {
  static_assert(BLOCK % 64 == 0 && BLOCK <= 1024, "block of whole waves");
  constexpr int kW = BLOCK / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const T inc = wave_inclusive_sum(v);
  if (lane == 63) s[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kW; ++k) {
    const T c = s[k];
    before += k < w ? c : (T)0;
    all += c;
  }
  __syncthreads();
  total = all;
  return before + inc - v;
}

template <int BLOCK, typename T>
__device__ __forceinline__ T block_sum(T v, T* s) {
  T total;
  block_exclusive_sum<BLOCK>(v, s, total);
  return total;
}

// ---- device-wide exclusive scan: out[i] = in[0] + ... + in[i - 1] ----------

// Tile sums: block b adds the items of tile b.
template <typename TI>
__global__ __launch_bounds__(kTileThreads) void k_scan_tiles(const TI* in, int64_t n, int64_t* tsum) {
  __shared__ int64_t s[kTileThreads / 64];
  const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kTileItems;
  int64_t v = 0;
#pragma unroll
  for (int k = 0; k < kTileItems; ++k)
    if (i0 + k < n) v += (int64_t)in[i0 + k];
  const int64_t t = block_sum<kTileThreads>(v, s);
  if (threadIdx.x == 0) tsum[blockIdx.x] = t;
}

// Exclusive scan of the nt tile sums in place, in one block; the total goes
// to *total (when given).
__global__ __launch_bounds__(kTopThreads) void k_scan_top(int64_t* tsum, int64_t nt, int64_t* total) {
  __shared__ int64_t s[kTopThreads / 64];
  int64_t running = 0;
  for (int64_t base = 0; base < nt; base += kTopThreads) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nt ? tsum[i] : 0;
    int64_t all;
    const int64_t pre = block_exclusive_sum<kTopThreads>(v, s, all);
    if (i < nt) tsum[i] = running + pre;
    running += all;
  }
  if (threadIdx.x == 0 && total) *total = running;
}

// Tile b scanned again from its offset tsum[b].
template <typename TI, typename TO>
__global__ __launch_bounds__(kTileThreads) void k_scan_apply(const TI* in, int64_t n, const int64_t* tsum, TO* out) {
  __shared__ int64_t s[kTileThreads / 64];
  const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kTileItems;
  int64_t v[kTileItems];
  int64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kTileItems; ++k) {
    v[k] = i0 + k < n ? (int64_t)in[i0 + k] : 0;
    sum += v[k];
  }
  int64_t all;
  int64_t o = tsum[blockIdx.x] + block_exclusive_sum<kTileThreads>(sum, s, all);
#pragma unroll
  for (int k = 0; k < kTileItems; ++k)
    if (i0 + k < n) {
      out[i0 + k] = (TO)o;
      o += v[k];
    }
}

__host__ __device__ inline int64_t scan_tiles_of(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

// Exclusive scan of in[0, n) into out[0, n) (in and out may not alias);
// tsum holds scan_tiles_of(n) entries; the total goes to *total when given.
template <typename TI, typename TO>
inline hipError_t device_exclusive_scan(const TI* in, TO* out, int64_t n, int64_t* tsum, int64_t* total,
                                        hipStream_t s) {
  const int64_t nt = scan_tiles_of(n);
  if (nt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan_tiles<TI>, dim3((unsigned)nt), dim3(kTileThreads), 0, s, in, n, tsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kTopThreads), 0, s, tsum, nt, total);
  hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3((unsigned)nt), dim3(kTileThreads), 0, s, in, n,
                     (const int64_t*)tsum, out);
  return hipGetLastError();
}

}  // namespace
}  // namespace pr
