// Deterministic device-wide exclusive scan (three passes, fixed order).
// Wave64 inclusive scan by shuffles, then an LDS scan of wave totals per block,
// then a single-block scan of block totals.
#include "internal.hpp"

namespace gps {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int l = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T u = __shfl_up(v, off, kWave);
    if (l >= off) v += u;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* excl) {
  __shared__ T wsum[kScanThreads / kWave];
  const int w = threadIdx.x / kWave;
  const int l = threadIdx.x & (kWave - 1);
  T inc = wave_inclusive_scan(v);
  if (l == kWave - 1) wsum[w] = inc;
  __syncthreads();
  T base = 0, total = 0;
#pragma unroll
  for (int i = 0; i < kScanThreads / kWave; ++i) {
    if (i < w) base += wsum[i];
    total += wsum[i];
  }
  *excl = base + inc - v;
  __syncthreads();
  return total;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kScanThreads) k_tile_sums(const TI* __restrict__ in, int64_t n,
                                                            TO* __restrict__ tile_sum) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
  TO s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + static_cast<int64_t>(i) * kScanThreads + threadIdx.x;
    if (idx < n) s += static_cast<TO>(in[idx]);
  }
  TO ex;
  TO tot = block_exclusive_scan<TO>(s, &ex);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

// Exclusive scan of the tile sums in place by one block; writes the total to *total.
template <typename TO>
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(TO* __restrict__ tile_sum, int64_t ntiles,
                                                             TO* __restrict__ total) {
  TO carry = 0;
  for (int64_t b = 0; b < ntiles; b += kScanThreads) {
    const int64_t i = b + threadIdx.x;
    TO v = i < ntiles ? tile_sum[i] : 0;
    TO ex;
    TO tot = block_exclusive_scan<TO>(v, &ex);
    if (i < ntiles) tile_sum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const TI* __restrict__ in, int64_t n,
                                                             const TO* __restrict__ tile_off,
                                                             TO* __restrict__ out) {
  // each thread owns kScanItems consecutive elements of the tile
  __shared__ TI stage[kScanTile];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + static_cast<int64_t>(i) * kScanThreads + threadIdx.x;
    stage[i * kScanThreads + threadIdx.x] = idx < n ? in[idx] : TI(0);
  }
  __syncthreads();
  TO local[kScanItems];
  TO s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    local[i] = s;
    s += static_cast<TO>(stage[threadIdx.x * kScanItems + i]);
  }
  TO ex;
  block_exclusive_scan<TO>(s, &ex);
  const TO off = tile_off[blockIdx.x] + ex;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + static_cast<int64_t>(threadIdx.x) * kScanItems + i;
    if (idx < n) out[idx] = off + local[i];
  }
}

template <typename TI, typename TO>
void scan_impl(gp_ctx* c, const TI* in, TO* out, int64_t n) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  TmpBuf tiles(c, sizeof(TO) * (ntiles > 0 ? ntiles : 1));
  if (n > 0) {
    hipLaunchKernelGGL((k_tile_sums<TI, TO>), dim3(static_cast<unsigned>(ntiles)), dim3(kScanThreads), 0,
                       c->stream, in, n, tiles.as<TO>());
    check_launch("scan tile sums");
  }
  hipLaunchKernelGGL((k_scan_tiles<TO>), dim3(1), dim3(kScanThreads), 0, c->stream, tiles.as<TO>(), ntiles,
                     out + n);
  check_launch("scan tiles");
  if (n > 0) {
    hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3(static_cast<unsigned>(ntiles)), dim3(kScanThreads), 0,
                       c->stream, in, n, tiles.as<TO>(), out);
    check_launch("scan apply");
  }
}

}  // namespace

void scan_i32_to_i64(gp_ctx* c, const int32_t* in, int64_t* out, int64_t n) {
  scan_impl<int32_t, int64_t>(c, in, out, n);
}

void scan_i32_to_i32(gp_ctx* c, const int32_t* in, int32_t* out, int64_t n) {
  scan_impl<int32_t, int32_t>(c, in, out, n);
}

int64_t read_i64(gp_ctx* c, const int64_t* dev) {
  int64_t* h = static_cast<int64_t*>(pinned(c, sizeof(int64_t)));
  GPS_HIP(hipMemcpyAsync(h, dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return *h;
}

}  // namespace gps
