// Deterministic device-wide exclusive scan of integers (two passes): per-tile
// sums, then per tile a wave64 inclusive scan by shuffles and an LDS scan of
// wave totals, offset by the sum of the earlier tiles' sums.
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

// Sum of the tile sums before this block's tile (integers: exact in any order).
template <typename TO>
__device__ __forceinline__ TO tiles_before(const TO* __restrict__ tile_sum) {
  __shared__ TO red[kScanThreads / kWave];
  TO v = 0;
  for (unsigned t = threadIdx.x; t < blockIdx.x; t += kScanThreads) v += tile_sum[t];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  TO s = 0;
#pragma unroll
  for (int i = 0; i < kScanThreads / kWave; ++i) s += red[i];
  __syncthreads();
  return s;
}

// Each block adds the tile sums before its tile itself, so no pass scans the
// tile sums; the last block also writes the total to out[n].
template <typename TI, typename TO>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const TI* __restrict__ in, int64_t n,
                                                             const TO* __restrict__ tile_sum,
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
  const TO tile = block_exclusive_scan<TO>(s, &ex);
  const TO before = tiles_before<TO>(tile_sum);
  const TO off = before + ex;
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = before + tile;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + static_cast<int64_t>(threadIdx.x) * kScanItems + i;
    if (idx < n) out[idx] = off + local[i];
  }
}

template <typename TO>
__global__ void k_scan_zero(TO* __restrict__ out) { out[0] = 0; }

template <typename TI, typename TO>
void scan_impl(gp_ctx* c, const TI* in, TO* out, int64_t n) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  // the tile sums live in a work-space slot of the context: scans run one after
  // another on its stream, and no allocation call sits between the launches
  TO* tiles = static_cast<TO*>(workspace(c, 13, sizeof(TO) * (ntiles > 0 ? ntiles : 1)));
  if (n > 0) {
    hipLaunchKernelGGL((k_tile_sums<TI, TO>), dim3(static_cast<unsigned>(ntiles)), dim3(kScanThreads), 0,
                       c->stream, in, n, tiles);
    check_launch("scan tile sums");
  }
  if (n > 0) {
    hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3(static_cast<unsigned>(ntiles)), dim3(kScanThreads), 0,
                       c->stream, in, n, tiles, out);
    check_launch("scan apply");
  } else {
    hipLaunchKernelGGL((k_scan_zero<TO>), dim3(1), dim3(1), 0, c->stream, out);
    check_launch("scan empty");
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
