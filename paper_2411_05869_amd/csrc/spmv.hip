// CSR products with the assembled matrix (binned order).
//
// SpMV: rows with at most kLongRow entries are handled by groups of G lanes
// (G consecutive lanes stride over the row, then a fixed shuffle tree sums
// the partials), longer rows by one wave each (listed at assembly).  Every
// row's sum is formed in the same order on every call, so results are
// bitwise reproducible; no floating-point atomics are used.
//
// SpMM: k <= 32 right-hand sides, X and Y row-major n x ld, optional
// symmetric diagonal scaling Y = S K S X (see k_spmm).
#include <type_traits>

#include "device.hpp"

namespace gps {
namespace {

constexpr int kThreads = 256;
constexpr int kG = 8;

constexpr int kU = 4;   // independent loads in flight per lane

inline unsigned round_up8(unsigned v) { return (v + 7u) & ~7u; }

// Partial row sum over entries [s, e) for lane `sub` of a group of G lanes: each
// lane keeps kU (column, value) pairs in flight before gathering x, so a row's
// loads overlap instead of forming a dependent chain.  Lanes past the row end
// read x[self] with weight 0.
template <typename VT, typename XT, typename AT, int G>
__device__ __forceinline__ AT spmv_part(int64_t s, int64_t e, int sub, int32_t self, const int32_t* __restrict__ col,
                                        const VT* __restrict__ val, const XT* __restrict__ x) {
  AT acc = 0;
  for (int64_t j0 = s + sub; j0 < e; j0 += kU * G) {
    int32_t c[kU];
    AT v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t j = j0 + u * G;
      const bool in = j < e;
      c[u] = in ? col[j] : self;
      v[u] = in ? static_cast<AT>(val[j]) : AT(0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) acc += v[u] * static_cast<AT>(x[c[u]]);
  }
  return acc;
}

// CSR part of the product (entries after each row's leading group entries).
// One launch: blocks [0, nb_long) take the listed long rows, one wave per row
// (dispatched first, they set the tail); the remaining blocks take rows of at
// most kLongRow entries with kG lanes per row.  Rows with group entries add
// the group-block part that k_group_spmv wrote to y before.
template <typename VT, typename XT, typename AT, typename YT>
__global__ void __launch_bounds__(kThreads) k_spmv(int64_t n, unsigned nb_long, int64_t nlong,
                                                   const int32_t* __restrict__ rows, const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ gskip,
                                                   const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                   const XT* __restrict__ x, YT* __restrict__ y) {
  if (blockIdx.x >= nb_long) {
    const unsigned b = xcd_remap(blockIdx.x - nb_long, gridDim.x - nb_long);
    const int64_t row = (b * static_cast<int64_t>(kThreads) + threadIdx.x) / kG;
    const int sub = threadIdx.x & (kG - 1);
    if (row >= n) return;
    const int32_t gs = gskip[row];
    const int64_t s = rp[row] + gs, e = rp[row + 1];
    if (e - s > kLongRow) return;  // uniform within the group
    AT acc = spmv_part<VT, XT, AT, kG>(s, e, sub, static_cast<int32_t>(row), col, val, x);
#pragma unroll
    for (int off = kG / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kG);
    if (sub == 0) y[row] = static_cast<YT>(gs ? static_cast<AT>(y[row]) + acc : acc);
  } else {
    const unsigned b = xcd_remap(blockIdx.x, nb_long);
    const int64_t w = (b * static_cast<int64_t>(kThreads) + threadIdx.x) / kWave;
    if (w >= nlong) return;
    const int lane = lane_id();
    const int32_t row = rows[w];
    const int32_t gs = gskip[row];
    const int64_t s = rp[row] + gs, e = rp[row + 1];
    AT acc = spmv_part<VT, XT, AT, kWave>(s, e, lane, row, col, val, x);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane == 0) y[row] = static_cast<YT>(gs ? static_cast<AT>(y[row]) + acc : acc);
  }
}

// SpMM, Y = S K S X (S = diag(scale), or K X without scale), k <= 32 columns of
// a row-major block with leading dimension ld.
//
// A wave stages 64 consecutive entries of a row at a time: lane l loads entry
// l (column id and value * scale[column]) with one coalesced access.  The
// entries are then consumed in pairs: half-wave h = l >> 5 takes entry 2i + h
// and lane l works on column l & 31, receiving the entry's column id and
// weight from the staging lane by ds_bpermute.  All X gathers of a staged
// chunk are independent, so kUm of them are in flight per lane.
// Blocks [0, nb_short) give each short row (<= kLongRow entries) one wave;
// the remaining blocks give each long row a whole block: wave w takes the
// chunks w, w + 4, ... and the four partial rows are added in a fixed order.
constexpr int kUm = 8;

template <typename T>
__device__ __forceinline__ T shfl_any(T v, int src) {
  return __shfl(v, src, kWave);
}

template <typename VT, typename T, bool SCALE>
__device__ __forceinline__ T spmm_chunk(int64_t j0, int64_t e, int32_t self, const int32_t* __restrict__ col,
                                        const VT* __restrict__ val, const T* __restrict__ X,
                                        const T* __restrict__ scale, int ld, int cl, int lane, int h) {
  // stage up to 64 entries
  const int64_t j = j0 + lane;
  int32_t q = self;
  T v = 0;
  if (j < e) {
    q = col[j];
    v = static_cast<T>(val[j]);
    if constexpr (SCALE) v *= scale[q];
  }
  const int m = static_cast<int>(min<int64_t>(e - j0, kWave));
  const int npairs = (m + 1) >> 1;
  T acc = 0;
  for (int i0 = 0; i0 < npairs; i0 += kUm) {
    int32_t qq[kUm];
    T vv[kUm];
#pragma unroll
    for (int u = 0; u < kUm; ++u) {
      const int src = (2 * (i0 + u) + h) & (kWave - 1);  // entries past m carry weight 0
      qq[u] = shfl_any(q, src);
      vv[u] = shfl_any(v, src);
      if (i0 + u >= npairs) vv[u] = 0;
    }
    T xv[kUm];
#pragma unroll
    for (int u = 0; u < kUm; ++u) xv[u] = X[static_cast<int64_t>(qq[u]) * ld + cl];
#pragma unroll
    for (int u = 0; u < kUm; ++u) acc += vv[u] * xv[u];
  }
  return acc;
}

template <typename VT, typename T, bool SCALE>
__global__ void __launch_bounds__(kThreads) k_spmm(int64_t n, unsigned nb_short, int64_t nlong,
                                                   const int32_t* __restrict__ rows, int k, int ld,
                                                   const int64_t* __restrict__ rp, const int32_t* __restrict__ gskip,
                                                   const int32_t* __restrict__ col,
                                                   const VT* __restrict__ val, const T* __restrict__ X,
                                                   T* __restrict__ Y, const T* __restrict__ scale) {
  const int lane = lane_id();
  const int c = lane & 31;
  const int cl = c < k ? c : k - 1;  // lanes past k re-read column k-1 (in bounds), never store
  const int h = lane >> 5;
  const int w = threadIdx.x / kWave;
  if (blockIdx.x < nb_short) {
    const int64_t row = xcd_remap(blockIdx.x, nb_short) * static_cast<int64_t>(kThreads / kWave) + w;
    if (row >= n) return;
    const int32_t gs = gskip[row];
    const int64_t s = rp[row] + gs, e = rp[row + 1];
    if (e - s > kLongRow) return;
    T acc = 0;
    for (int64_t j0 = s; j0 < e; j0 += kWave)
      acc += spmm_chunk<VT, T, SCALE>(j0, e, static_cast<int32_t>(row), col, val, X, scale, ld, cl, lane, h);
    acc += __shfl_xor(acc, 32, kWave);
    if (h == 0 && c < k) {
      if (gs) acc = Y[row * ld + c] + acc;
      if constexpr (SCALE) acc *= scale[row];
      Y[row * ld + c] = acc;
    }
  } else {
    __shared__ T part[kThreads / kWave][32];
    const int64_t li = xcd_remap(blockIdx.x - nb_short, gridDim.x - nb_short);
    if (li >= nlong) return;  // uniform over the block
    const int32_t row = rows[li];
    const int32_t gs = gskip[row];
    const int64_t s = rp[row] + gs, e = rp[row + 1];
    T acc = 0;
    for (int64_t j0 = s + static_cast<int64_t>(w) * kWave; j0 < e; j0 += kThreads)
      acc += spmm_chunk<VT, T, SCALE>(j0, e, row, col, val, X, scale, ld, cl, lane, h);
    acc += __shfl_xor(acc, 32, kWave);
    if (h == 0) part[w][c] = acc;
    __syncthreads();
    if (w == 0 && h == 0 && c < k) {
      T t = part[0][c];
#pragma unroll
      for (int i = 1; i < kThreads / kWave; ++i) t += part[i][c];
      if (gs) t = Y[static_cast<int64_t>(row) * ld + c] + t;
      if constexpr (SCALE) t *= scale[row];
      Y[static_cast<int64_t>(row) * ld + c] = t;
    }
  }
}

// Group-block part of the product: for the rows of one tile (same mask M,
// at most kTileRows rows) y[row] = sum_k val[row, k] x[U_M[k]] over the
// row's leading |U_M| entries.  x[U_M] is staged in LDS one chunk at a time
// and each staged value serves the four rows a wave owns.
constexpr int kGChunk = 1024;

template <typename VT, typename XT, typename AT, typename YT>
__global__ void __launch_bounds__(kThreads) k_group_spmv(const int32_t* __restrict__ tiles,
                                                         const int32_t* __restrict__ grows,
                                                         const int64_t* __restrict__ uoff,
                                                         const int32_t* __restrict__ ulist,
                                                         const int64_t* __restrict__ rp, const VT* __restrict__ val,
                                                         const XT* __restrict__ x, YT* __restrict__ y) {
  __shared__ AT xs[kGChunk];
  constexpr int kRows = kTileRows / (kThreads / kWave);
  const int4 t = reinterpret_cast<const int4*>(tiles)[xcd_remap(blockIdx.x, gridDim.x)];
  const int32_t* U = ulist + uoff[t.x];
  const int64_t nU = uoff[t.x + 1] - uoff[t.x];
  const int w = threadIdx.x / kWave, lane = lane_id();
  int64_t base[kRows];
  bool has[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int i = w + r * (kThreads / kWave);
    has[r] = i < t.z;
    base[r] = has[r] ? rp[grows[t.y + i]] : 0;
  }
  AT acc[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) acc[r] = 0;
  constexpr int kPer = kGChunk / kThreads;
  AT xr[kPer];
  auto load = [&](int64_t c0) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int64_t k = c0 + threadIdx.x + i * kThreads;
      xr[i] = k < nU ? static_cast<AT>(x[U[k]]) : AT(0);
    }
  };
  load(0);
  for (int64_t c0 = 0; c0 < nU; c0 += kGChunk) {
    const int clen = static_cast<int>(min<int64_t>(kGChunk, nU - c0));
    __syncthreads();  // the previous chunk has been consumed
#pragma unroll
    for (int i = 0; i < kPer; ++i) xs[threadIdx.x + i * kThreads] = xr[i];
    __syncthreads();
    if (c0 + kGChunk < nU) load(c0 + kGChunk);   // in flight while this chunk is consumed
    for (int k0 = lane; k0 < clen; k0 += 4 * kWave) {
      AT v[4][kRows];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          const int k = k0 + u * kWave;
          v[u][r] = (has[r] && k < clen) ? static_cast<AT>(val[base[r] + c0 + k]) : AT(0);
        }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + u * kWave;
        const AT xk = k < clen ? xs[k] : AT(0);
#pragma unroll
        for (int r = 0; r < kRows; ++r) acc[r] += v[u][r] * xk;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    AT a = acc[r];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
    if (lane == 0 && has[r]) y[grows[t.y + w + r * (kThreads / kWave)]] = static_cast<YT>(a);
  }
}

template <typename VT, typename XT, typename AT, typename YT>
void spmv_impl(gp_ctx* c, const gp_matrix* m, const XT* x, YT* y) {
  const VT* val = static_cast<const VT*>(m->val);
  // long-row blocks padded to a multiple of the XCD count so that both block
  // ranges start on XCD 0 (see xcd_remap)
  const unsigned nb_short = grid_for(m->n * kG, kThreads);
  const unsigned nb_long = m->n_long > 0 ? round_up8(grid_for(m->n_long * kWave, kThreads)) : 0;
  ProfScope ps(c, sizeof(VT) == 4 ? (sizeof(XT) == 4 ? "spmv_f32" : "spmv_f32val_f64") : "spmv_f64");
  if (m->ntiles > 0)
    hipLaunchKernelGGL((k_group_spmv<VT, XT, AT, YT>), dim3(static_cast<unsigned>(m->ntiles)), dim3(kThreads), 0,
                       c->stream, m->g_tiles, m->g_rows, m->g_uoff, m->g_ulist, m->row_ptr, val, x, y);
  hipLaunchKernelGGL((k_spmv<VT, XT, AT, YT>), dim3(nb_short + nb_long), dim3(kThreads), 0, c->stream, m->n,
                     nb_long, m->n_long, m->long_rows, m->row_ptr, m->gskip, m->col, val, x, y);
  check_launch("spmv");
}

}  // namespace

void spmv_f64(gp_ctx* c, const gp_matrix* m, const double* x, double* y) {
  if (m->prec == GP_MIXED)
    spmv_impl<float, double, double, double>(c, m, x, y);
  else
    spmv_impl<double, double, double, double>(c, m, x, y);
}

void spmv_f32(gp_ctx* c, const gp_matrix* m, const float* x, float* y) {
  if (m->prec == GP_MIXED)
    spmv_impl<float, float, float, float>(c, m, x, y);
  else
    spmv_impl<double, float, float, float>(c, m, x, y);
}

// Group-block part of the SpMM: for the rows of one tile (same mask M),
// Y[row, :] = sum_k val[row, k] scale[u_k] X[u_k, :] over U_M = (u_k) (the row
// scaling is applied by the CSR part).  Chunks of kMChunk rows of X (scaled)
// are staged in LDS; each wave owns kRows rows, stages their values for the
// chunk in its own LDS slice, and lane (c, h) adds the entries k = h, h + 2, ...
// of column c, so every X value read from LDS feeds kRows multiply-adds.
constexpr int kMChunk = 64;

template <typename VT, typename T, bool SCALE>
__global__ void __launch_bounds__(kThreads) k_group_spmm(const int32_t* __restrict__ tiles,
                                                         const int32_t* __restrict__ grows,
                                                         const int64_t* __restrict__ uoff,
                                                         const int32_t* __restrict__ ulist, int k, int ld,
                                                         const int64_t* __restrict__ rp, const VT* __restrict__ val,
                                                         const T* __restrict__ X, T* __restrict__ Y,
                                                         const T* __restrict__ scale) {
  constexpr int kW = kThreads / kWave;
  constexpr int kRows = kTileRows / kW;
  __shared__ T xs[kMChunk][32];
  __shared__ T vs[kW][kRows][kMChunk];
  const int4 t = reinterpret_cast<const int4*>(tiles)[xcd_remap(blockIdx.x, gridDim.x)];
  const int32_t* U = ulist + uoff[t.x];
  const int64_t nU = uoff[t.x + 1] - uoff[t.x];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int c = lane & 31, h = lane >> 5;
  const int cl = c < k ? c : k - 1;
  int64_t base[kRows];
  bool has[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int i = w + r * kW;
    has[r] = i < t.z;
    base[r] = has[r] ? rp[grows[t.y + i]] : 0;
  }
  T acc[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) acc[r] = 0;
  for (int64_t c0 = 0; c0 < nU; c0 += kMChunk) {
    const int clen = static_cast<int>(min<int64_t>(kMChunk, nU - c0));
    __syncthreads();
    // stage X rows of the chunk: thread -> (row of chunk, column)
    for (int idx = threadIdx.x; idx < kMChunk * 32; idx += kThreads) {
      const int kk = idx >> 5, cc = idx & 31;
      T v = 0;
      if (kk < clen && cc < k) {
        const int32_t q = U[c0 + kk];
        v = X[static_cast<int64_t>(q) * ld + cc];
        if constexpr (SCALE) v *= scale[q];
      }
      xs[kk][cc] = v;
    }
    // this wave's rows: values of the chunk
#pragma unroll
    for (int r = 0; r < kRows; ++r)
      vs[w][r][lane] = (has[r] && lane < clen) ? static_cast<T>(val[base[r] + c0 + lane]) : T(0);
    __syncthreads();
    for (int kk = h; kk < clen; kk += 2) {
      const T xv = xs[kk][cl];
#pragma unroll
      for (int r = 0; r < kRows; ++r) acc[r] += vs[w][r][kk] * xv;
    }
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const T a = acc[r] + __shfl_xor(acc[r], 32, kWave);
    if (h == 0 && c < k && has[r]) Y[static_cast<int64_t>(grows[t.y + w + r * kW]) * ld + c] = a;
  }
}

template <typename T>
void spmm(gp_ctx* c, const gp_matrix* m, int k, int ld, const T* X, T* Y, const T* scale) {
  if (k > 32 || ld < k) throw Error{GP_EINVAL, "spmm: at most 32 right-hand sides per call"};
  ProfScope ps(c, "spmm");
  const unsigned nb_short = round_up8(grid_for(m->n, kThreads / kWave));
  const unsigned nb = nb_short + static_cast<unsigned>(m->n_long);
  auto go = [&](auto vt, auto sc) {
    using VT = decltype(vt);
    constexpr bool SC = decltype(sc)::value;
    if (m->ntiles > 0)
      hipLaunchKernelGGL((k_group_spmm<VT, T, SC>), dim3(static_cast<unsigned>(m->ntiles)), dim3(kThreads), 0,
                         c->stream, m->g_tiles, m->g_rows, m->g_uoff, m->g_ulist, k, ld, m->row_ptr,
                         static_cast<const VT*>(m->val), X, Y, scale);
    hipLaunchKernelGGL((k_spmm<VT, T, SC>), dim3(nb), dim3(kThreads), 0, c->stream, m->n, nb_short, m->n_long,
                       m->long_rows, k, ld, m->row_ptr, m->gskip, m->col, static_cast<const VT*>(m->val), X, Y,
                       scale);
  };
  if (m->prec == GP_MIXED) {
    if (scale)
      go(float{}, std::true_type{});
    else
      go(float{}, std::false_type{});
  } else {
    if (scale)
      go(double{}, std::true_type{});
    else
      go(double{}, std::false_type{});
  }
  check_launch("spmm");
}

template void spmm<float>(gp_ctx*, const gp_matrix*, int, int, const float*, float*, const float*);
template void spmm<double>(gp_ctx*, const gp_matrix*, int, int, const double*, double*, const double*);

}  // namespace gps
