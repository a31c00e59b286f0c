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
#include <algorithm>
#include <type_traits>

#include "device.hpp"

namespace gps {
namespace {

constexpr int kThreads = 256;
constexpr int kG = 8;


inline unsigned round_up8(unsigned v) { return (v + 7u) & ~7u; }

// Partial row sum over entries [s, e) for lane `sub` of a group of G lanes: each
// lane takes 4 consecutive entries at a time (column ids and values by one
// 16-byte load each; a load may run up to 3 entries past the row, which stays
// inside the padded arrays) and gathers their 4 x values together.  Entries past
// the row end read x[self] with weight 0.
template <typename VT, typename XT, typename AT, int G>
__device__ __forceinline__ AT spmv_part(int64_t s, int64_t e, int sub, int32_t self, const int32_t* __restrict__ col,
                                        const VT* __restrict__ val, const XT* __restrict__ x) {
  AT acc = 0;
  for (int64_t j0 = s + 4 * sub; j0 < e; j0 += 4 * G) {
    int32_t c[4];
    VT v[4];
    __builtin_memcpy(c, col + j0, sizeof(c));
    __builtin_memcpy(v, val + j0, sizeof(v));
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = j0 + u < e;
      c[u] = in ? c[u] : self;
      v[u] = in ? v[u] : VT(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += static_cast<AT>(v[u]) * static_cast<AT>(x[c[u]]);
  }
  return acc;
}

// The same sum with the column ids stored as int16 offsets from the row.
template <typename VT, typename XT, typename AT, int G>
__device__ __forceinline__ AT spmv_part16(int64_t s, int64_t e, int sub, int32_t self, const int16_t* __restrict__ off,
                                          const VT* __restrict__ val, const XT* __restrict__ x) {
  AT acc = 0;
  for (int64_t j0 = s + 4 * sub; j0 < e; j0 += 4 * G) {
    int16_t o[4];
    VT v[4];
    __builtin_memcpy(o, off + j0, sizeof(o));
    __builtin_memcpy(v, val + j0, sizeof(v));
    int32_t c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = j0 + u < e;
      c[u] = in ? self + static_cast<int32_t>(o[u]) : self;
      v[u] = in ? v[u] : VT(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += static_cast<AT>(v[u]) * static_cast<AT>(x[c[u]]);
  }
  return acc;
}

// CSR part of the product (entries after each row's leading group entries).
// With off16 (int16 offsets col - row, two bytes per entry instead of four)
// the short rows read the offsets; the long rows always read col.
// One launch: blocks [0, nb_long) take the listed long rows, one wave per row
// (dispatched first, they set the tail); the remaining blocks take rows of at
// most kLongRow entries with kG lanes per row.  Rows with group entries add
// the group-block part that k_group_spmv wrote to y before.
template <typename VT, typename XT, typename AT, typename YT>
__global__ void __launch_bounds__(kThreads) k_spmv(int64_t n, unsigned nb_long, int64_t nlong,
                                                   const int32_t* __restrict__ rows, const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ gskip,
                                                   const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                   const XT* __restrict__ x, YT* __restrict__ y,
                                                   const int16_t* __restrict__ off16, const int* __restrict__ skip) {
  if (skip && *skip) return;  // a device-side decision cancelled this product
  solve_wave_priority();
  if (blockIdx.x >= nb_long) {
    const unsigned b = xcd_remap(blockIdx.x - nb_long, gridDim.x - nb_long);
    const int64_t row = (b * static_cast<int64_t>(kThreads) + threadIdx.x) / kG;
    const int sub = threadIdx.x & (kG - 1);
    if (row < n) {
      const int32_t gs = gskip[row];
      const int64_t s = rp[row] + gs, e = rp[row + 1];
      if (e - s <= kLongRow) {  // uniform within the group
        AT acc = off16 ? spmv_part16<VT, XT, AT, kG>(s, e, sub, static_cast<int32_t>(row), off16, val, x)
                       : spmv_part<VT, XT, AT, kG>(s, e, sub, static_cast<int32_t>(row), col, val, x);
#pragma unroll
        for (int off = kG / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kG);
        if (sub == 0) y[row] = static_cast<YT>(gs ? static_cast<AT>(y[row]) + acc : acc);
      }
    }
  } else {
    const unsigned b = xcd_remap(blockIdx.x, nb_long);
    const int64_t w = (b * static_cast<int64_t>(kThreads) + threadIdx.x) / kWave;
    if (w < nlong) {
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
}

// SpMM, Y = S K S X (S = diag(scale), or K X without scale), k <= 32 columns of
// a row-major block with leading dimension ld: the CSR part row by row.  With
// 16-byte X loads (VEC) only its long-row blocks run (nb_short = 0); the
// short rows then go through the row quads (k_spmm_quad).
//
// A wave stages 64 consecutive entries of a row at a time: lane l loads entry
// l (column id and value * scale[column]) with one coalesced access.  The
// entries are then consumed in pairs: half-wave h = l >> 5 takes entry 2i + h
// and lane l works on column l & 31, receiving the entry's column id and
// weight from the staging lane by ds_bpermute.  All X gathers of a staged
// chunk are independent, so kUm of them are in flight per lane.
// Blocks [0, nb_short) give each wave kRowsPerWave consecutive rows: the
// bounds of all of them are read at once, and the first chunk of the next
// row is staged while the X gathers of the current row are in flight, so the
// dependent loads of consecutive rows overlap.  Rows of more than kLongRow
// entries are skipped there; the remaining blocks give each such row a whole
// block: wave w takes the chunks w, w + 4, ... and the four partial rows are
// added in a fixed order.
constexpr int kUm = 8;
constexpr int kRowsPerWave = 8;

template <typename T>
__device__ __forceinline__ T shfl_any(T v, int src) {
  return __shfl(v, src, kWave);
}

// lane l stages entry j0 + l of [j0, e): its column id q (self when past the
// end) and weight v (0 past the end)
template <typename VT, typename T, bool SCALE>
__device__ __forceinline__ void spmm_stage(int64_t j0, int64_t e, int32_t self, const int32_t* __restrict__ col,
                                           const VT* __restrict__ val, const T* __restrict__ scale, int lane,
                                           int32_t& q, T& v) {
  const int64_t j = j0 + lane;
  q = self;
  v = 0;
  if (j < e) {
    q = col[j];
    v = static_cast<T>(val[j]);
    if constexpr (SCALE) v *= scale[q];
  }
}

// sum over the m staged entries of v * X[q, column]
template <typename T>
__device__ __forceinline__ T spmm_consume(int32_t q, T v, int m, const T* __restrict__ X, int ld, int cl, int h) {
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

// The same sum with 16-byte X loads, for blocks whose rows hold at least 32
// values at 16-byte alignment: lane l works on the kCpl consecutive columns
// kCpl (l % kLpe) ... of entry slot l / kLpe, so one load instruction serves
// kWave / kLpe entries.  Returns the lane's kCpl partial sums; the slots are
// added by the caller.
template <typename T>
struct Vec16 {
  static constexpr int kCpl = 16 / sizeof(T);   // columns per lane
  static constexpr int kLpe = 32 / kCpl;         // lanes per entry
  static constexpr int kEpi = kWave / kLpe;      // entries per load instruction
  T v[kCpl];
};
constexpr int kUq = 4;

template <typename T>
__device__ __forceinline__ Vec16<T> spmm_consume16(int32_t q, T v, int m, const T* __restrict__ X, int ld,
                                                    int lane) {
  using V = Vec16<T>;
  const int g = lane / V::kLpe, cp = lane % V::kLpe;
  const int nq = (m + V::kEpi - 1) / V::kEpi;
  V acc;
#pragma unroll
  for (int u = 0; u < V::kCpl; ++u) acc.v[u] = 0;
  for (int i0 = 0; i0 < nq; i0 += kUq) {
    int32_t qq[kUq];
    T vv[kUq];
#pragma unroll
    for (int u = 0; u < kUq; ++u) {
      const int src = (V::kEpi * (i0 + u) + g) & (kWave - 1);  // entries past m carry weight 0
      qq[u] = shfl_any(q, src);
      vv[u] = shfl_any(v, src);
      if (i0 + u >= nq) vv[u] = 0;
    }
    V xv[kUq];
#pragma unroll
    for (int u = 0; u < kUq; ++u) __builtin_memcpy(xv[u].v, X + static_cast<int64_t>(qq[u]) * ld + cp * V::kCpl, 16);
#pragma unroll
    for (int u = 0; u < kUq; ++u)
#pragma unroll
      for (int t = 0; t < V::kCpl; ++t) acc.v[t] += vv[u] * xv[u].v[t];
  }
  return acc;
}

// adds the entry slots of spmm_consume16 (lanes l, l + kLpe, ...), fixed order
template <typename T>
__device__ __forceinline__ void slot_sum(Vec16<T>& a) {
#pragma unroll
  for (int off = Vec16<T>::kLpe; off < kWave; off <<= 1)
#pragma unroll
    for (int t = 0; t < Vec16<T>::kCpl; ++t) a.v[t] += __shfl_xor(a.v[t], off, kWave);
}

template <typename VT, typename T, bool SCALE, bool VEC>
__global__ void __launch_bounds__(kThreads) k_spmm(int64_t n, unsigned nb_short, int64_t nlong,
                                                   const int32_t* __restrict__ rows, int k, int ld,
                                                   const int64_t* __restrict__ rp, const int32_t* __restrict__ gskip,
                                                   const int32_t* __restrict__ col,
                                                   const VT* __restrict__ val, const T* __restrict__ X,
                                                   T* __restrict__ Y, const T* __restrict__ scale,
                                                   const double* __restrict__ colscale) {
  using V = Vec16<T>;
  const int lane = lane_id();
  const int c = lane & 31;
  const int cl = c < k ? c : k - 1;  // lanes past k re-read column k-1 (in bounds), never store
  const int h = lane >> 5;
  const int w = threadIdx.x / kWave;
  // column factors, read once: lane c (pair path) or the lane's kCpl columns (VEC)
  T csc = 1, csv[V::kCpl];
#pragma unroll
  for (int t = 0; t < V::kCpl; ++t) csv[t] = 1;
  if (colscale) {
    csc = static_cast<T>(colscale[cl]);
#pragma unroll
    for (int t = 0; t < V::kCpl; ++t) csv[t] = static_cast<T>(colscale[min((lane % V::kLpe) * V::kCpl + t, k - 1)]);
  }
  // finishes a row: acc holds the pair-path sum (VEC false) or the lane's
  // slot sums (VEC true); adds the group part already in Y, scales, stores
  auto finish = [&](int64_t row, int32_t gs, T acc, V accv) {
    if constexpr (VEC) {
      slot_sum<T>(accv);
      if (lane < V::kLpe) {
        T* yr = Y + row * ld + lane * V::kCpl;
#pragma unroll
        for (int t = 0; t < V::kCpl; ++t) {
          if (lane * V::kCpl + t >= k) break;
          T a = accv.v[t];
          if (gs) a = yr[t] + a;
          if constexpr (SCALE) a *= scale[row];
          if (colscale) a *= csv[t];
          yr[t] = a;
        }
      }
    } else {
      acc += __shfl_xor(acc, 32, kWave);
      if (h == 0 && c < k) {
        if (gs) acc = Y[row * ld + c] + acc;
        if constexpr (SCALE) acc *= scale[row];
        if (colscale) acc *= csc;
        Y[row * ld + c] = acc;
      }
    }
  };
  auto consume = [&](int32_t q, T v, int m, T& acc, V& accv) {
    if constexpr (VEC) {
      const V a = spmm_consume16<T>(q, v, m, X, ld, lane);
#pragma unroll
      for (int t = 0; t < V::kCpl; ++t) accv.v[t] += a.v[t];
    } else {
      acc += spmm_consume<T>(q, v, m, X, ld, cl, h);
    }
  };
  if (blockIdx.x < nb_short) {
    const int64_t r0 = (xcd_remap(blockIdx.x, nb_short) * static_cast<int64_t>(kThreads / kWave) + w) * kRowsPerWave;
    if (r0 >= n) return;
    const int nr = static_cast<int>(min<int64_t>(kRowsPerWave, n - r0));
    // lane l < nr: first non-group entry, end and group flag of row r0 + l
    int64_t rs = 0, re = 0;
    int32_t rg = 0;
    if (lane < nr) {
      rg = gskip[r0 + lane];
      rs = rp[r0 + lane] + rg;
      re = rp[r0 + lane + 1];
    }
    int32_t q = 0;
    T v = 0;
    {
      const int64_t s = shfl_any(rs, 0), e = shfl_any(re, 0);
      if (e - s <= kLongRow) spmm_stage<VT, T, SCALE>(s, e, static_cast<int32_t>(r0), col, val, scale, lane, q, v);
    }
    for (int r = 0; r < nr; ++r) {
      const int64_t row = r0 + r;
      const int64_t s = shfl_any(rs, r), e = shfl_any(re, r);
      const int32_t gs = shfl_any(rg, r);
      // stage the next row's first chunk while this row's gathers run
      int32_t qn = 0;
      T vn = 0;
      if (r + 1 < nr) {
        const int64_t sn = shfl_any(rs, r + 1), en = shfl_any(re, r + 1);
        if (en - sn <= kLongRow)
          spmm_stage<VT, T, SCALE>(sn, en, static_cast<int32_t>(row + 1), col, val, scale, lane, qn, vn);
      }
      if (e - s <= kLongRow) {
        T acc = 0;
        V accv;
#pragma unroll
        for (int t = 0; t < V::kCpl; ++t) accv.v[t] = 0;
        consume(q, v, static_cast<int>(min<int64_t>(e - s, kWave)), acc, accv);
        for (int64_t j0 = s + kWave; j0 < e; j0 += kWave) {
          int32_t q2;
          T v2;
          spmm_stage<VT, T, SCALE>(j0, e, static_cast<int32_t>(row), col, val, scale, lane, q2, v2);
          consume(q2, v2, static_cast<int>(min<int64_t>(e - j0, kWave)), acc, accv);
        }
        finish(row, gs, acc, accv);
      }
      q = qn;
      v = vn;
    }
  } else {
    __shared__ T part[kThreads / kWave][32];
    const int64_t li = xcd_remap(blockIdx.x - nb_short, gridDim.x - nb_short);
    if (li >= nlong) return;  // uniform over the block
    const int32_t row = rows[li];
    const int32_t gs = gskip[row];
    const int64_t s = rp[row] + gs, e = rp[row + 1];
    T acc = 0;
    V accv;
#pragma unroll
    for (int t = 0; t < V::kCpl; ++t) accv.v[t] = 0;
    for (int64_t j0 = s + static_cast<int64_t>(w) * kWave; j0 < e; j0 += kThreads) {
      int32_t q;
      T v;
      spmm_stage<VT, T, SCALE>(j0, e, row, col, val, scale, lane, q, v);
      consume(q, v, static_cast<int>(min<int64_t>(e - j0, kWave)), acc, accv);
    }
    if constexpr (VEC) {
      slot_sum<T>(accv);
      if (lane < V::kLpe)
#pragma unroll
        for (int t = 0; t < V::kCpl; ++t) part[w][lane * V::kCpl + t] = accv.v[t];
    } else {
      acc += __shfl_xor(acc, 32, kWave);
      if (h == 0) part[w][c] = acc;
    }
    __syncthreads();
    if (w == 0 && h == 0 && c < k) {
      T t = part[0][c];
#pragma unroll
      for (int i = 1; i < kThreads / kWave; ++i) t += part[i][c];
      if (gs) t = Y[static_cast<int64_t>(row) * ld + c] + t;
      if constexpr (SCALE) t *= scale[row];
      if (colscale) t *= csc;
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
                                                         const XT* __restrict__ x, YT* __restrict__ y,
                                                         const int* __restrict__ skip) {
  if (skip && *skip) return;  // uniform over the launch
  solve_wave_priority();
  __shared__ AT xs[kGChunk];
  constexpr int kRows = kTileRows / (kThreads / kWave);
  // tiles come largest first; block b runs on XCD b % 8, so every XCD gets an
  // equal share of large and small tiles and the small ones fill the tail
  const int4 t = reinterpret_cast<const int4*>(tiles)[blockIdx.x];
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
    // lane takes entries k .. k + 3 (one 16-byte load per row for float32
    // values; a load may run past the row's group entries, into the row's
    // CSR part, the next row or the zeroed padding after the last row, and
    // those entries get weight 0); one such group per row at a time
    // keeps the kernel at 80 registers (6 waves per SIMD), which measured
    // faster than two groups in flight at 4 waves per SIMD
    for (int k0 = 4 * lane; k0 < clen; k0 += 4 * kWave) {
      VT v[1][kRows][4];
#pragma unroll
      for (int h = 0; h < 1; ++h) {
        const int k = k0 + h * 4 * kWave;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          if (k < clen) {  // a group past the chunk is not loaded (it could run past the array)
            __builtin_memcpy(v[h][r], val + base[r] + c0 + k, 4 * sizeof(VT));
          } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) v[h][r][u] = VT(0);
          }
        }
      }
#pragma unroll
      for (int h = 0; h < 1; ++h) {
        const int k = k0 + h * 4 * kWave;
        AT xk[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xk[u] = k + u < clen ? xs[min(k + u, kGChunk - 1)] : AT(0);
#pragma unroll
        for (int r = 0; r < kRows; ++r)
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[r] += (has[r] ? static_cast<AT>(v[h][r][u]) : AT(0)) * xk[u];
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

// offsets col - row of the CSR part (flag 1 when one does not fit in int16)
__global__ void __launch_bounds__(kThreads) k_col16(int64_t n, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ gskip, const int32_t* __restrict__ col,
                                                    int16_t* __restrict__ off, int* __restrict__ err) {
  // kG lanes per row, as in the product, so consecutive lanes touch consecutive entries
  const int64_t t = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  const int64_t row = t / kG;
  if (row >= n) return;
  for (int64_t j = rp[row] + gskip[row] + (t & (kG - 1)); j < rp[row + 1]; j += kG) {
    const int64_t d = static_cast<int64_t>(col[j]) - row;
    if (d < -32768 || d > 32767) {
      atomicOr(err, 1);
      return;
    }
    off[j] = static_cast<int16_t>(d);
  }
}

template <typename VT, typename XT, typename AT, typename YT>
void spmv_launch(gp_ctx* c, const gp_matrix* m, const XT* x, YT* y, const int* skip = nullptr) {
  const VT* val = static_cast<const VT*>(m->val);
  // long-row blocks padded to a multiple of the XCD count so that both block
  // ranges start on XCD 0 (see xcd_remap)
  const unsigned nb_short = grid_for(m->n * kG, kThreads);
  const unsigned nb_long = m->n_long > 0 ? round_up8(grid_for(m->n_long * kWave, kThreads)) : 0;
  if (m->ntiles > 0)
    hipLaunchKernelGGL((k_group_spmv<VT, XT, AT, YT>), dim3(static_cast<unsigned>(m->ntiles)), dim3(kThreads), 0,
                       c->stream, m->g_tiles, m->g_rows, m->g_uoff, m->g_ulist, m->row_ptr, val, x, y, skip);
  hipLaunchKernelGGL((k_spmv<VT, XT, AT, YT>), dim3(nb_short + nb_long), dim3(kThreads), 0, c->stream, m->n,
                     nb_long, m->n_long, m->long_rows, m->row_ptr, m->gskip, m->col, val, x, y, m->col16, skip);
  check_launch("spmv");
}

template <typename VT, typename XT, typename AT, typename YT>
void spmv_impl(gp_ctx* c, const gp_matrix* m, const XT* x, YT* y, const int* skip) {
  ProfScope ps(c, sizeof(VT) == 4 ? (sizeof(XT) == 4 ? "spmv_f32" : "spmv_f32val_f64") : "spmv_f64");
  spmv_launch<VT, XT, AT, YT>(c, m, x, y, skip);
}

}  // namespace

void free_col16(gp_ctx* c, gp_matrix* m) {
  if (m->col16) dev_free(c, m->col16, sizeof(int16_t) * (m->nnz + kCsrPad));
  m->col16 = nullptr;
}

static void build_col16(gp_ctx* c, gp_matrix* m) {
  if (m->col16_tried) return;
  m->col16_tried = true;
  ProfScope ps(c, "col16_build");
  // the offsets are a cache: without room for them (allocator or context
  // budget) the products keep reading the int32 column ids
  try {
    m->col16 = dev_new<int16_t>(c, m->nnz + kCsrPad);
  } catch (const Error& e) {
    if (e.st != GP_ENOMEM) throw;
    m->col16 = nullptr;
    return;
  }
  GPS_HIP(hipMemsetAsync(c->err_flag, 0, sizeof(int), c->stream));
  hipLaunchKernelGGL(k_col16, dim3(grid_for(m->n * kG, kThreads)), dim3(kThreads), 0, c->stream, m->n, m->row_ptr,
                     m->gskip, m->col, m->col16, c->err_flag);
  check_launch("col16");
  int* h = static_cast<int*>(pinned(c, sizeof(int)));
  GPS_HIP(hipMemcpyAsync(h, c->err_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  if (*h)
    free_col16(c, m);
  else
    m->bytes += sizeof(int16_t) * (m->nnz + kCsrPad);
}

// The same product with whatever caches the matrix already holds: nothing is
// built, allocated, timed or waited for (the int16 offsets are read when an
// earlier product built them; both column forms give bitwise equal sums).
void spmv_f64_enqueue(gp_ctx* c, const gp_matrix* m, const double* x, double* y) {
  if (m->prec == GP_MIXED)
    spmv_launch<float, double, double, double>(c, m, x, y);
  else
    spmv_launch<double, double, double, double>(c, m, x, y);
}

void spmv_f64(gp_ctx* c, const gp_matrix* m, const double* x, double* y, const int* skip) {
  build_col16(c, const_cast<gp_matrix*>(m));
  if (m->prec == GP_MIXED)
    spmv_impl<float, double, double, double>(c, m, x, y, skip);
  else
    spmv_impl<double, double, double, double>(c, m, x, y, skip);
}


namespace {

// Group-block part of the SpMM on the matrix cores.  For the rows of one
// super-tile (same mask M, at most kSuperRows rows) the product is the dense
// contraction Y[rows, 0:32] = V[rows, U_M] (S X)[U_M, 0:32] (the row scaling is
// applied by the CSR part).  One block takes one piece: the super-tile's rows
// times at most kPiece consecutive entries of U_M, so that every block does a
// similar amount of work whatever |U_M| is.  The piece's column ids and
// scales are read into LDS first; then chunks of kMChunk rows of S X are
// staged in LDS (double-buffered) and shared by the eight waves: waves w and
// w + 4 own the 16 rows 16 w ... 16 w + 15 and take the first and second half
// of the k-steps of each chunk on the 16x16x4 MFMA.  Lane (i, kk) = (lane %
// 16, lane / 16) holds A[i][kk] = V[row 16 w + i, 4 s + kk] and B[kk][i] =
// (S X)[U_M[4 s + kk], i] (a second MFMA covers columns 16-31).  The halves
// are added in a fixed order; a super-tile of one piece writes Y, otherwise
// each piece writes its partial block and k_group_reduce adds the pieces in
// order, so the result is deterministic.  Lane l of an MFMA result holds
// four entries v = 0..3 of column l % 16: rows l / 16 + 4 v.
typedef double mfma_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mfma_d4 mfma16x16x4(double a, double b, mfma_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  using type = mfma_d4;
  static __device__ __forceinline__ int row(int kk, int v) { return kk + 4 * v; }
};

constexpr int kMThreads = 512;                   // 8 waves: 4 row groups x 2 halves of each chunk
constexpr int kMChunk = 64;                      // U_M entries per staged chunk
constexpr int kMSteps = kMChunk / 4 / 2;         // MFMA k-steps per wave per chunk
constexpr int kXPer = kMChunk * 32 / kMThreads;  // X values staged per thread
static_assert(kSuperRows == 4 * 16, "one row group of 16 per wave pair");
static_assert(kMSteps == 8 && kMChunk == 64, "lane (i, kk) of a wave half takes 8 consecutive entries");
static_assert(kPiece % kMChunk == 0 && kPiece <= kMThreads, "piece = whole chunks, ids loaded in one pass");

template <typename VT, typename T, bool SCALE>
__global__ void __launch_bounds__(kMThreads) k_group_spmm_mfma(const int32_t* __restrict__ pieces,
                                                               const int32_t* __restrict__ grows,
                                                               const int64_t* __restrict__ uoff,
                                                               const int32_t* __restrict__ ulist, int k, int ld,
                                                               const int64_t* __restrict__ rp,
                                                               const VT* __restrict__ val, const T* __restrict__ X,
                                                               T* __restrict__ Y, const T* __restrict__ scale,
                                                               T* __restrict__ part) {
  using Acc = typename MfmaAcc<T>::type;
  __shared__ T xs[2][kMChunk][33];
  __shared__ int32_t us[kPiece];
  __shared__ T ss[SCALE ? kPiece : 1];
  const unsigned pid = xcd_remap(blockIdx.x, gridDim.x);
  const int4 t = reinterpret_cast<const int4*>(pieces)[pid];
  const int nUall = static_cast<int>(uoff[t.x + 1] - uoff[t.x]);
  const int kstart = t.w;
  const int len = min(kPiece, nUall - kstart);
  const bool whole = kstart == 0 && len == nUall;   // the only piece of its super-tile
  if (threadIdx.x < kPiece) {
    int32_t q = 0;
    if (static_cast<int>(threadIdx.x) < len) q = ulist[uoff[t.x] + kstart + threadIdx.x];
    us[threadIdx.x] = q;
    if constexpr (SCALE) ss[threadIdx.x] = static_cast<int>(threadIdx.x) < len ? scale[q] : T(0);
  }
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int rg = w & 3, half = w >> 2;   // rows 16 rg ... 16 rg + 15; steps of this half of each chunk
  const int i = lane & 15, kk = lane >> 4;
  const bool wave_rows = 16 * rg < t.z;  // uniform over the wave
  // chunk entry of k-step s for this lane (the A and B operands agree on it):
  // lane (i, kk) takes 8 consecutive entries, loaded with one vector load
  auto ent = [&](int s) { return half * (kMChunk / 2) + 8 * kk + s; };
  // A operands, V[row 16 rg + i, kstart + c0 + ent(s)]; rows past the tile read
  // row 0 of the tile and are zeroed.  The loads are clamped into the row's
  // leading U_M entries; a vector load may run up to 7 entries further, which
  // stays inside the value array (its length carries kCsrPad entries of
  // padding).
  const int r = 16 * rg + i;
  const bool rvalid = r < t.z;
  const VT* vrow = val + rp[grows[t.y + (rvalid ? r : 0)]] + kstart;
  VT areg[kMSteps], acur[kMSteps];
  auto load_a = [&](int c0) {
    const int e0 = c0 + ent(0);
    VT v[kMSteps];
    __builtin_memcpy(v, vrow + min(e0, len - 1), sizeof(v));
#pragma unroll
    for (int s = 0; s < kMSteps; ++s) areg[s] = (rvalid && e0 + s < len) ? v[s] : VT(0);
  };
  load_a(0);
  __syncthreads();
  // staging of X: thread -> (chunk row, kXPer consecutive columns); rows of
  // at least 32 values are read with vector loads (columns past k are read
  // but only feed output columns that are never stored)
  constexpr int kSegs = 32 / kXPer;
  const int xr = threadIdx.x / kSegs, xc0 = (threadIdx.x % kSegs) * kXPer;
  const bool xvec = ld >= 32;
  T xreg[kXPer];
  auto load_x = [&](int c0) {
    const int e = min(c0 + xr, len - 1);
    const T* xp = X + static_cast<int64_t>(us[e]) * ld;
    if (xvec) {
      __builtin_memcpy(xreg, xp + xc0, sizeof(xreg));
    } else {
#pragma unroll
      for (int u = 0; u < kXPer; ++u) xreg[u] = xp[min(xc0 + u, k - 1)];
    }
    T sq = c0 + xr < len ? T(1) : T(0);
    if constexpr (SCALE) sq *= ss[e];
#pragma unroll
    for (int u = 0; u < kXPer; ++u) xreg[u] *= sq;
  };
  auto store_x = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kXPer; ++u) xs[buf][xr][xc0 + u] = xreg[u];
  };
  Acc acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  load_x(0);
  store_x(0);
#pragma unroll
  for (int s = 0; s < kMSteps; ++s) acur[s] = areg[s];
  __syncthreads();
  for (int c0 = 0, buf = 0; c0 < len; c0 += kMChunk, buf ^= 1) {
    const bool more = c0 + kMChunk < len;  // uniform over the block
    if (more) {
      load_x(c0 + kMChunk);
      load_a(c0 + kMChunk);
    }
    if (wave_rows) {
      T b0[kMSteps], b1[kMSteps];
#pragma unroll
      for (int s = 0; s < kMSteps; ++s) {
        b0[s] = xs[buf][ent(s)][i];
        b1[s] = xs[buf][ent(s)][i + 16];
      }
#pragma unroll
      for (int s = 0; s < kMSteps; ++s) {
        const T a = static_cast<T>(acur[s]);
        acc0 = mfma16x16x4(a, b0[s], acc0);
        acc1 = mfma16x16x4(a, b1[s], acc1);
      }
    }
    if (more) {
      store_x(buf ^ 1);
#pragma unroll
      for (int s = 0; s < kMSteps; ++s) acur[s] = areg[s];
    }
    __syncthreads();
  }
  // the second half adds into the first in a fixed order (xs is free now)
  T(*red)[16][33] = reinterpret_cast<T(*)[16][33]>(&xs[0][0][0]);
  static_assert(sizeof(xs) >= 4 * 16 * 33 * sizeof(T), "reduction buffer fits in the staging buffer");
  if (half == 1 && wave_rows) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = MfmaAcc<T>::row(kk, v);
      red[rg][rr][i] = acc0[v];
      red[rg][rr][i + 16] = acc1[v];
    }
  }
  __syncthreads();
  if (half == 0 && wave_rows) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = MfmaAcc<T>::row(kk, v);
      const int row = 16 * rg + rr;
      if (row >= t.z) continue;
      const T y0 = acc0[v] + red[rg][rr][i], y1 = acc1[v] + red[rg][rr][i + 16];
      T* yr = whole ? Y + static_cast<int64_t>(grows[t.y + row]) * ld
                    : part + (static_cast<int64_t>(pid) * kSuperRows + row) * 32;
      const int kc = whole ? k : 32;
      if (i < kc) yr[i] = y0;
      if (i + 16 < kc) yr[i + 16] = y1;
    }
  }
}

// Adds the partial blocks of the pieces of each super-tile with more than one
// piece, in piece order, into Y.  Block (super-tile, group of kRedRows rows),
// thread -> (row, column).
constexpr int kRedRows = kThreads / 32;

template <typename T>
__global__ void __launch_bounds__(kThreads) k_group_reduce(const int32_t* __restrict__ stiles,
                                                           const int32_t* __restrict__ grows, int k, int ld,
                                                           const T* __restrict__ part, T* __restrict__ Y) {
  constexpr int kGroups = kSuperRows / kRedRows;
  const int4 t = reinterpret_cast<const int4*>(stiles)[blockIdx.x / kGroups];
  const int row = (blockIdx.x % kGroups) * kRedRows + threadIdx.x / 32, col = threadIdx.x & 31;
  if (t.w <= 1 || row >= t.y || col >= k) return;  // single pieces write Y themselves
  const T* pp = part + (static_cast<int64_t>(t.z) * kSuperRows + row) * 32 + col;
  constexpr int64_t kStride = static_cast<int64_t>(kSuperRows) * 32;
  T acc = pp[0];
  int p = 1;
  for (; p + 4 <= t.w; p += 4) {
    const T a0 = pp[p * kStride], a1 = pp[(p + 1) * kStride], a2 = pp[(p + 2) * kStride], a3 = pp[(p + 3) * kStride];
    acc += a0;
    acc += a1;
    acc += a2;
    acc += a3;
  }
  for (; p < t.w; ++p) acc += pp[p * kStride];
  Y[static_cast<int64_t>(grows[t.x + row]) * ld + col] = acc;
}

}  // namespace

namespace {

// ------------------------------------------------------------ row quads
// The CSR part of the 32-column product reads one 256-byte row of X per
// stored entry.  Rows next to each other along the grid axis with the most
// cells (at the space-time workload: one station on consecutive days) share
// most of their columns, so the rows are listed along that axis (a line: the
// cells with all other cell coordinates fixed, binned order within a cell),
// in segments of kSlabCells cells of a line, and every four consecutive
// listed rows of a segment form a quad that stores the ascending union of its
// rows' columns once, with the four rows' values per entry: one gather of an
// X row serves four rows.  Consecutive quads share many X rows, which then
// come from the caches (k_line_rows gives the order of the segments).
constexpr int kQuad = 4;
constexpr int kLineThreads = 256;
constexpr int kSlabCells = 16;  // cells of a line per listed segment

struct LineGeom {
  int a;            // axis along which a line runs
  int nother;       // number of other axes
  int o[2];         // the other axes, fastest first
  int32_t g[3];     // cells per axis
  int64_t stride[3];
  int64_t nlines;   // lines of the grid
  int64_t lpr;      // lines per region (the lines are cut into kXcds contiguous regions)
  int32_t slab;     // cells of a line per segment
  int32_t nslab;    // segments per line
};

// exclusive prefix sum over the block of v (kLineThreads threads); *total
// receives the block's sum
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* total) {
  __shared__ int32_t wsum[kLineThreads / kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  __syncthreads();  // wsum of an earlier call has been read
  if (lane == kWave - 1) wsum[w] = x;
  __syncthreads();
  int32_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kLineThreads / kWave; ++i) {
    if (i < w) before += wsum[i];
    all += wsum[i];
  }
  *total = all;
  return before + x - v;
}

// The rows are listed segment by segment: a segment is the rows of lg.slab
// consecutive cells of one line (binned order within a cell), padded to a
// multiple of four.  Segments are ordered by region (kXcds contiguous ranges
// of lines), then slab, then line: the 32-column product gives each XCD a
// contiguous range of quads, so an XCD sweeps its region slab by slab and the
// X rows that neighbouring lines share are read while they are in its L2.
// Block per segment.  PASS 0: the segment's row count padded to a multiple of
// four (lpad).  PASS 1: its rows, then the padding (-1).
template <int PASS>
__global__ void __launch_bounds__(kLineThreads) k_line_rows(LineGeom lg, const int32_t* __restrict__ cell_start,
                                                             int32_t* __restrict__ lpad, const int64_t* __restrict__ loff,
                                                             int32_t* __restrict__ trow) {
  const int64_t S = blockIdx.x;
  const int64_t j = S % lg.lpr, rs = S / lg.lpr;
  const int64_t region = rs / lg.nslab;
  const int slab = static_cast<int>(rs % lg.nslab);
  const int64_t L = region * lg.lpr + j;
  int64_t running = 0;
  const int64_t out0 = PASS == 1 ? loff[S] : 0;
  if (L < lg.nlines) {
    int64_t base = 0, r = L;
    for (int k = 0; k < lg.nother; ++k) {
      const int ax = lg.o[k];
      base += (r % lg.g[ax]) * lg.stride[ax];
      r /= lg.g[ax];
    }
    const int64_t sa = lg.stride[lg.a];
    const int c0 = slab * lg.slab, c1 = min(c0 + lg.slab, lg.g[lg.a]);
    for (int i0 = c0; i0 < c1; i0 += kLineThreads) {
      const int i = i0 + static_cast<int>(threadIdx.x);
      int32_t cs = 0, cnt = 0;
      if (i < c1) {
        const int64_t key = base + i * sa;
        cs = cell_start[key];
        cnt = cell_start[key + 1] - cs;
      }
      int32_t total;
      const int32_t ex = block_excl_scan(cnt, &total);
      if constexpr (PASS == 1)
        for (int32_t t = 0; t < cnt; ++t) trow[out0 + running + ex + t] = cs + t;
      running += total;
    }
  }
  const int64_t pad = (running + kQuad - 1) / kQuad * kQuad;
  if constexpr (PASS == 0) {
    if (threadIdx.x == 0) lpad[S] = static_cast<int32_t>(pad);
  } else {
    for (int64_t t = running + threadIdx.x; t < pad; t += kLineThreads) trow[out0 + t] = -1;
  }
}

// orders the LDS accesses of one wave (its own slice; no block barrier)
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The CSR-part column lists of the rows of quad g (listed rows 4g .. 4g+3;
// padding and rows with more than kLongRow entries count as empty): begin and
// end of each.
__device__ __forceinline__ void quad_lists(int64_t g, const int32_t* __restrict__ trow,
                                           const int64_t* __restrict__ rp, const int32_t* __restrict__ gskip,
                                           int64_t (&h)[kQuad], int64_t (&e)[kQuad]) {
#pragma unroll
  for (int i = 0; i < kQuad; ++i) {
    const int32_t r = trow[g * kQuad + i];
    h[i] = e[i] = 0;
    if (r >= 0) {
      const int64_t s = rp[r] + gskip[r], t = rp[r + 1];
      if (t - s <= kLongRow) {
        h[i] = s;
        e[i] = t;
      }
    }
  }
}

// first index of list[0, len) with list[i] >= c (lower) or > c (upper)
template <bool UPPER>
__device__ __forceinline__ int list_bound(const int32_t* lst, int len, int32_t c) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (UPPER ? lst[mid] <= c : lst[mid] < c)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One wave per quad.  The four rows' CSR-part column lists (ascending, at
// most kLongRow each) are loaded into the wave's LDS slice; every entry (row
// i, position j, column c) finds its place in the merged order by (column,
// row): j plus, in each other row k, the number of columns < c (k > i) or
// <= c (k < i).  Equal columns are then adjacent, at most one per row; the
// first of each run starts a quad entry, numbered by a ballot scan.
// PASS 0 writes the number of entries of each quad, PASS 1 the ascending
// column ids with the four rows' values (0 where a row lacks the column).
constexpr int kQuadMax = kQuad * kLongRow;

template <typename VT, int PASS>
__global__ void __launch_bounds__(kThreads) k_quad_build(int64_t ngroups, const int32_t* __restrict__ trow,
                                                         const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ gskip,
                                                         const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                         int32_t* __restrict__ cnt, const int64_t* __restrict__ qptr,
                                                         int32_t* __restrict__ qcol, VT* __restrict__ qval) {
  __shared__ int32_t lc[kThreads / kWave][kQuad][kLongRow];
  __shared__ int32_t mc[kThreads / kWave][kQuadMax];
  __shared__ int16_t mij[kThreads / kWave][kQuadMax];  // row * kLongRow + position
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int64_t g = blockIdx.x * static_cast<int64_t>(kThreads / kWave) + w;
  if (g >= ngroups) return;  // uniform over the wave
  int64_t h[kQuad], e[kQuad];
  quad_lists(g, trow, rp, gskip, h, e);
  int len[kQuad], off[kQuad + 1];
  off[0] = 0;
#pragma unroll
  for (int i = 0; i < kQuad; ++i) {
    len[i] = static_cast<int>(e[i] - h[i]);
    off[i + 1] = off[i] + len[i];
  }
  const int T = off[kQuad];
#pragma unroll
  for (int i = 0; i < kQuad; ++i)
    for (int j = lane; j < len[i]; j += kWave) lc[w][i][j] = col[h[i] + j];
  wave_sync_lds();
  for (int t = lane; t < T; t += kWave) {
    int i = 0;
#pragma unroll
    for (int k = 1; k < kQuad; ++k)
      if (t >= off[k]) i = k;
    const int j = t - off[i];
    const int32_t c = lc[w][i][j];
    int pos = j;
#pragma unroll
    for (int k = 0; k < kQuad; ++k) {
      if (k < i) pos += list_bound<true>(lc[w][k], len[k], c);
      if (k > i) pos += list_bound<false>(lc[w][k], len[k], c);
    }
    mc[w][pos] = c;
    mij[w][pos] = static_cast<int16_t>(i * kLongRow + j);
  }
  wave_sync_lds();
  int64_t out0 = PASS == 1 ? qptr[g] : 0;
  int running = 0;
  for (int b = 0; b < T; b += kWave) {
    const int p = b + lane;
    const bool first = p < T && (p == 0 || mc[w][p] != mc[w][p - 1]);
    const uint64_t bal = __ballot(first);
    if constexpr (PASS == 1) {
      if (first) {
        const int64_t out = out0 + running + __popcll(bal & lanes_below());
        const int32_t c = mc[w][p];
        VT v[kQuad];
#pragma unroll
        for (int i = 0; i < kQuad; ++i) v[i] = VT(0);
#pragma unroll
        for (int d = 0; d < kQuad; ++d) {
          if (p + d < T && mc[w][p + d] == c) {
            const int ij = mij[w][p + d];
            const int row = ij / kLongRow, j = ij % kLongRow;
#pragma unroll
            for (int i = 0; i < kQuad; ++i)
              if (row == i) v[i] = val[h[i] + j];
          }
        }
        qcol[out] = c;
#pragma unroll
        for (int i = 0; i < kQuad; ++i) qval[out * kQuad + i] = v[i];
      }
    }
    running += __popcll(bal);
  }
  if constexpr (PASS == 0)
    if (lane == 0) cnt[g] = running;
}

// Row codes of the listed rows for the product: -1 for padding and for rows
// with more than kLongRow entries past their group part, the row for a row
// without a group part, -(row + 2) for a row with one.
__global__ void __launch_bounds__(kThreads) k_quad_codes(int64_t ntrow, const int32_t* __restrict__ trow,
                                                         const int64_t* __restrict__ rp,
                                                         const int32_t* __restrict__ gskip, int32_t* __restrict__ code) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i >= ntrow) return;
  const int32_t r = trow[i];
  int32_t c = -1;
  if (r >= 0) {
    const int32_t gs = gskip[r];
    if (rp[r + 1] - rp[r] - gs <= kLongRow) c = gs ? -r - 2 : r;
  }
  code[i] = c;
}

// CSR part of Y = S K S X D for the short rows, one quad at a time (four
// consecutive listed rows share most of their local columns): lane l
// stages union entry j0 + l of the group (column id and the four rows'
// weights, times the column's scale) in the wave's LDS slice; then each
// 16-byte load of an X row serves all four rows.  The same column split as
// spmm_consume16 (lane l: kCpl columns of entry slot l / kLpe), slot sums in
// a fixed order, group part added from Y.
constexpr int kQuadsPerWave = 2;
constexpr int kQuadUq = 2;  // X loads in flight per lane (two keep the kernel at 68 registers)
// Beside another stream's kernels the row-quad product takes 15 KB of dynamic
// LDS more per block: with its 9 KB of static LDS, six blocks (six waves per
// SIMD) fit in a CU's 160 KB instead of the seven its registers allow, and the
// other stream's waves find free slots (measured beside the solve: 6.88 ->
// 6.94 likelihood evaluations per second; alone the product is 2% slower).
constexpr unsigned kShareLds = 15 * 1024;

template <typename VT, bool SCALE>
__global__ void __launch_bounds__(kThreads) k_spmm_quad(int64_t ngroups, const int64_t* __restrict__ qptr,
                                                        const int32_t* __restrict__ qcol,
                                                        const VT* __restrict__ qval, const int32_t* __restrict__ code,
                                                        int k, int ld,
                                                        const double* __restrict__ X, double* __restrict__ Y,
                                                        const double* __restrict__ scale,
                                                        const double* __restrict__ colscale) {
  using V = Vec16<double>;
  __shared__ int32_t sq[kThreads / kWave][kWave];
  __shared__ double sv[kThreads / kWave][kWave][kQuad];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int gs_lane = lane / V::kLpe, cp = lane % V::kLpe;
  double csv[V::kCpl];
#pragma unroll
  for (int t = 0; t < V::kCpl; ++t) csv[t] = colscale ? colscale[min(cp * V::kCpl + t, k - 1)] : 1.0;
  const int64_t wave = static_cast<int64_t>(xcd_remap(blockIdx.x, gridDim.x)) * (kThreads / kWave) + w;
  for (int gi = 0; gi < kQuadsPerWave; ++gi) {
    const int64_t g = wave * kQuadsPerWave + gi;
    if (g >= ngroups) return;  // uniform over the wave
    const int64_t s = qptr[g], e = qptr[g + 1];
    V acc[kQuad];
#pragma unroll
    for (int r = 0; r < kQuad; ++r)
#pragma unroll
      for (int t = 0; t < V::kCpl; ++t) acc[r].v[t] = 0;
    for (int64_t j0 = s; j0 < e; j0 += kWave) {
      const int m = static_cast<int>(min<int64_t>(kWave, e - j0));
      wave_sync_lds();  // the previous chunk has been read
      // Column ids are staged first and the first X rows requested while the
      // column scales are still on their way; the weights (value times the
      // column's scale) follow through the second stage.
      int32_t q = 0;
      VT raw[kQuad];
      double sc = 1.0;
#pragma unroll
      for (int r = 0; r < kQuad; ++r) raw[r] = VT(0);
      if (lane < m) {
        q = qcol[j0 + lane];
#pragma unroll
        for (int r = 0; r < kQuad; ++r) raw[r] = qval[(j0 + lane) * kQuad + r];
      }
      sq[w][lane] = q;
      if (SCALE && lane < m) sc = scale[q];
      wave_sync_lds();
      const int nq = (m + V::kEpi - 1) / V::kEpi;
      int32_t qn[kQuadUq];
      V xn[kQuadUq];
#pragma unroll
      for (int u = 0; u < kQuadUq; ++u) {
        qn[u] = sq[w][(V::kEpi * u + gs_lane) & (kWave - 1)];
        __builtin_memcpy(xn[u].v, X + static_cast<int64_t>(qn[u]) * ld + cp * V::kCpl, 16);
      }
#pragma unroll
      for (int r = 0; r < kQuad; ++r) sv[w][lane][r] = static_cast<double>(raw[r]) * sc;
      wave_sync_lds();
      for (int i0 = 0; i0 < nq; i0 += kQuadUq) {
        int32_t qq[kQuadUq];
        double vv[kQuadUq][kQuad];
#pragma unroll
        for (int u = 0; u < kQuadUq; ++u) {
          const int idx = (V::kEpi * (i0 + u) + gs_lane) & (kWave - 1);  // past m: q = 0, weights 0
          qq[u] = sq[w][idx];
#pragma unroll
          for (int r = 0; r < kQuad; ++r) vv[u][r] = (i0 + u < nq) ? sv[w][idx][r] : 0.0;
        }
        V xv[kQuadUq];
        if (i0 == 0) {
#pragma unroll
          for (int u = 0; u < kQuadUq; ++u) xv[u] = xn[u];
        } else {
#pragma unroll
          for (int u = 0; u < kQuadUq; ++u)
            __builtin_memcpy(xv[u].v, X + static_cast<int64_t>(qq[u]) * ld + cp * V::kCpl, 16);
        }
#pragma unroll
        for (int u = 0; u < kQuadUq; ++u)
#pragma unroll
          for (int r = 0; r < kQuad; ++r)
#pragma unroll
            for (int t = 0; t < V::kCpl; ++t) acc[r].v[t] += vv[u][r] * xv[u].v[t];
      }
    }
#pragma unroll
    for (int r = 0; r < kQuad; ++r) {
      slot_sum<double>(acc[r]);
      const int32_t cr = code[g * kQuad + r];
      if (cr == -1) continue;  // padding, or a row written by the long-row blocks
      const bool grow = cr < -1;
      const int64_t row = grow ? -static_cast<int64_t>(cr) - 2 : cr;
      if (lane < V::kLpe) {
        double* yr = Y + row * ld + lane * V::kCpl;
#pragma unroll
        for (int t = 0; t < V::kCpl; ++t) {
          if (lane * V::kCpl + t >= k) break;
          double a = acc[r].v[t];
          if (grow) a = yr[t] + a;
          if constexpr (SCALE) a *= scale[row];
          if (colscale) a *= csv[t];
          yr[t] = a;
        }
      }
    }
  }
}

}  // namespace

void free_quads(gp_ctx* c, gp_matrix* m) {
  const size_t vbytes = m->prec == GP_MIXED ? sizeof(float) : sizeof(double);
  const int64_t ng = m->ntrow / kQuad;
  if (m->trow) dev_free(c, m->trow, sizeof(int32_t) * std::max<int64_t>(m->ntrow, 1));
  if (m->qptr) dev_free(c, m->qptr, sizeof(int64_t) * (ng + 1));
  if (m->qcol) dev_free(c, m->qcol, sizeof(int32_t) * std::max<int64_t>(m->nquad, 1));
  if (m->qval) dev_free(c, m->qval, vbytes * kQuad * std::max<int64_t>(m->nquad, 1));
  m->trow = nullptr;
  m->qptr = nullptr;
  m->qcol = nullptr;
  m->qval = nullptr;
  m->ntrow = m->nquad = 0;
}

static void build_quads(gp_ctx* c, gp_matrix* m) {
  if (m->qptr) return;
  ProfScope ps(c, "quad_build");
  const gp_dataset* ds = m->ds;
  try {
    // lines along the axis with the most cells (ties: the lowest axis)
    LineGeom lg{};
    lg.a = 0;
    for (int k = 1; k < ds->d; ++k)
      if (ds->g[k] > ds->g[lg.a]) lg.a = k;
    int64_t st = 1;
    for (int k = 0; k < 3; ++k) {
      lg.g[k] = k < ds->d ? ds->g[k] : 1;
      lg.stride[k] = st;
      st *= lg.g[k];
    }
    lg.nother = 0;
    for (int k = 0; k < ds->d; ++k)
      if (k != lg.a) lg.o[lg.nother++] = k;
    const int64_t nlines = ds->ncells / lg.g[lg.a];
    GPS_REQUIRE(nlines * lg.g[lg.a] == ds->ncells, GP_EDEVICE, "quad build: grid does not match the dataset's cells");
    lg.nlines = nlines;
    lg.lpr = (nlines + kXcds - 1) / kXcds;
    lg.slab = kSlabCells;
    lg.nslab = (lg.g[lg.a] + kSlabCells - 1) / kSlabCells;
    const int64_t nseg = static_cast<int64_t>(kXcds) * lg.nslab * lg.lpr;
    GPS_REQUIRE(nseg < (int64_t(1) << 31), GP_ENOMEM, "quad build: too many segments");
    TmpBuf lpad(c, sizeof(int32_t) * nseg), loff(c, sizeof(int64_t) * (nseg + 1));
    hipLaunchKernelGGL((k_line_rows<0>), dim3(static_cast<unsigned>(nseg)), dim3(kLineThreads), 0, c->stream, lg,
                       ds->cell_start, lpad.as<int32_t>(), nullptr, nullptr);
    check_launch("line rows");
    scan_i32_to_i64(c, lpad.as<int32_t>(), loff.as<int64_t>(), nseg);
    m->ntrow = read_i64(c, loff.as<int64_t>() + nseg);
    GPS_REQUIRE(m->ntrow < (int64_t(1) << 31), GP_ENOMEM, "quad build: too many rows");
    m->trow = dev_new<int32_t>(c, std::max<int64_t>(m->ntrow, 1));
    TmpBuf trow(c, sizeof(int32_t) * std::max<int64_t>(m->ntrow, 1));
    hipLaunchKernelGGL((k_line_rows<1>), dim3(static_cast<unsigned>(nseg)), dim3(kLineThreads), 0, c->stream, lg,
                       ds->cell_start, nullptr, loff.as<int64_t>(), trow.as<int32_t>());
    check_launch("line rows");
    const int64_t ng = m->ntrow / kQuad;
    TmpBuf cnt(c, sizeof(int32_t) * std::max<int64_t>(ng, 1));
    m->qptr = dev_new<int64_t>(c, ng + 1);
    auto go = [&](auto vt) {
      using VT = decltype(vt);
      const VT* val = static_cast<const VT*>(m->val);
      const unsigned nbb = grid_for(ng, kThreads / kWave);
      hipLaunchKernelGGL((k_quad_build<VT, 0>), dim3(nbb), dim3(kThreads), 0, c->stream, ng, trow.as<int32_t>(),
                         m->row_ptr, m->gskip, m->col, val, cnt.as<int32_t>(), nullptr, nullptr, nullptr);
      check_launch("quad count");
      scan_i32_to_i64(c, cnt.as<int32_t>(), m->qptr, ng);
      m->nquad = read_i64(c, m->qptr + ng);
      m->qcol = dev_new<int32_t>(c, std::max<int64_t>(m->nquad, 1));
      m->qval = dev_alloc(c, sizeof(VT) * kQuad * std::max<int64_t>(m->nquad, 1));
      hipLaunchKernelGGL((k_quad_build<VT, 1>), dim3(nbb), dim3(kThreads), 0, c->stream, ng, trow.as<int32_t>(),
                         m->row_ptr, m->gskip, m->col, val, nullptr, m->qptr, m->qcol, static_cast<VT*>(m->qval));
      check_launch("quad fill");
      hipLaunchKernelGGL(k_quad_codes, dim3(grid_for(m->ntrow, kThreads)), dim3(kThreads), 0, c->stream, m->ntrow,
                         trow.as<int32_t>(), m->row_ptr, m->gskip, m->trow);
      check_launch("quad row codes");
      sync(c);  // the temporaries are released when their scopes end
      m->bytes += sizeof(int32_t) * m->ntrow + sizeof(int64_t) * (ng + 1) + (sizeof(int32_t) + sizeof(VT) * kQuad) * m->nquad;
    };
    if (m->prec == GP_MIXED)
      go(float{});
    else
      go(double{});
  } catch (...) {
    free_quads(c, m);
    throw;
  }
}

// the work space of a 32-column product (partial blocks of multi-piece super-tiles)
static size_t spmm_part_bytes(const gp_matrix* m) { return sizeof(double) * kSuperRows * 32 * m->npieces; }

void spmm_reserve(gp_ctx* c, const gp_matrix* m) {
  if (m->npieces > 0) (void)workspace(c, 55, spmm_part_bytes(m));
}

template <typename T>
void spmm(gp_ctx* c, const gp_matrix* m, int k, int ld, const T* X, T* Y, const T* scale, const double* colscale,
          bool share) {
  static_assert(std::is_same<T, double>::value, "the products take float64 vectors");
  if (k > 32 || ld < k) throw Error{GP_EINVAL, "spmm: at most 32 right-hand sides per call"};
  // 16-byte X loads need rows of at least 32 values at 16-byte alignment
  const bool vec = ld >= 32 && (ld * sizeof(T)) % 16 == 0 && reinterpret_cast<uintptr_t>(X) % 16 == 0;
  gp_matrix* mm = const_cast<gp_matrix*>(m);  // the quads are a cache of the matrix
  if (vec) build_quads(c, mm);
  ProfScope ps(c, "spmm");
  // partial blocks of the pieces of multi-piece super-tiles
  T* part = m->npieces > 0 ? static_cast<T*>(workspace(c, 55, spmm_part_bytes(m))) : nullptr;
  const unsigned nb_short = round_up8(grid_for((m->n + kRowsPerWave - 1) / kRowsPerWave, kThreads / kWave));
  const unsigned nb = nb_short + static_cast<unsigned>(m->n_long);
  auto go = [&](auto vt, auto sc) {
    using VT = decltype(vt);
    constexpr bool SC = decltype(sc)::value;
    if (m->npieces > 0) {
      const int32_t* st = m->g_tiles + 4 * m->ntiles;
      hipLaunchKernelGGL((k_group_spmm_mfma<VT, T, SC>), dim3(static_cast<unsigned>(m->npieces)), dim3(kMThreads), 0,
                         c->stream, st + 4 * m->nstiles, m->g_rows, m->g_uoff, m->g_ulist, k, ld, m->row_ptr,
                         static_cast<const VT*>(m->val), X, Y, scale, part);
      hipLaunchKernelGGL((k_group_reduce<T>), dim3(static_cast<unsigned>(m->nstiles * (kSuperRows / kRedRows))),
                         dim3(kThreads), 0, c->stream,
                         st, m->g_rows, k, ld, part, Y);
    }
    if (vec) {
      // short rows over the row quads; the long rows by k_spmm's block-per-row path
      const int64_t ng = mm->ntrow / kQuad;
      if (ng > 0) {
        const unsigned nbq =
            static_cast<unsigned>(round_up8(grid_for((ng + kQuadsPerWave - 1) / kQuadsPerWave, kThreads / kWave)));
        hipLaunchKernelGGL((k_spmm_quad<VT, SC>), dim3(nbq), dim3(kThreads), share ? kShareLds : 0, c->stream, ng,
                           mm->qptr, mm->qcol,
                           static_cast<const VT*>(mm->qval), mm->trow, k, ld, X, Y, scale, colscale);
      }
      if (m->n_long > 0)
        hipLaunchKernelGGL((k_spmm<VT, T, SC, true>), dim3(static_cast<unsigned>(m->n_long)), dim3(kThreads), 0,
                           c->stream, m->n, 0u, m->n_long, m->long_rows, k, ld, m->row_ptr, m->gskip, m->col,
                           static_cast<const VT*>(m->val), X, Y, scale, colscale);
    } else {
      hipLaunchKernelGGL((k_spmm<VT, T, SC, false>), dim3(nb), dim3(kThreads), 0, c->stream, m->n, nb_short,
                         m->n_long, m->long_rows, k, ld, m->row_ptr, m->gskip, m->col, static_cast<const VT*>(m->val),
                         X, Y, scale, colscale);
    }
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

template void spmm<double>(gp_ctx*, const gp_matrix*, int, int, const double*, double*, const double*,
                           const double*, bool);

void build_product_caches(gp_ctx* c, gp_matrix* m) {
  build_col16(c, m);
  build_quads(c, m);
}

}  // namespace gps
