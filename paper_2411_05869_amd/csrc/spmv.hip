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

// One launch: blocks [0, nb_long) take the listed long rows, one wave per row
// (dispatched first, they set the tail); the remaining blocks take rows of at
// most kLongRow entries with kG lanes per row.
template <typename VT, typename XT, typename AT, typename YT>
__global__ void __launch_bounds__(kThreads) k_spmv(int64_t n, unsigned nb_long, int64_t nlong,
                                                   const int32_t* __restrict__ rows, const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                   const XT* __restrict__ x, YT* __restrict__ y) {
  if (blockIdx.x >= nb_long) {
    const unsigned b = xcd_remap(blockIdx.x - nb_long, gridDim.x - nb_long);
    const int64_t row = (b * static_cast<int64_t>(kThreads) + threadIdx.x) / kG;
    const int sub = threadIdx.x & (kG - 1);
    if (row >= n) return;
    const int64_t s = rp[row], e = rp[row + 1];
    if (e - s > kLongRow) return;  // uniform within the group
    AT acc = spmv_part<VT, XT, AT, kG>(s, e, sub, static_cast<int32_t>(row), col, val, x);
#pragma unroll
    for (int off = kG / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kG);
    if (sub == 0) y[row] = static_cast<YT>(acc);
  } else {
    const unsigned b = xcd_remap(blockIdx.x, nb_long);
    const int64_t w = (b * static_cast<int64_t>(kThreads) + threadIdx.x) / kWave;
    if (w >= nlong) return;
    const int lane = lane_id();
    const int32_t row = rows[w];
    const int64_t s = rp[row], e = rp[row + 1];
    AT acc = spmv_part<VT, XT, AT, kWave>(s, e, lane, row, col, val, x);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane == 0) y[row] = static_cast<YT>(acc);
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
                                                   const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
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
    const int64_t s = rp[row], e = rp[row + 1];
    if (e - s > kLongRow) return;
    T acc = 0;
    for (int64_t j0 = s; j0 < e; j0 += kWave)
      acc += spmm_chunk<VT, T, SCALE>(j0, e, static_cast<int32_t>(row), col, val, X, scale, ld, cl, lane, h);
    acc += __shfl_xor(acc, 32, kWave);
    if (h == 0 && c < k) {
      if constexpr (SCALE) acc *= scale[row];
      Y[row * ld + c] = acc;
    }
  } else {
    __shared__ T part[kThreads / kWave][32];
    const int64_t li = xcd_remap(blockIdx.x - nb_short, gridDim.x - nb_short);
    if (li >= nlong) return;  // uniform over the block
    const int32_t row = rows[li];
    const int64_t s = rp[row], e = rp[row + 1];
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
      if constexpr (SCALE) t *= scale[row];
      Y[static_cast<int64_t>(row) * ld + c] = t;
    }
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
  hipLaunchKernelGGL((k_spmv<VT, XT, AT, YT>), dim3(nb_short + nb_long), dim3(kThreads), 0, c->stream, m->n,
                     nb_long, m->n_long, m->long_rows, m->row_ptr, m->col, val, x, y);
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

template <typename T>
void spmm(gp_ctx* c, const gp_matrix* m, int k, int ld, const T* X, T* Y, const T* scale) {
  if (k > 32 || ld < k) throw Error{GP_EINVAL, "spmm: at most 32 right-hand sides per call"};
  ProfScope ps(c, "spmm");
  const unsigned nb_short = round_up8(grid_for(m->n, kThreads / kWave));
  const unsigned nb = nb_short + static_cast<unsigned>(m->n_long);
  auto go = [&](auto vt, auto sc) {
    using VT = decltype(vt);
    constexpr bool SC = decltype(sc)::value;
    hipLaunchKernelGGL((k_spmm<VT, T, SC>), dim3(nb), dim3(kThreads), 0, c->stream, m->n, nb_short, m->n_long,
                       m->long_rows, k, ld, m->row_ptr, m->col, static_cast<const VT*>(m->val), X, Y, scale);
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
