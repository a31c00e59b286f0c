// CSR products with the assembled matrix (binned order).
//
// SpMV: rows with at most kLongRow entries are handled by groups of G lanes
// (G consecutive lanes stride over the row, then a fixed shuffle tree sums
// the partials), longer rows by one wave each (listed at assembly).  Every
// row's sum is formed in the same order on every call, so results are
// bitwise reproducible; no floating-point atomics are used.
//
// SpMM: one half-wave per row, lane = right-hand side (k <= 32), X and Y
// row-major n x ld.  Optional symmetric diagonal scaling Y = S K S X.
#include "device.hpp"

namespace gps {
namespace {

constexpr int kThreads = 256;
constexpr int kG = 8;

// One launch: blocks [0, nb_short) take rows of at most kLongRow entries with
// kG lanes per row; the remaining blocks take the listed long rows, one wave
// per row.
template <typename VT, typename XT, typename AT, typename YT>
__global__ void __launch_bounds__(kThreads) k_spmv(int64_t n, unsigned nb_short, int64_t nlong,
                                                   const int32_t* __restrict__ rows, const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                   const XT* __restrict__ x, YT* __restrict__ y) {
  if (blockIdx.x < nb_short) {
    const int64_t row = (blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x) / kG;
    const int sub = threadIdx.x & (kG - 1);
    if (row >= n) return;
    const int64_t s = rp[row], e = rp[row + 1];
    if (e - s > kLongRow) return;  // uniform within the group
    AT acc = 0;
    for (int64_t j = s + sub; j < e; j += kG) acc += static_cast<AT>(val[j]) * static_cast<AT>(x[col[j]]);
#pragma unroll
    for (int off = kG / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kG);
    if (sub == 0) y[row] = static_cast<YT>(acc);
  } else {
    const int64_t w = ((blockIdx.x - nb_short) * static_cast<int64_t>(kThreads) + threadIdx.x) / kWave;
    if (w >= nlong) return;
    const int lane = lane_id();
    const int32_t row = rows[w];
    const int64_t s = rp[row], e = rp[row + 1];
    AT acc = 0;
    for (int64_t j = s + lane; j < e; j += kWave) acc += static_cast<AT>(val[j]) * static_cast<AT>(x[col[j]]);
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane == 0) y[row] = static_cast<YT>(acc);
  }
}

template <typename VT, typename T>
__global__ void __launch_bounds__(kThreads) k_spmm(int64_t n, int k, int ld, const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                   const T* __restrict__ X, T* __restrict__ Y,
                                                   const T* __restrict__ scale) {
  const int64_t row = (blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x) / 32;
  const int c = threadIdx.x & 31;
  if (row >= n) return;
  const int64_t s = rp[row], e = rp[row + 1];
  T acc = 0;
  if (c < k) {
    if (scale) {
      for (int64_t j = s; j < e; ++j) {
        const int32_t q = col[j];
        acc += static_cast<T>(val[j]) * (scale[q] * X[static_cast<int64_t>(q) * ld + c]);
      }
      acc *= scale[row];
    } else {
      for (int64_t j = s; j < e; ++j) {
        const int32_t q = col[j];
        acc += static_cast<T>(val[j]) * X[static_cast<int64_t>(q) * ld + c];
      }
    }
    Y[row * ld + c] = acc;
  }
}

template <typename VT, typename XT, typename AT, typename YT>
void spmv_impl(gp_ctx* c, const gp_matrix* m, const XT* x, YT* y) {
  const VT* val = static_cast<const VT*>(m->val);
  const unsigned nb_short = grid_for(m->n * kG, kThreads);
  const unsigned nb_long = m->n_long > 0 ? grid_for(m->n_long * kWave, kThreads) : 0;
  ProfScope ps(c, sizeof(VT) == 4 ? (sizeof(XT) == 4 ? "spmv_f32" : "spmv_f32val_f64") : "spmv_f64");
  hipLaunchKernelGGL((k_spmv<VT, XT, AT, YT>), dim3(nb_short + nb_long), dim3(kThreads), 0, c->stream, m->n,
                     nb_short, m->n_long, m->long_rows, m->row_ptr, m->col, val, x, y);
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
  if (k > 32) throw Error{GP_EINVAL, "spmm: at most 32 right-hand sides per call"};
  ProfScope ps(c, "spmm");
  if (m->prec == GP_MIXED)
    hipLaunchKernelGGL((k_spmm<float, T>), dim3(grid_for(m->n * 32, kThreads)), dim3(kThreads), 0, c->stream, m->n, k,
                       ld, m->row_ptr, m->col, static_cast<const float*>(m->val), X, Y, scale);
  else
    hipLaunchKernelGGL((k_spmm<double, T>), dim3(grid_for(m->n * 32, kThreads)), dim3(kThreads), 0, c->stream, m->n,
                       k, ld, m->row_ptr, m->col, static_cast<const double*>(m->val), X, Y, scale);
  check_launch("spmm");
}

template void spmm<float>(gp_ctx*, const gp_matrix*, int, int, const float*, float*, const float*);
template void spmm<double>(gp_ctx*, const gp_matrix*, int, int, const double*, double*, const double*);

}  // namespace gps
