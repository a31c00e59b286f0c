// Export of the binned CSR in original point order with ascending columns,
// and original-order permutations of vectors (debug / parity paths).
#include <algorithm>

#include "device.hpp"

namespace gps {
namespace {

constexpr int kThreads = 256;

__global__ void k_orig_lengths(int64_t n, const int32_t* __restrict__ iperm, const int64_t* __restrict__ rp,
                               int32_t* __restrict__ len) {
  const int64_t o = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (o >= n) return;
  const int32_t p = iperm[o];
  len[o] = static_cast<int32_t>(rp[p + 1] - rp[p]);
}

// One wave per original row: copy the row with columns mapped to original ids.
template <typename VT>
__global__ void k_copy_rows(int64_t n, const int32_t* __restrict__ iperm, const int32_t* __restrict__ perm,
                            const int64_t* __restrict__ rp, const int32_t* __restrict__ col, const VT* __restrict__ val,
                            const int64_t* __restrict__ orp, int32_t* __restrict__ tcol, double* __restrict__ tval) {
  const int64_t o = (blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x) / kWave;
  if (o >= n) return;
  const int32_t p = iperm[o];
  const int64_t s = rp[p], len = rp[p + 1] - rp[p], d = orp[o];
  for (int64_t j = lane_id(); j < len; j += kWave) {
    tcol[d + j] = perm[col[s + j]];
    tval[d + j] = static_cast<double>(val[s + j]);
  }
}

// One wave per row: rank sort of the (unique) column ids from the staging copy.
__global__ void k_sort_rows(int64_t n, const int64_t* __restrict__ orp, const int32_t* __restrict__ tcol,
                            const double* __restrict__ tval, int32_t* __restrict__ col, double* __restrict__ val) {
  const int64_t o = (blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x) / kWave;
  if (o >= n) return;
  const int64_t s = orp[o], len = orp[o + 1] - orp[o];
  for (int64_t j = lane_id(); j < len; j += kWave) {
    const int32_t v = tcol[s + j];
    int64_t rank = 0;
    for (int64_t b = 0; b < len; ++b) rank += tcol[s + b] < v ? 1 : 0;
    col[s + rank] = v;
    val[s + rank] = tval[s + j];
  }
}

template <typename T>
__global__ void k_to_binned(int64_t n, int k, const int32_t* __restrict__ perm, const T* __restrict__ x,
                            T* __restrict__ xb) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i >= n * k) return;
  const int64_t p = i / k, c = i % k;
  xb[i] = x[static_cast<int64_t>(perm[p]) * k + c];
}

template <typename T>
__global__ void k_to_orig(int64_t n, int k, const int32_t* __restrict__ perm, const T* __restrict__ yb,
                          T* __restrict__ y) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i >= n * k) return;
  const int64_t p = i / k, c = i % k;
  y[static_cast<int64_t>(perm[p]) * k + c] = yb[i];
}

}  // namespace

void export_csr(gp_ctx* c, const gp_matrix* m, int64_t* row_ptr, int32_t* col, double* val) {
  const int64_t n = m->n;
  const gp_dataset* ds = m->ds;
  TmpBuf len(c, sizeof(int32_t) * n);
  hipLaunchKernelGGL(k_orig_lengths, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, n, ds->iperm,
                     m->row_ptr, len.as<int32_t>());
  check_launch("export lengths");
  scan_i32_to_i64(c, len.as<int32_t>(), row_ptr, n);
  TmpBuf tcol(c, sizeof(int32_t) * std::max<int64_t>(m->nnz, 1));
  TmpBuf tval(c, sizeof(double) * std::max<int64_t>(m->nnz, 1));
  if (m->prec == GP_MIXED)
    hipLaunchKernelGGL((k_copy_rows<float>), dim3(grid_for(n * kWave, kThreads)), dim3(kThreads), 0, c->stream, n,
                       ds->iperm, ds->perm, m->row_ptr, m->col, static_cast<const float*>(m->val), row_ptr,
                       tcol.as<int32_t>(), tval.as<double>());
  else
    hipLaunchKernelGGL((k_copy_rows<double>), dim3(grid_for(n * kWave, kThreads)), dim3(kThreads), 0, c->stream, n,
                       ds->iperm, ds->perm, m->row_ptr, m->col, static_cast<const double*>(m->val), row_ptr,
                       tcol.as<int32_t>(), tval.as<double>());
  check_launch("export copy");
  hipLaunchKernelGGL(k_sort_rows, dim3(grid_for(n * kWave, kThreads)), dim3(kThreads), 0, c->stream, n, row_ptr,
                     tcol.as<int32_t>(), tval.as<double>(), col, val);
  check_launch("export sort");
  sync(c);
}

template <typename T>
void permute_to_binned(gp_ctx* c, const gp_dataset* ds, int k, const T* x, T* xb) {
  hipLaunchKernelGGL((k_to_binned<T>), dim3(grid_for(ds->n * k, kThreads)), dim3(kThreads), 0, c->stream, ds->n, k,
                     ds->perm, x, xb);
  check_launch("to binned");
}

template <typename T>
void permute_to_orig(gp_ctx* c, const gp_dataset* ds, int k, const T* yb, T* y) {
  hipLaunchKernelGGL((k_to_orig<T>), dim3(grid_for(ds->n * k, kThreads)), dim3(kThreads), 0, c->stream, ds->n, k,
                     ds->perm, yb, y);
  check_launch("to original");
}

template void permute_to_binned<double>(gp_ctx*, const gp_dataset*, int, const double*, double*);
template void permute_to_orig<double>(gp_ctx*, const gp_dataset*, int, const double*, double*);

}  // namespace gps
