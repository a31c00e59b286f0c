// Block-Jacobi preconditioner for the conjugate-gradient solve.
//
// Blocks are the cells of the dataset's spatial hash: the points of a cell
// are consecutive in binned order, so each block is a diagonal block
// K[bs:be, bs:be] of the matrix.  Cells holding more than kMaxBlock points are
// split into consecutive pieces of at most kMaxBlock.  Every diagonal block of
// the symmetric positive-definite K is itself positive definite, so the
// block-diagonal M = blkdiag(K_bb) is a valid preconditioner; it captures the
// strongest couplings (nearest neighbours within a cell) that the point
// Jacobi preconditioner ignores.  Each block's inverse is formed once per
// matrix in float64 (Gauss-Jordan without pivoting, one wave per block, lane i
// holding row i) and applied as a small dense product per row.
#include <algorithm>
#include <type_traits>

#include "device.hpp"

namespace gps {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlock = 32;

// flag[p] = 1 when p starts a block (first point of its cell, or every
// kMaxBlock-th point inside a large cell)
__global__ void __launch_bounds__(kThreads) k_block_flags(int64_t n, const int32_t* __restrict__ key,
                                                          const int32_t* __restrict__ cell_start,
                                                          int32_t* __restrict__ flag) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (p >= n) return;
  const int64_t off = p - cell_start[key[p]];
  flag[p] = (off % kMaxBlock) == 0 ? 1 : 0;
}

__global__ void __launch_bounds__(kThreads) k_block_starts(int64_t n, const int32_t* __restrict__ flag,
                                                           const int32_t* __restrict__ pos,
                                                           int32_t* __restrict__ bstart, int32_t* __restrict__ rowblk,
                                                           int32_t* __restrict__ bsq) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (p >= n) return;
  // block of p: the last start at or before p
  const int32_t b = pos[p] + flag[p] - 1;
  rowblk[p] = b;
  if (flag[p]) bstart[b] = static_cast<int32_t>(p);
}

__global__ void __launch_bounds__(kThreads) k_block_sizes(int64_t nblk, int64_t n, int32_t* __restrict__ bstart,
                                                          int32_t* __restrict__ bsq) {
  const int64_t b = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (b > nblk) return;
  if (b == nblk) {
    bstart[nblk] = static_cast<int32_t>(n);
    return;
  }
  const int64_t e = (b + 1 < nblk) ? bstart[b + 1] : n;
  const int64_t sz = e - bstart[b];
  bsq[b] = static_cast<int32_t>(sz * sz);
}

// Gauss-Jordan inversion of the diagonal blocks with BS lanes per block (a
// wave takes 64 / BS blocks): lane i of the group holds row i of the block.
// One launch per size class takes the blocks with BS/2 < size <= BS (BS = 4
// also takes sizes 1..2), so the work follows the block's own size.  The
// dense block is gathered from the CSR (its columns are a contiguous run of
// each of the row's two ascending runs: group entries, then the rest).
template <typename VT, int BS>
__global__ void __launch_bounds__(kThreads) k_block_invert(int64_t nblk, const int32_t* __restrict__ bstart,
                                                           const int64_t* __restrict__ boff,
                                                           const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ gskip,
                                                           const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                           double* __restrict__ binv, int* __restrict__ bad) {
  const int64_t g = (blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x) / BS;
  const int lane = threadIdx.x % BS;
  // every lane of a group sees the same block; groups past the end or of
  // another size class take no part but still join the shuffles (width BS)
  int32_t bs = 0;
  int sz = 0;
  if (g < nblk) {
    bs = bstart[g];
    sz = bstart[g + 1] - bs;
  }
  const bool mine = g < nblk && sz <= BS && (BS == 4 ? true : sz > BS / 2);
  if (__ballot(mine) == 0) return;  // uniform: no block of this class in the wave
  double a[BS];
#pragma unroll
  for (int j = 0; j < BS; ++j) a[j] = 0.0;
  if (mine && lane < sz) {
    const int32_t row = bs + lane;
    const int64_t runs[3] = {rp[row], rp[row] + gskip[row], rp[row + 1]};
    for (int rr = 0; rr < 2; ++rr) {
      int64_t lo = runs[rr], hi = runs[rr + 1];
      while (lo < hi) {  // first entry with column >= bs
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < bs)
          lo = mid + 1;
        else
          hi = mid;
      }
      for (int64_t j = lo; j < runs[rr + 1]; ++j) {
        const int32_t cidx = col[j] - bs;
        if (cidx >= sz) break;
#pragma unroll
        for (int t = 0; t < BS; ++t)
          if (t == cidx) a[t] = static_cast<double>(val[j]);
      }
    }
  }
  // in-place Gauss-Jordan inversion (symmetric positive definite: no pivoting)
  bool ok = true;
  const int steps = mine ? sz : 0;
  int wsteps = steps;  // pivots needed by any group of the wave
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) wsteps = max(wsteps, __shfl_xor(wsteps, off, kWave));
  for (int k = 0; k < wsteps; ++k) {
    double rk[BS];
#pragma unroll
    for (int j = 0; j < BS; ++j) rk[j] = __shfl(a[j], k, BS);
    if (k >= steps) continue;  // uniform within the group
    double piv = 0.0;
#pragma unroll
    for (int j = 0; j < BS; ++j)
      if (j == k) piv = rk[j];
    if (!(piv > 0.0)) ok = false;
    const double ip = 1.0 / piv;
    // pivot row: a[k][j] /= piv, a[k][k] = 1 / piv
#pragma unroll
    for (int j = 0; j < BS; ++j) rk[j] = (j == k) ? ip : rk[j] * ip;
    if (lane == k) {
#pragma unroll
      for (int j = 0; j < BS; ++j) a[j] = rk[j];
    } else if (lane < sz) {
      double f = 0.0;
#pragma unroll
      for (int j = 0; j < BS; ++j)
        if (j == k) f = a[j];
#pragma unroll
      for (int j = 0; j < BS; ++j) a[j] = (j == k) ? -f * ip : a[j] - f * rk[j];
    }
  }
  if (mine && !ok && lane == 0) atomicOr(bad, 1);
  if (mine && lane < sz) {
    double* out = binv + boff[g] + static_cast<int64_t>(lane) * sz;
#pragma unroll
    for (int j = 0; j < BS; ++j)
      if (j < sz) out[j] = a[j];
  }
}

}  // namespace

static void build_block_jacobi_impl(gp_ctx* c, gp_matrix* m);

void build_block_jacobi(gp_ctx* c, gp_matrix* m) {
  if (m->binv) return;
  // a failure (allocation, non-positive pivot) leaves no partial state behind,
  // so a later call builds the preconditioner again from scratch
  try {
    build_block_jacobi_impl(c, m);
  } catch (...) {
    free_block_jacobi(c, m);
    throw;
  }
}

static void build_block_jacobi_impl(gp_ctx* c, gp_matrix* m) {
  const gp_dataset* ds = m->ds;
  const int64_t n = m->n;
  int32_t* flag = static_cast<int32_t*>(workspace(c, 70, sizeof(int32_t) * n));
  int32_t* pos = static_cast<int32_t*>(workspace(c, 71, sizeof(int32_t) * (n + 1)));
  hipLaunchKernelGGL(k_block_flags, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, n, ds->key,
                     ds->cell_start, flag);
  check_launch("block flags");
  scan_i32_to_i32(c, flag, pos, n);
  int32_t* h = static_cast<int32_t*>(pinned(c, sizeof(int32_t)));
  GPS_HIP(hipMemcpyAsync(h, pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  const int64_t nblk = *h;
  m->nblk = nblk;
  m->bstart = dev_new<int32_t>(c, nblk + 1);
  m->rowblk = dev_new<int32_t>(c, n);
  m->boff = dev_new<int64_t>(c, nblk + 1);
  int32_t* bsq = static_cast<int32_t*>(workspace(c, 72, sizeof(int32_t) * std::max<int64_t>(nblk, 1)));
  hipLaunchKernelGGL(k_block_starts, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, n, flag, pos,
                     m->bstart, m->rowblk, bsq);
  hipLaunchKernelGGL(k_block_sizes, dim3(grid_for(nblk + 1, kThreads)), dim3(kThreads), 0, c->stream, nblk, n,
                     m->bstart, bsq);
  check_launch("block sizes");
  scan_i32_to_i64(c, bsq, m->boff, nblk);
  const int64_t total = read_i64(c, m->boff + nblk);
  m->binv_len = total;
  m->binv = dev_new<double>(c, std::max<int64_t>(total, 1));
  GPS_HIP(hipMemsetAsync(c->err_flag, 0, sizeof(int), c->stream));
  {
    ProfScope ps(c, "precond_setup");
    auto go = [&](auto vt) {
      using VT = decltype(vt);
      const VT* val = static_cast<const VT*>(m->val);
      auto one = [&](auto bsz) {
        constexpr int BS = decltype(bsz)::value;
        hipLaunchKernelGGL((k_block_invert<VT, BS>), dim3(grid_for(nblk * BS, kThreads)), dim3(kThreads), 0,
                           c->stream, nblk, m->bstart, m->boff, m->row_ptr, m->gskip, m->col, val, m->binv,
                           c->err_flag);
      };
      one(std::integral_constant<int, 4>{});
      one(std::integral_constant<int, 8>{});
      one(std::integral_constant<int, 16>{});
      one(std::integral_constant<int, 32>{});
    };
    if (m->prec == GP_MIXED)
      go(float{});
    else
      go(double{});
    check_launch("block inverse");
  }
  int* herr = static_cast<int*>(pinned(c, sizeof(int)));
  GPS_HIP(hipMemcpyAsync(herr, c->err_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  if (*herr) throw Error{GP_ENOTPD, "block-Jacobi setup met a non-positive pivot: matrix not positive definite"};
  m->bytes += sizeof(int32_t) * (nblk + 1 + n) + sizeof(int64_t) * (nblk + 1) + sizeof(double) * total;
}

void free_block_jacobi(gp_ctx* c, gp_matrix* m) {
  if (m->bstart) dev_free(c, m->bstart, sizeof(int32_t) * (m->nblk + 1));
  if (m->rowblk) dev_free(c, m->rowblk, sizeof(int32_t) * m->n);
  if (m->boff) dev_free(c, m->boff, sizeof(int64_t) * (m->nblk + 1));
  if (m->binv) dev_free(c, m->binv, sizeof(double) * std::max<int64_t>(m->binv_len, 1));
  m->bstart = m->rowblk = nullptr;
  m->boff = nullptr;
  m->binv = nullptr;
}

}  // namespace gps
