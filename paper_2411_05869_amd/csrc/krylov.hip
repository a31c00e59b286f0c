// Krylov drivers: Jacobi-preconditioned conjugate gradients for y^T K^-1 y,
// stochastic Lanczos quadrature for log det K, and an exact Lanczos log-det
// with full re-orthogonalisation for small n (Sec. 3.3: the log-determinant
// and linear-solve tasks).
//
// Reductions are two-level with a fixed grid and a fixed tree (reduce.hpp), so
// every scalar is bitwise reproducible.  Scalars stay in device memory between
// kernels; the host reads them only at check points.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "device.hpp"
#include "reduce.hpp"

namespace gps {
namespace {

constexpr int kThreads = kRedThreads;
constexpr int kRedBlocks = 512;
constexpr int kCheckEvery = 8;
constexpr int kLoadBatch = 4;  // strided elements a thread loads at once in the streaming kernels

// A batched solve stacks independent problems along the rows (a block-diagonal
// matrix, vectors concatenated); blockIdx.y selects the problem.  Every
// problem keeps the grid, the partial-sum layout and the reduction order a
// solve of its own length uses, so its scalars equal that solve's bitwise.
// off == nullptr: one problem, of the length the kernel is given.
struct Seg {
  const int64_t* off = nullptr;  // problems + 1 row offsets into the stacked vectors
  int pstride = 0;               // doubles between the partial-sum arrays of consecutive problems
};

// first row of this block's problem; n becomes its length
__device__ __forceinline__ int64_t seg_begin(const Seg& g, int64_t& n) {
  if (!g.off) return 0;
  const int64_t b = g.off[blockIdx.y];
  n = g.off[blockIdx.y + 1] - b;
  return b;
}

// blocks of a per-row grid of a problem of n rows (grid_for on the device)
__device__ __forceinline__ int seg_blocks(int64_t n, int per_block) {
  const int64_t b = (n + per_block - 1) / per_block;
  return static_cast<int>(b < 1 ? 1 : b);
}

// ---------------------------------------------------------------- reductions
__global__ void __launch_bounds__(kThreads) k_dot_part(int64_t n, const double* __restrict__ a,
                                                       const double* __restrict__ b, double* __restrict__ part,
                                                       Seg g = {}) {
  const int64_t o = seg_begin(g, n);
  a += o;
  b += o;
  part += blockIdx.y * g.pstride;
  double v[1] = {0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    v[0] += a[i] * b[i];
  block_sum_store<1>(v, part);
}

__global__ void __launch_bounds__(kThreads) k_sum_part(const double* __restrict__ part, int nb, double* __restrict__ out,
                                                       Seg g = {}) {
  part += blockIdx.y * g.pstride;
  double r[1];
  reduce_partials<1>(part, nb, r);
  if (threadIdx.x == 0) out[blockIdx.y] = r[0];
}

__global__ void __launch_bounds__(kThreads) k_logsum_part(int64_t n, const double* __restrict__ a,
                                                          double* __restrict__ part, Seg g = {}) {
  a += seg_begin(g, n);
  part += blockIdx.y * g.pstride;
  double v[1] = {0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    v[0] += log(a[i]);
  block_sum_store<1>(v, part);
}

// ---------------------------------------------------------------- PCG
struct CgScalars {
  double rz, rz_old, pq, alpha, beta, rr, yy, pad;
  int status;  // 0 ok, 1 non-positive curvature / non-finite
};

// The skip flags of a device-driven solve (CgCtl, one per problem of a batch)
// are read by every kernel of the iterations: a kernel returns at once while
// its problem's flag is set.
constexpr int kCtlInts = static_cast<int>(sizeof(CgCtl) / sizeof(int));  // flag stride between problems
static_assert(sizeof(CgCtl) % sizeof(int) == 0, "CgCtl is a whole number of ints");

// this block's problem's skip flag (null: never skip)
__device__ __forceinline__ bool seg_skip(const int* skip) {
  return skip && skip[blockIdx.y * kCtlInts];
}

// Preconditioner description passed to the kernels (block Jacobi if binv != null,
// otherwise point Jacobi with the matrix diagonal).
struct Precond {
  const double* diag;
  const int32_t* rowblk;
  const int32_t* bstart;
  const int64_t* boff;
  const double* binv;
};

__device__ __forceinline__ double precond_row(const Precond& M, const double* __restrict__ r, int64_t i) {
  if (!M.binv) return r[i] / M.diag[i];
  const int32_t b = M.rowblk[i];
  const int32_t bs = M.bstart[b];
  const int sz = M.bstart[b + 1] - bs;
  const double* row = M.binv + M.boff[b] + static_cast<int64_t>(i - bs) * sz;
  double z = 0.0;
  for (int j = 0; j < sz; ++j) z += row[j] * r[bs + j];
  return z;
}

// One CG step after the product q = K p.  Every block adds the kRedBlocks
// partials of p.q (pq_part, same fixed order in every block) and forms alpha =
// rz / pq; then, kStepRows rows per thread (the block-Jacobi product is a
// short chain of dependent gathers, so a nearly full grid keeps enough of them
// in flight):
// x += alpha p, rn = r - alpha q, z = M^-1 rn, and per-block partials of rn.z and
// rn.rn.  Block 0 records pq, alpha, rz_old = rz and the status (non-positive
// curvature).
constexpr int kStepRows = 2;
constexpr int kPreEntries = 4;  // block entries per row loaded before alpha is known (blocks average 2.8 points)

template <typename QT>
__global__ void __launch_bounds__(kThreads) k_pcg_step(int64_t n, Precond M, CgScalars* __restrict__ s,
                                                       const double* __restrict__ pq_part,
                                                       const double* __restrict__ p, const QT* __restrict__ q,
                                                       double* __restrict__ x, const double* __restrict__ r,
                                                       double* __restrict__ rn, double* __restrict__ z,
                                                       double* __restrict__ part, const int* __restrict__ skip,
                                                       Seg g = {}) {
  if (seg_skip(skip)) return;
  solve_wave_priority();
  const int64_t o = seg_begin(g, n);
  if (g.off && static_cast<int>(blockIdx.x) >= seg_blocks(n, kThreads * kStepRows)) return;
  const int64_t e = o + n;  // rows o .. e of the stacked vectors (the preconditioner is indexed by stacked rows)
  s += blockIdx.y;
  pq_part += blockIdx.y * g.pstride;
  part += blockIdx.y * g.pstride;
  // Everything a row reads is independent of alpha, so the row's vectors, its
  // block (row -> block -> start and offset) and the block's first kPreEntries
  // weights and r, q values are requested before the kRedBlocks partials of
  // p.q are reduced; the arithmetic afterwards is the same, in the same order.
  // Row i of z = M^-1 (r - alpha q) forms the block's entries of the new
  // residual from r and q the same way as the row's own, so every thread sees
  // bitwise the same values without waiting for the others.
  double xv[kStepRows], pv[kStepRows], rv[kStepRows], qv[kStepRows], dv[kStepRows];
  constexpr int kPreSlots = kPreEntries > 0 ? kPreEntries : 1;
  double wpre[kStepRows][kPreSlots], rpre[kStepRows][kPreSlots], qpre[kStepRows][kPreSlots];
  const double* brow[kStepRows];
  int32_t bs[kStepRows];
  int sz[kStepRows];
#pragma unroll
  for (int u = 0; u < kStepRows; ++u) {
    const int64_t i = o + (blockIdx.x * static_cast<int64_t>(kStepRows) + u) * kThreads + threadIdx.x;
    sz[u] = 0;
    if (i < e) {
      xv[u] = x[i];
      pv[u] = p[i];
      rv[u] = r[i];
      qv[u] = static_cast<double>(q[i]);
      if (M.binv) {
        const int32_t b = M.rowblk[i];
        bs[u] = M.bstart[b];
        sz[u] = M.bstart[b + 1] - bs[u];
        brow[u] = M.binv + M.boff[b] + static_cast<int64_t>(i - bs[u]) * sz[u];
#pragma unroll
        for (int j = 0; j < kPreEntries; ++j) {
          if (j < sz[u]) {
            wpre[u][j] = brow[u][j];
            rpre[u][j] = r[bs[u] + j];
            qpre[u][j] = static_cast<double>(q[bs[u] + j]);
          }
        }
      } else {
        dv[u] = M.diag[i];
      }
    }
  }
  double pqv[1];
  reduce_partials<1>(pq_part, kRedBlocks, pqv);
  const double pq = pqv[0], rz = s->rz;
  const bool ok = pq > 0.0 && isfinite(pq);
  const double alpha = ok ? rz / pq : 0.0;
  double v[2] = {0, 0};
#pragma unroll
  for (int u = 0; u < kStepRows; ++u) {
    const int64_t i = o + (blockIdx.x * static_cast<int64_t>(kStepRows) + u) * kThreads + threadIdx.x;
    if (i < e) {
      x[i] = xv[u] + alpha * pv[u];
      const double ri = rv[u] - alpha * qv[u];
      double zi;
      if (M.binv) {
        // z_i = sum_j binv[i][j] (r_j - alpha q_j) over the block, j ascending
        zi = 0.0;
#pragma unroll
        for (int j = 0; j < kPreEntries; ++j)
          if (j < sz[u]) zi += wpre[u][j] * (rpre[u][j] - alpha * qpre[u][j]);
        for (int j = kPreEntries; j < sz[u]; ++j)
          zi += brow[u][j] * (r[bs[u] + j] - alpha * static_cast<double>(q[bs[u] + j]));
      } else {
        zi = ri / dv[u];
      }
      rn[i] = ri;
      z[i] = zi;
      v[0] += ri * zi;
      v[1] += ri * ri;
    }
  }
  block_sum_store<2>(v, part);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s->pq = pq;
    s->alpha = alpha;
    s->rz_old = rz;
    if (!ok) s->status = 1;
  }
}

// New direction after a step: every block adds the step's nb partials (same
// fixed order) into rz, rr and beta = rz / rz_old, then p = z + beta p.  Block
// 0 records rz, rr, beta and flags non-finite values.
__global__ void __launch_bounds__(kThreads) k_pcg_direction(int64_t n, CgScalars* __restrict__ s,
                                                            const double* __restrict__ part, int nb,
                                                            const double* __restrict__ z, double* __restrict__ p,
                                                            const int* __restrict__ skip, Seg g = {}) {
  if (seg_skip(skip)) return;
  solve_wave_priority();
  const int64_t o = seg_begin(g, n);
  if (g.off) nb = seg_blocks(n, kThreads * kStepRows);  // the step's partials of this problem
  z += o;
  p += o;
  s += blockIdx.y;
  part += blockIdx.y * g.pstride;
  // the first batch of z and p is requested before the partial sums are
  // reduced, and each later batch before the previous one is stored
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  const int64_t i0 = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  double zv[kLoadBatch], pv[kLoadBatch];
  auto load = [&](int64_t i) {
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int64_t k = i + u * stride;
      zv[u] = k < n ? z[k] : 0.0;
      pv[u] = k < n ? p[k] : 0.0;
    }
  };
  load(i0);
  double sums[2];
  reduce_partials<2>(part, nb, sums);
  const double beta = sums[0] / s->rz_old;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s->rz = sums[0];
    s->rr = sums[1];
    s->beta = beta;
    if (!isfinite(sums[0]) || !isfinite(sums[1])) s->status = 1;
  }
  for (int64_t i = i0; i < n; i += kLoadBatch * stride) {
    double out[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) out[u] = zv[u] + beta * pv[u];
    if (i + kLoadBatch * stride < n) load(i + kLoadBatch * stride);
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u)
      if (i + u * stride < n) p[i + u * stride] = out[u];
  }
}

// x = 0, r = y; partial sums of y.y
__global__ void __launch_bounds__(kThreads) k_pcg_init(int64_t n, const double* __restrict__ y, double* __restrict__ x,
                                                       double* __restrict__ r, double* __restrict__ part, Seg g = {}) {
  const int64_t o = seg_begin(g, n);
  y += o;
  x += o;
  r += o;
  part += blockIdx.y * g.pstride;
  double v[1] = {0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double yi = y[i];
    x[i] = 0.0;
    r[i] = yi;
    v[0] += yi * yi;
  }
  block_sum_store<1>(v, part);
}

__global__ void __launch_bounds__(kThreads) k_yy_fin(const double* __restrict__ part, int nb, CgScalars* __restrict__ s,
                                                     Seg g = {}) {
  part += blockIdx.y * g.pstride;
  s += blockIdx.y;
  double r[1];
  reduce_partials<1>(part, nb, r);
  if (threadIdx.x == 0) {
    s->yy = r[0];
    s->status = 0;
  }
}

// z = M^-1 r, one thread per row (full grid: the block products are short,
// dependent gathers); per-block partial sums of r.z and r.r
__global__ void __launch_bounds__(kThreads) k_precond(int64_t n, Precond M, const double* __restrict__ r,
                                                      double* __restrict__ z, double* __restrict__ part,
                                                      const int* __restrict__ skip = nullptr, Seg g = {}) {
  if (seg_skip(skip)) return;
  const int64_t o = seg_begin(g, n);
  if (g.off && static_cast<int>(blockIdx.x) >= seg_blocks(n, kThreads)) return;
  part += blockIdx.y * g.pstride;
  double v[2] = {0, 0};
  const int64_t i = o + blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;  // stacked row
  if (i < o + n) {
    const double ri = r[i];
    const double zi = precond_row(M, r, i);
    z[i] = zi;
    v[0] = ri * zi;
    v[1] = ri * ri;
  }
  block_sum_store<2>(v, part);
}

// per-block partials of p.q (kRedBlocks blocks, grid-stride)
template <typename QT>
__global__ void __launch_bounds__(kThreads) k_pq_part(int64_t n, const double* __restrict__ p,
                                                      const QT* __restrict__ q, double* __restrict__ part,
                                                      const int* __restrict__ skip, Seg g = {}) {
  if (seg_skip(skip)) return;
  solve_wave_priority();
  const int64_t o = seg_begin(g, n);
  p += o;
  q += o;
  part += blockIdx.y * g.pstride;
  // four strided elements loaded at once, then added in the order of a plain
  // grid-stride loop (the sum does not depend on the unrolling)
  double v[1] = {0};
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n; i += kLoadBatch * stride) {
    double pv[kLoadBatch], qv[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int64_t k = i + u * stride;
      pv[u] = k < n ? p[k] : 0.0;
      qv[u] = k < n ? static_cast<double>(q[k]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u)
      if (i + u * stride < n) v[0] += pv[u] * qv[u];
  }
  block_sum_store<1>(v, part);
}

// mode 0: iteration (rz_old <- rz, rz <- r.z, beta = rz / rz_old)
// mode 3: iteration whose step already set rz_old

// mode 1: residual replacement (rz_old kept)
// mode 2: start (rz <- r.z, no beta)
// (batched: per_block = rows per partial of the kernel that wrote them)
__global__ void __launch_bounds__(kThreads) k_beta_fin(const double* __restrict__ part, int nb,
                                                       CgScalars* __restrict__ s, int mode,
                                                       const int* __restrict__ skip = nullptr, Seg g = {},
                                                       int per_block = 0) {
  if (seg_skip(skip)) return;
  int64_t n = 0;
  seg_begin(g, n);
  if (g.off) nb = seg_blocks(n, per_block);
  part += blockIdx.y * g.pstride;
  s += blockIdx.y;
  double r[2];
  reduce_partials<2>(part, nb, r);
  if (threadIdx.x == 0) {
    if (mode == 0) s->rz_old = s->rz;  // mode 3: set by the step
    s->rz = r[0];
    s->rr = r[1];
    s->beta = mode == 2 ? 0.0 : r[0] / s->rz_old;
    if (!isfinite(r[0]) || !isfinite(r[1])) s->status = 1;
  }
}

// p = z + beta p (beta = 0 at the start)
__global__ void __launch_bounds__(kThreads) k_pcg_pupdate(int64_t n, const CgScalars* __restrict__ s,
                                                          const double* __restrict__ z, double* __restrict__ p,
                                                          const int* __restrict__ skip = nullptr, Seg g = {}) {
  if (seg_skip(skip)) return;
  const int64_t o = seg_begin(g, n);
  z += o;
  p += o;
  const double beta = s[blockIdx.y].beta;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    p[i] = beta == 0.0 ? z[i] : z[i] + beta * p[i];
}

// r = y - Kx (Kx given)
__global__ void __launch_bounds__(kThreads) k_true_resid(int64_t n, const double* __restrict__ y,
                                                         const double* __restrict__ kx, double* __restrict__ r,
                                                         const int* __restrict__ skip = nullptr, Seg g = {}) {
  if (seg_skip(skip)) return;
  const int64_t o = seg_begin(g, n);
  y += o;
  kx += o;
  r += o;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    r[i] = y[i] - kx[i];
}

// ---------------------------------------------------------------- Lanczos
__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Probe entry for (seed, probe, original index): sign of the SplitMix64 output at
// counter (probe << 40 | index) + 1 of the generator started at state seed.
__device__ __forceinline__ double rademacher(uint64_t seed, uint64_t probe, uint64_t idx) {
  const uint64_t k = ((probe << 40) | idx) + 1ull;
  const uint64_t out = splitmix_mix(seed + k * 0x9E3779B97F4A7C15ull);
  return (out >> 63) ? -1.0 : 1.0;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_lz_init(int64_t n, int k, int ld, int probe0, uint64_t seed,
                                                      const int32_t* __restrict__ perm, T* __restrict__ V,
                                                      T* __restrict__ Vprev) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i >= n * ld) return;
  const int64_t p = i / ld;
  const int l = static_cast<int>(i % ld);
  T v = 0;
  if (l < k) v = static_cast<T>(rademacher(seed, static_cast<uint64_t>(probe0 + l), static_cast<uint64_t>(perm[p])));
  V[i] = v;
  Vprev[i] = 0;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_scale_vec(int64_t n, const double* __restrict__ diag,
                                                        T* __restrict__ s) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i < n) s[i] = static_cast<T>(1.0 / sqrt(diag[i]));
}

// The Lanczos vectors are kept unnormalised: v_j = w_{j-1} * inv_cur, with w the
// residual block of the previous step, so no pass normalises them; the products
// and the alpha / beta kernels apply the factor where v is read.
struct LzState {
  double alpha[32];
  double beta[32];       // beta of the current step (norm of W)
  double beta_prev[32];  // used by the next step
  double inv_cur[32];    // v_j = Vcur * inv_cur (0 for finished probes)
  double inv_prev[32];   // v_{j-1} = Vprev * inv_prev
  double dcorr[32];      // w_{j-1} . v_{j-1} of the previous step
  int active[32];
  int steps[32];
};

// A Lanczos step makes two passes over the blocks after the product.  The
// product W = S K S V (v_j = V inv_cur) is not scaled by inv_cur;
// k_lz_vw_part forms partial sums of V[:, l] . W[:, l], and
// alpha_j = v_j . (A v_j - beta_j v_{j-1}) is then inv_cur^2 times their
// total minus w_{j-1} . v_{j-1}, the term kept from the previous step
// (v_j = w_{j-1} / beta_j), so that the second pass applies inv_cur and both
// subtractions at once (in exact arithmetic the same alpha as subtracting
// beta_j v_{j-1} before the dot product).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_lz_vw_part(int64_t n, int ld, const T* __restrict__ V,
                                                         const T* __restrict__ W, double* __restrict__ part,
                                                         Seg g = {}) {
  const int64_t o = seg_begin(g, n) * ld;
  V += o;
  W += o;
  part += blockIdx.y * g.pstride;
  const int l = threadIdx.x & 31;
  const int rl = threadIdx.x >> 5;
  double acc = 0;
  const int64_t S = static_cast<int64_t>(gridDim.x) * 8;
  int64_t p = blockIdx.x * 8ll + rl;
  for (; p + 3 * S < n; p += 4 * S) {
    T wv[4], vv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = (p + u * S) * ld + l;
      wv[u] = W[i];
      vv[u] = V[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += static_cast<double>(vv[u]) * static_cast<double>(wv[u]);
  }
  for (; p < n; p += S) {
    const int64_t i = p * ld + l;
    acc += static_cast<double>(V[i]) * static_cast<double>(W[i]);
  }
  __shared__ double sh[8][32];
  sh[rl][l] = acc;
  __syncthreads();
  if (rl == 0) {
    double t = 0;
    for (int j = 0; j < 8; ++j) t += sh[j][l];
    part[blockIdx.x * 32 + l] = t;
  }
}

// W holds S K S V without the factor inv_cur of v_j:
// W[:, l] = (W inv_cur - beta_prev v_{j-1}) - alpha v_j; partial sums of
// |W[:, l]|^2 at part[b * 64 + l] and of W[:, l] . V[:, l] (unnormalised v_j)
// at part[b * 64 + 32 + l]
template <typename T>
__global__ void __launch_bounds__(kThreads) k_lz_update(int64_t n, int ld, const LzState* __restrict__ st,
                                                        const T* __restrict__ V, const T* __restrict__ Vprev,
                                                        T* __restrict__ W, double* __restrict__ part, Seg g = {}) {
  const int64_t o = seg_begin(g, n) * ld;
  V += o;
  Vprev += o;
  W += o;
  st += blockIdx.y;
  part += blockIdx.y * g.pstride;
  const int l = threadIdx.x & 31;
  const int rl = threadIdx.x >> 5;
  const T a = static_cast<T>(st->alpha[l]), bp = static_cast<T>(st->beta_prev[l]);
  const T ic = static_cast<T>(st->inv_cur[l]), ip = static_cast<T>(st->inv_prev[l]);
  double an = 0, ad = 0;
  const int64_t S = static_cast<int64_t>(gridDim.x) * 8;
  int64_t p = blockIdx.x * 8ll + rl;
  for (; p + 3 * S < n; p += 4 * S) {
    T wv[4], vv[4], pv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = (p + u * S) * ld + l;
      wv[u] = W[i];
      vv[u] = V[i];
      pv[u] = Vprev[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T w1 = wv[u] * ic - bp * (pv[u] * ip);
      const T w = w1 - a * (vv[u] * ic);
      W[(p + u * S) * ld + l] = w;
      an += static_cast<double>(w) * static_cast<double>(w);
      ad += static_cast<double>(w) * static_cast<double>(vv[u]);
    }
  }
  for (; p < n; p += S) {
    const int64_t i = p * ld + l;
    const T w1 = W[i] * ic - bp * (Vprev[i] * ip);
    const T w = w1 - a * (V[i] * ic);
    W[i] = w;
    an += static_cast<double>(w) * static_cast<double>(w);
    ad += static_cast<double>(w) * static_cast<double>(V[i]);
  }
  __shared__ double sh[2][8][32];
  sh[0][rl][l] = an;
  sh[1][rl][l] = ad;
  __syncthreads();
  if (rl == 0) {
    double t = 0, d = 0;
    for (int j = 0; j < 8; ++j) {
      t += sh[0][j][l];
      d += sh[1][j][l];
    }
    part[blockIdx.x * 64 + l] = t;
    part[blockIdx.x * 64 + 32 + l] = d;
  }
}

// Full re-orthogonalisation (classical Gram-Schmidt, applied twice by the
// driver) of the residual block W against the normalised Lanczos vectors
// Q[0..nv) (each n x 32): H[i][l] = sum_p Q[i][p][l] W[p][l], then
// W[:, l] -= sum_i H[i][l] Q[i][:, l].  Block (b, i) of k_ro_dot adds rows
// b * 8 + r, stride 8 gridDim.x, for its eight row lanes r, then the lanes in
// order; k_ro_fin adds the blocks of each vector in order.
__global__ void __launch_bounds__(kThreads) k_lz_store_q(int64_t n, const double* __restrict__ V,
                                                         const LzState* __restrict__ st, double* __restrict__ Qj) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i < n * 32) Qj[i] = V[i] * st->inv_cur[i & 31];
}

__global__ void __launch_bounds__(kThreads) k_ro_dot(int64_t n, const double* __restrict__ Q,
                                                     const double* __restrict__ W, double* __restrict__ part) {
  const int l = threadIdx.x & 31;
  const int rl = threadIdx.x >> 5;
  const int64_t vi = blockIdx.y;
  const double* q = Q + vi * n * 32;
  double acc = 0;
  for (int64_t p = blockIdx.x * 8ll + rl; p < n; p += static_cast<int64_t>(gridDim.x) * 8) acc += q[p * 32 + l] * W[p * 32 + l];
  __shared__ double sh[8][32];
  sh[rl][l] = acc;
  __syncthreads();
  if (rl == 0) {
    double t = 0;
    for (int j = 0; j < 8; ++j) t += sh[j][l];
    part[(vi * gridDim.x + blockIdx.x) * 32 + l] = t;
  }
}

__global__ void __launch_bounds__(32) k_ro_fin(const double* __restrict__ part, int nb, double* __restrict__ H) {
  const int64_t vi = blockIdx.x;
  const int l = threadIdx.x;
  double t = 0;
  for (int b = 0; b < nb; ++b) t += part[(vi * nb + b) * 32 + l];
  H[vi * 32 + l] = t;
}

__global__ void __launch_bounds__(kThreads) k_ro_update(int64_t n, int nv, const double* __restrict__ Q,
                                                        const double* __restrict__ H, double* __restrict__ W) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i >= n * 32) return;
  const int l = static_cast<int>(i & 31);
  double w = W[i];
  for (int v = 0; v < nv; ++v) w -= H[v * 32 + l] * Q[static_cast<int64_t>(v) * n * 32 + i];
  W[i] = w;
}

// after re-orthogonalisation: partial sums of |W[:, l]|^2 at part[b * 64 + l]
// and of W[:, l] . V[:, l] at part[b * 64 + 32 + l]
__global__ void __launch_bounds__(kThreads) k_lz_norm_dot(int64_t n, const double* __restrict__ V,
                                                          const double* __restrict__ W, double* __restrict__ part) {
  const int l = threadIdx.x & 31;
  const int rl = threadIdx.x >> 5;
  double an = 0, ad = 0;
  for (int64_t p = blockIdx.x * 8ll + rl; p < n; p += static_cast<int64_t>(gridDim.x) * 8) {
    const double w = W[p * 32 + l];
    an += w * w;
    ad += w * V[p * 32 + l];
  }
  __shared__ double sh[2][8][32];
  sh[0][rl][l] = an;
  sh[1][rl][l] = ad;
  __syncthreads();
  if (rl == 0) {
    double t = 0, d = 0;
    for (int q = 0; q < 8; ++q) {
      t += sh[0][q][l];
      d += sh[1][q][l];
    }
    part[blockIdx.x * 64 + l] = t;
    part[blockIdx.x * 64 + 32 + l] = d;
  }
}

// mode 0: alpha = inv_cur^2 x (sum of V . S K S V) - dcorr; mode 1: beta +
// breakdown (j = step index, last = final step) from the partials of |w|^2,
// and dcorr = inv_cur x the sum of w . V (those partials 32 after the first,
// 64 per block).
// 32 columns; each of kFinGroups groups of 32 threads sums the partials b = g,
// g + kFinGroups, ... of its column (four interleaved accumulators, so several
// loads are in flight), then the groups are added in order.
constexpr int kFinGroups = 32;

// (batched: problem blockIdx.y, its coefficients tstride doubles apart)
__global__ void __launch_bounds__(kFinGroups * 32) k_lz_fin(const double* __restrict__ part, int nb, int k, int mode,
                                                            int j, int last, double tol, LzState* __restrict__ st,
                                                            double* __restrict__ Ta, double* __restrict__ Tb,
                                                            Seg sg = {}, int64_t tstride = 0) {
  part += blockIdx.y * sg.pstride;
  st += blockIdx.y;
  Ta += blockIdx.y * tstride;
  Tb += blockIdx.y * tstride;
  __shared__ double sh[kFinGroups][32];
  __shared__ double sh2[kFinGroups][32];
  const int l = threadIdx.x & 31;
  const int g = threadIdx.x >> 5;
  const int ps = mode == 1 ? 64 : 32;
  double a4[4] = {0, 0, 0, 0}, d4[4] = {0, 0, 0, 0};
  int b = g;
  for (; b + 3 * kFinGroups < nb; b += 4 * kFinGroups)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a4[u] += part[(b + u * kFinGroups) * ps + l];
      if (mode == 1) d4[u] += part[(b + u * kFinGroups) * ps + 32 + l];
    }
#pragma unroll
  for (int u = 0; u < 3; ++u)
    if (b + u * kFinGroups < nb) {
      a4[u] += part[(b + u * kFinGroups) * ps + l];
      if (mode == 1) d4[u] += part[(b + u * kFinGroups) * ps + 32 + l];
    }
  sh[g][l] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  sh2[g][l] = (d4[0] + d4[1]) + (d4[2] + d4[3]);
  __syncthreads();
  if (g == 0 && l < k) {
    double t = 0;
    for (int q = 0; q < kFinGroups; ++q) t += sh[q][l];
    if (mode == 1) {
      double d = 0;
      for (int q = 0; q < kFinGroups; ++q) d += sh2[q][l];
      st->dcorr[l] = d * st->inv_cur[l];  // read before the rotation below
    } else {
      t = t * st->inv_cur[l] * st->inv_cur[l] - st->dcorr[l];
    }
    if (mode == 0) {
      st->alpha[l] = t;
      if (st->active[l]) Ta[j * 32 + l] = t;
    } else {
      const double beta = sqrt(t);
      if (st->active[l]) {
        if (last) {
          st->steps[l] = j + 1;
        } else if (!(beta > tol) || !isfinite(beta)) {
          st->steps[l] = j + 1;
          st->active[l] = 0;
        } else {
          Tb[j * 32 + l] = beta;
        }
      }
      st->beta[l] = st->active[l] ? beta : 0.0;
      st->beta_prev[l] = st->beta[l];
      // the residual block becomes the next v (unnormalised); finished probes get 0
      st->inv_prev[l] = st->inv_cur[l];
      st->inv_cur[l] = st->active[l] ? 1.0 / beta : 0.0;
    }
  }
}

// Symmetric tridiagonal eigen-decomposition by implicit QR sweeps with
// Wilkinson shifts (Givens rotations chasing the bulge), tracking only the
// first row of the eigenvector matrix.  a: diagonal (-> eigenvalues),
// b: off-diagonal (destroyed), q: first row of the eigenvector matrix.
__device__ bool tridiag_eig_first_row(double* a, double* b, double* q, int m) {
  for (int i = 0; i < m; ++i) q[i] = i == 0 ? 1.0 : 0.0;
  const double eps = 2.220446049250313e-16;
  int hi = m - 1;
  int iters = 0;
  while (hi > 0) {
    if (fabs(b[hi - 1]) <= eps * (fabs(a[hi - 1]) + fabs(a[hi]))) {
      b[hi - 1] = 0.0;
      --hi;
      continue;
    }
    if (++iters > 60 * m) return false;
    int lo = hi - 1;
    while (lo > 0 && fabs(b[lo - 1]) > eps * (fabs(a[lo - 1]) + fabs(a[lo]))) --lo;
    const double dlt = 0.5 * (a[hi - 1] - a[hi]);
    const double bb = b[hi - 1];
    const double den = dlt + copysign(hypot(dlt, bb), dlt == 0.0 ? 1.0 : dlt);
    const double mu = a[hi] - bb * bb / den;
    double x = a[lo] - mu;
    double z = b[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = z / r;
      }
      if (k > lo) b[k - 1] = r;
      const double ak = a[k], ak1 = a[k + 1], bk = b[k];
      a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      const double qk = q[k], qk1 = q[k + 1];
      q[k] = c * qk + s * qk1;
      q[k + 1] = -s * qk + c * qk1;
      if (k + 1 < hi) {
        x = b[k];
        z = s * b[k + 1];
        b[k + 1] = c * b[k + 1];
      }
    }
  }
  return true;
}

// One thread per probe: Gamma_l = |z|^2 sum_t tau_t^2 log theta_t.
// One thread per probe; the tridiagonal matrix and the eigenvector row live in
// LDS (rows padded against bank conflicts), kQuadProbes probes per block.
constexpr int kQuadProbes = 8;
constexpr int kQuadMax = 128;

// (batched: problem blockIdx.y, |z|^2 its length)
__global__ void __launch_bounds__(kQuadProbes) k_quadrature(int k, const double* __restrict__ Ta,
                                                            const double* __restrict__ Tb,
                                                            const LzState* __restrict__ st, double znorm2,
                                                            double* __restrict__ gam, int* __restrict__ bad,
                                                            Seg sg = {}, int64_t tstride = 0) {
  if (sg.off) {
    int64_t n = 0;
    seg_begin(sg, n);
    znorm2 = static_cast<double>(n);
    Ta += blockIdx.y * tstride;
    Tb += blockIdx.y * tstride;
    st += blockIdx.y;
    gam += blockIdx.y * 32;
    bad += blockIdx.y;
  }
  __shared__ double sa[kQuadProbes][kQuadMax + 1], sb[kQuadProbes][kQuadMax + 1], sq[kQuadProbes][kQuadMax + 1];
  const int l = blockIdx.x * kQuadProbes + threadIdx.x;
  if (l >= k) return;
  double* a = sa[threadIdx.x];
  double* b = sb[threadIdx.x];
  double* q = sq[threadIdx.x];
  const int m = st->steps[l];
  for (int j = 0; j < m; ++j) {
    a[j] = Ta[j * 32 + l];
    b[j] = j + 1 < m ? Tb[j * 32 + l] : 0.0;
  }
  double g = 0;
  if (!tridiag_eig_first_row(a, b, q, m)) {
    atomicOr(bad, 1);
  } else {
    for (int t = 0; t < m; ++t) {
      if (!(a[t] > 0.0)) atomicOr(bad, 2);
      g += q[t] * q[t] * log(a[t]);
    }
  }
  gam[l] = znorm2 * g;
}

// ------------------------------------------------------------- exact mode
__global__ void __launch_bounds__(kThreads) k_gemv_t(int64_t n, int nv, const double* __restrict__ V,
                                                     const double* __restrict__ w, double* __restrict__ h) {
  // one block per basis vector
  const int i = blockIdx.x;
  if (i >= nv) return;
  double v[1] = {0};
  const double* vi = V + static_cast<int64_t>(i) * n;
  for (int64_t p = threadIdx.x; p < n; p += kThreads) v[0] += vi[p] * w[p];
  __shared__ double sh[kThreads / kWave];
  double x = v[0];
  for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
  if (lane_id() == 0) sh[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int j = 0; j < kThreads / kWave; ++j) s += sh[j];
    h[i] = s;
  }
}

__global__ void __launch_bounds__(kThreads) k_gemv_n_sub(int64_t n, int nv, const double* __restrict__ V,
                                                         const double* __restrict__ h, double* __restrict__ w) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (p >= n) return;
  double s = 0;
  for (int i = 0; i < nv; ++i) s += V[static_cast<int64_t>(i) * n + p] * h[i];
  w[p] -= s;
}

__global__ void __launch_bounds__(kThreads) k_axpby2(int64_t n, double a, const double* __restrict__ x, double b,
                                                     const double* __restrict__ y, double* __restrict__ w) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (p < n) w[p] = w[p] - a * x[p] - b * y[p];
}

__global__ void __launch_bounds__(kThreads) k_scale_into(int64_t n, double s, const double* __restrict__ x,
                                                         double* __restrict__ y) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (p < n) y[p] = s * x[p];
}

__global__ void __launch_bounds__(kThreads) k_probe_vec(int64_t n, uint64_t seed, uint64_t probe,
                                                        const int32_t* __restrict__ perm, double* __restrict__ v) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (p < n) v[p] = rademacher(seed, probe, static_cast<uint64_t>(perm[p]));
}

}  // namespace

// ================================================================== host

double dot_f64(gp_ctx* c, const double* a, const double* b, int64_t n) {
  double* part = static_cast<double*>(workspace(c, 40, sizeof(double) * kRedBlocks));
  double* out = static_cast<double*>(workspace(c, 41, sizeof(double) * 2));
  hipLaunchKernelGGL(k_dot_part, dim3(kRedBlocks), dim3(kThreads), 0, c->stream, n, a, b, part);
  hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(kThreads), 0, c->stream, part, kRedBlocks, out);
  check_launch("dot");
  double* h = static_cast<double*>(pinned(c, sizeof(double)));
  GPS_HIP(hipMemcpyAsync(h, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return *h;
}

static double logsum_f64(gp_ctx* c, const double* a, int64_t n) {
  double* part = static_cast<double*>(workspace(c, 40, sizeof(double) * kRedBlocks));
  double* out = static_cast<double*>(workspace(c, 41, sizeof(double) * 2));
  hipLaunchKernelGGL(k_logsum_part, dim3(kRedBlocks), dim3(kThreads), 0, c->stream, n, a, part);
  hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(kThreads), 0, c->stream, part, kRedBlocks, out);
  check_launch("logsum");
  double* h = static_cast<double*>(pinned(c, sizeof(double)));
  GPS_HIP(hipMemcpyAsync(h, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  return *h;
}

SolveResult pcg_solve(gp_ctx* c, gp_matrix* m, const double* y, double* x, double rtol, int max_iter, int precond) {
  const int64_t n = m->n;
  if (precond == GP_PRECOND_BLOCK_JACOBI) build_block_jacobi(c, m);
  Precond M{m->diag, nullptr, nullptr, nullptr, nullptr};
  if (precond == GP_PRECOND_BLOCK_JACOBI) {
    M.rowblk = m->rowblk;
    M.bstart = m->bstart;
    M.boff = m->boff;
    M.binv = m->binv;
  }
  // the residual alternates between two buffers: a step reads one and writes the other
  double* rc = static_cast<double*>(workspace(c, 20, sizeof(double) * n));
  double* rnx = static_cast<double*>(workspace(c, 29, sizeof(double) * n));
  double* z = static_cast<double*>(workspace(c, 21, sizeof(double) * n));
  double* p = static_cast<double*>(workspace(c, 22, sizeof(double) * n));
  double* q = static_cast<double*>(workspace(c, 23, sizeof(double) * n));
  double* part = static_cast<double*>(workspace(c, 26, sizeof(double) * 4 * kRedBlocks));
  const unsigned nbp = grid_for(n, kThreads);
  const unsigned nbs = grid_for(n, kThreads * kStepRows);
  double* ppart = static_cast<double*>(workspace(c, 28, sizeof(double) * 2 * nbp));
  CgScalars* s = static_cast<CgScalars*>(workspace(c, 27, sizeof(CgScalars)));
  CgScalars* hs = static_cast<CgScalars*>(pinned(c, sizeof(CgScalars)));
  const dim3 G(kRedBlocks), B(kThreads);
  auto read = [&]() {
    GPS_HIP(hipMemcpyAsync(hs, s, sizeof(CgScalars), hipMemcpyDeviceToHost, c->stream));
    side_pump(c);  // the side stream's queue topped up before the host waits
    sync(c);
    return *hs;
  };
  // z = M^-1 r and the scalars r.z, r.r (mode: see k_beta_fin)
  auto apply_precond = [&](int mode) {
    ProfScope ps(c, "pcg_precond");
    hipLaunchKernelGGL(k_precond, dim3(nbp), B, 0, c->stream, n, M, rc, z, ppart);
    hipLaunchKernelGGL(k_beta_fin, dim3(1), B, 0, c->stream, ppart, static_cast<int>(nbp), s, mode);
  };
  auto true_residual = [&]() {
    spmv_f64(c, m, x, q);
    hipLaunchKernelGGL(k_true_resid, G, B, 0, c->stream, n, y, q, rc);
    apply_precond(1);
    check_launch("true residual");
    return read();
  };
  {
    ProfScope ps(c, "pcg_vector_ops");
    hipLaunchKernelGGL(k_pcg_init, G, B, 0, c->stream, n, y, x, rc, part);
    hipLaunchKernelGGL(k_yy_fin, dim3(1), B, 0, c->stream, part, kRedBlocks, s);
  }
  apply_precond(2);
  hipLaunchKernelGGL(k_pcg_pupdate, G, B, 0, c->stream, n, s, z, p);
  check_launch("pcg init");
  CgScalars sc = read();
  SolveResult res;
  GPS_REQUIRE(std::isfinite(sc.yy), GP_EINVAL, "y holds non-finite values");
  const double ynorm = std::sqrt(sc.yy);
  if (ynorm == 0.0) return res;
  const double target = rtol * ynorm;
  double last_true = ynorm;   // |y - K x| at the latest recomputation
  int it = 0;
  bool converged = false;
  // per iteration: q = K p, partials of p.q, the step (alpha, x, r, z and the
  // partials of r.z, r.r), the new direction (beta, p); the last step before a
  // host check leaves the direction to after the check
  double* pqp = part;                    // kRedBlocks partials of p.q
  double* spart = ppart;                 // 2 x nbs partials of r.z, r.r
  while (it < max_iter && !converged) {
    const int steps = std::min(kCheckEvery, max_iter - it);
    for (int t = 0; t < steps; ++t) {
      // float64 vectors; a GP_MIXED matrix contributes its float32 values
      spmv_f64(c, m, p, q);
      {
        ProfScope ps(c, "pcg_vector_ops");
        hipLaunchKernelGGL((k_pq_part<double>), G, B, 0, c->stream, n, p, q, pqp, nullptr);
        hipLaunchKernelGGL((k_pcg_step<double>), dim3(nbs), B, 0, c->stream, n, M, s, pqp, p, q, x, rc, rnx, z,
                           spart, nullptr);
        std::swap(rc, rnx);
        if (t + 1 < steps)
          hipLaunchKernelGGL(k_pcg_direction, G, B, 0, c->stream, n, s, spart, static_cast<int>(nbs), z, p, nullptr);
        else
          hipLaunchKernelGGL(k_beta_fin, dim3(1), B, 0, c->stream, spart, static_cast<int>(nbs), s, 3);
      }
      check_launch("pcg iteration");
      side_pump(c);
    }
    it += steps;
    sc = read();
    if (sc.status != 0) {
      res.st = GP_ENOTPD;
      break;
    }
    const double rn = std::sqrt(sc.rr);
    // at apparent convergence the residual is recomputed as y - K x and replaces
    // the recursive one
    if (rn <= target) {
      sc = true_residual();
      ++res.refreshes;
      last_true = std::sqrt(sc.rr);
      if (last_true <= target) converged = true;
    }
    if (!converged && it < max_iter) {
      hipLaunchKernelGGL(k_pcg_pupdate, G, B, 0, c->stream, n, s, z, p);
      check_launch("pcg direction");
    }
  }
  res.iters = it;
  if (!converged) {
    sc = true_residual();
    last_true = std::sqrt(sc.rr);
    if (res.st == GP_OK) res.st = last_true <= target ? GP_OK : GP_ENOTCONV;
  }
  res.relres = last_true / ynorm;
  res.quad = dot_f64(c, y, x, n);
  return res;
}

namespace {

// ------------------------------------------------ device-driven conjugate gradients
// The iterations of pcg_solve with every decision taken on the device: the
// host enqueues blocks of kCheckEvery iterations up to max_iter; after each
// block a control kernel compares the recursive residual with the target
// and, at apparent convergence, lets the true-residual pass run; every kernel
// of the iterations returns at once once the solve has ended (skip flags).
// For a batch the control kernels take one thread per problem and also gather
// the flags the problems share: a product of the stacked matrix is skipped
// only once every problem has set its flag.
constexpr int kCtlThreads = 64;

__device__ void ctl_gather(const CgCtl* __restrict__ ctl, int R, CtlAll* __restrict__ all) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int si = 1, st = 1, sf = 1;
    for (int r = 0; r < R; ++r) {
      si &= ctl[r].skip_iter != 0;
      st &= ctl[r].skip_true != 0;
      sf &= ctl[r].skip_final != 0;
    }
    all->skip_iter = si;
    all->skip_true = st;
    all->skip_final = sf;
  }
}

__global__ void __launch_bounds__(kCtlThreads) k_ctl_init(const CgScalars* __restrict__ s, CgCtl* __restrict__ ctl,
                                                          double rtol, int R, CtlAll* __restrict__ all) {
  for (int r = threadIdx.x; r < R; r += kCtlThreads) {
    CgCtl* cr = ctl + r;
    const double yy = s[r].yy;
    cr->iters = 0;
    cr->refreshes = 0;
    cr->skip_true = 1;
    cr->relres = 0.0;
    cr->target = rtol * sqrt(yy);
    if (!isfinite(yy)) {
      cr->status = GP_EINVAL;
      cr->skip_iter = cr->skip_final = 1;
    } else if (yy == 0.0) {
      cr->status = GP_OK;  // x = 0 is exact
      cr->skip_iter = cr->skip_final = 1;
    } else {
      cr->status = GP_OK;
      cr->skip_iter = cr->skip_final = 0;
    }
  }
  ctl_gather(ctl, R, all);
}

__global__ void __launch_bounds__(kCtlThreads) k_ctl_check(const CgScalars* __restrict__ s, CgCtl* __restrict__ ctl,
                                                           int steps, int R, CtlAll* __restrict__ all) {
  for (int r = threadIdx.x; r < R; r += kCtlThreads) {
    CgCtl* cr = ctl + r;
    if (cr->skip_iter) continue;
    cr->iters += steps;
    if (s[r].status != 0) {
      cr->status = GP_ENOTPD;
      cr->skip_iter = 1;
      continue;
    }
    cr->skip_true = sqrt(s[r].rr) <= cr->target ? 0 : 1;
  }
  ctl_gather(ctl, R, all);
}

__global__ void __launch_bounds__(kCtlThreads) k_ctl_after_true(const CgScalars* __restrict__ s,
                                                                CgCtl* __restrict__ ctl, int R,
                                                                CtlAll* __restrict__ all) {
  for (int r = threadIdx.x; r < R; r += kCtlThreads) {
    CgCtl* cr = ctl + r;
    if (cr->skip_true) continue;
    cr->skip_true = 1;
    cr->refreshes += 1;
    if (sqrt(s[r].rr) <= cr->target) {
      cr->skip_iter = 1;
      cr->skip_final = 1;
      cr->relres = sqrt(s[r].rr) / sqrt(s[r].yy);
    }
  }
  ctl_gather(ctl, R, all);
}

__global__ void __launch_bounds__(kCtlThreads) k_ctl_end(CgCtl* __restrict__ ctl, int R, CtlAll* __restrict__ all) {
  for (int r = threadIdx.x; r < R; r += kCtlThreads) {
    if (!ctl[r].skip_iter) {
      ctl[r].status = GP_ENOTCONV;
      ctl[r].skip_iter = 1;
    }
  }
  ctl_gather(ctl, R, all);
}

__global__ void __launch_bounds__(kCtlThreads) k_ctl_relres(const CgScalars* __restrict__ s, CgCtl* __restrict__ ctl,
                                                            int R) {
  for (int r = threadIdx.x; r < R; r += kCtlThreads) {
    CgCtl* cr = ctl + r;
    if (!cr->skip_final) {
      cr->relres = sqrt(s[r].rr) / sqrt(s[r].yy);
      if (cr->status == GP_ENOTCONV && sqrt(s[r].rr) <= cr->target) cr->status = GP_OK;
    }
  }
}

}  // namespace

// One device-driven solve, or a batch of R problems stacked along the rows of
// m (off: R + 1 device row offsets, nmax the longest problem).  poll: the host
// reads the shared iteration flag after every block of iterations and stops
// enqueueing once every problem has ended.
static void pcg_device_impl(gp_ctx* c, gp_matrix* m, const double* y, double* x, double rtol, int max_iter,
                            int precond, int R, const int64_t* off, int64_t nmax, bool poll, DeviceSolve* out) {
  const int64_t n = m->n;
  Precond M{m->diag, nullptr, nullptr, nullptr, nullptr};
  if (precond == GP_PRECOND_BLOCK_JACOBI) {
    M.rowblk = m->rowblk;
    M.bstart = m->bstart;
    M.boff = m->boff;
    M.binv = m->binv;
  }
  const bool batch = off != nullptr;
  const int64_t nrow = batch ? nmax : n;  // rows of the longest problem: sets the per-row grids
  const unsigned nbp = grid_for(nrow, kThreads);
  const unsigned nbs = grid_for(nrow, kThreads * kStepRows);
  Seg g;
  if (batch) {
    g.off = off;
    g.pstride = static_cast<int>(std::max<int64_t>(4 * kRedBlocks, 2 * static_cast<int64_t>(nbp)));
  }
  const size_t pbytes = sizeof(double) * (batch ? static_cast<size_t>(R) * g.pstride : 4 * kRedBlocks);
  const size_t ppbytes = sizeof(double) * (batch ? static_cast<size_t>(R) * g.pstride : 2 * nbp);
  double* rc = static_cast<double*>(workspace(c, 20, sizeof(double) * n));
  double* rnx = static_cast<double*>(workspace(c, 29, sizeof(double) * n));
  double* z = static_cast<double*>(workspace(c, 21, sizeof(double) * n));
  double* p = static_cast<double*>(workspace(c, 22, sizeof(double) * n));
  double* q = static_cast<double*>(workspace(c, 23, sizeof(double) * n));
  double* part = static_cast<double*>(workspace(c, 26, pbytes));
  double* ppart = static_cast<double*>(workspace(c, 28, ppbytes));
  CgScalars* s = static_cast<CgScalars*>(workspace(c, 27, sizeof(CgScalars) * R));
  CgCtl* ctl = static_cast<CgCtl*>(workspace(c, 24, sizeof(CgCtl) * R));
  CtlAll* all = static_cast<CtlAll*>(workspace(c, 130, sizeof(CtlAll)));
  // per-problem flags for the vector kernels, shared flags for the products
  const int* skip_iter = &ctl->skip_iter;
  const int* skip_true = &ctl->skip_true;
  const int* skip_final = &ctl->skip_final;
  const unsigned Ry = static_cast<unsigned>(R);
  const dim3 G(kRedBlocks, Ry), B(kThreads), G1(1, Ry), GP(nbp, Ry), GS(nbs, Ry), C(kCtlThreads);
  auto true_residual = [&](const int* gate, const int* shared_gate) {
    spmv_f64(c, m, x, q, shared_gate);
    hipLaunchKernelGGL(k_true_resid, G, B, 0, c->stream, nrow, y, q, rc, gate, g);
    hipLaunchKernelGGL(k_precond, GP, B, 0, c->stream, nrow, M, rc, z, ppart, gate, g);
    hipLaunchKernelGGL(k_beta_fin, G1, B, 0, c->stream, ppart, static_cast<int>(nbp), s, 1, gate, g, kThreads);
  };
  hipLaunchKernelGGL(k_pcg_init, G, B, 0, c->stream, nrow, y, x, rc, part, g);
  hipLaunchKernelGGL(k_yy_fin, G1, B, 0, c->stream, part, kRedBlocks, s, g);
  hipLaunchKernelGGL(k_ctl_init, dim3(1), C, 0, c->stream, s, ctl, rtol, R, all);
  hipLaunchKernelGGL(k_precond, GP, B, 0, c->stream, nrow, M, rc, z, ppart, skip_iter, g);
  hipLaunchKernelGGL(k_beta_fin, G1, B, 0, c->stream, ppart, static_cast<int>(nbp), s, 2, skip_iter, g, kThreads);
  hipLaunchKernelGGL(k_pcg_pupdate, G, B, 0, c->stream, nrow, s, z, p, skip_iter, g);
  check_launch("pcg init");
  double* pqp = part;
  double* spart = ppart;
  int* hflag = poll ? static_cast<int*>(pinned(c, sizeof(int))) : nullptr;
  for (int it = 0; it < max_iter; it += kCheckEvery) {
    const int steps = std::min(kCheckEvery, max_iter - it);
    for (int t = 0; t < steps; ++t) {
      spmv_f64(c, m, p, q, &all->skip_iter);
      ProfScope ps(c, "pcg_vector_ops");
      hipLaunchKernelGGL((k_pq_part<double>), G, B, 0, c->stream, nrow, p, q, pqp, skip_iter, g);
      hipLaunchKernelGGL((k_pcg_step<double>), GS, B, 0, c->stream, nrow, M, s, pqp, p, q, x, rc, rnx, z,
                         spart, skip_iter, g);
      std::swap(rc, rnx);
      if (t + 1 < steps)
        hipLaunchKernelGGL(k_pcg_direction, G, B, 0, c->stream, nrow, s, spart, static_cast<int>(nbs), z, p,
                           skip_iter, g);
      else
        hipLaunchKernelGGL(k_beta_fin, G1, B, 0, c->stream, spart, static_cast<int>(nbs), s, 3, skip_iter, g,
                           kThreads * kStepRows);
      side_pump(c);
    }
    hipLaunchKernelGGL(k_ctl_check, dim3(1), C, 0, c->stream, s, ctl, steps, R, all);
    true_residual(skip_true, &all->skip_true);
    hipLaunchKernelGGL(k_ctl_after_true, dim3(1), C, 0, c->stream, s, ctl, R, all);
    hipLaunchKernelGGL(k_pcg_pupdate, G, B, 0, c->stream, nrow, s, z, p, skip_iter, g);
    check_launch("pcg iteration block");
    if (poll) {
      GPS_HIP(hipMemcpyAsync(hflag, &all->skip_iter, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      side_pump(c);
      sync(c);
      if (*hflag) break;
    }
  }
  hipLaunchKernelGGL(k_ctl_end, dim3(1), C, 0, c->stream, ctl, R, all);
  true_residual(skip_final, &all->skip_final);
  hipLaunchKernelGGL(k_ctl_relres, dim3(1), C, 0, c->stream, s, ctl, R);
  // quad = y . x per problem
  Seg gq = g;
  if (batch) gq.pstride = kRedBlocks;
  double* qd = static_cast<double*>(workspace(c, 25, sizeof(double) * std::max(R, 2)));
  double* dpart = static_cast<double*>(workspace(c, 40, sizeof(double) * kRedBlocks * R));
  hipLaunchKernelGGL(k_dot_part, G, B, 0, c->stream, nrow, y, x, dpart, gq);
  hipLaunchKernelGGL(k_sum_part, G1, B, 0, c->stream, dpart, kRedBlocks, qd, gq);
  check_launch("pcg end");
  out->quad = qd;
  out->ctl = ctl;
}

void pcg_solve_device(gp_ctx* c, gp_matrix* m, const double* y, double* x, double rtol, int max_iter, int precond,
                      DeviceSolve* out) {
  pcg_device_impl(c, m, y, x, rtol, max_iter, precond, 1, nullptr, m->n, false, out);
}

void pcg_solve_batch(gp_ctx* c, gp_matrix* m, const double* y, double* x, double rtol, int max_iter, int precond,
                     int R, const int64_t* off, int64_t nmax, DeviceSolve* out) {
  pcg_device_impl(c, m, y, x, rtol, max_iter, precond, R, off, nmax, true, out);
}

namespace {

// ---------------------------------------------------------------- MINRES
// Preconditioned MINRES (Paige and Saunders; the paper's solver, Sec. 3.3):
// Lanczos in the M-inner product, Givens rotations on its tridiagonal matrix,
// three-term search directions.  Products in float64 arithmetic on the stored
// values; all vectors and scalars float64.  Scalars stay on the device; a
// one-thread kernel applies each rotation.
struct MrScalars {
  double beta, oldb, alfa, dbar, epsln, phibar, cs, sn, phi, gamma, delta, oldeps;
  double beta1, rr;
  int it, status;
};

// beta1 = sqrt(r . z) (start); the rotation state starts as in the reference method
__global__ void k_mr_start(const double* __restrict__ part, int nb, MrScalars* __restrict__ s) {
  double r[2];
  reduce_partials<2>(part, nb, r);
  if (threadIdx.x == 0) {
    const double b = sqrt(r[0]);
    s->beta1 = b;
    s->beta = b;
    s->oldb = 0.0;
    s->dbar = 0.0;
    s->epsln = 0.0;
    s->phibar = b;
    s->cs = -1.0;
    s->sn = 0.0;
    s->it = 0;
    s->status = (isfinite(b) && r[0] >= 0.0) ? 0 : 1;
  }
}

// v = z / beta (first vector)
__global__ void __launch_bounds__(kThreads) k_mr_first_v(int64_t n, const MrScalars* __restrict__ s,
                                                         const double* __restrict__ z, double* __restrict__ v) {
  const double sc = 1.0 / s->beta;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    v[i] = sc * z[i];
}

// partials of v . y1 with y1 = q - (beta / oldb) r1 (the second term from the
// second step on)
__global__ void __launch_bounds__(kThreads) k_mr_alpha(int64_t n, const MrScalars* __restrict__ s,
                                                       const double* __restrict__ q, const double* __restrict__ r1,
                                                       const double* __restrict__ v, double* __restrict__ part) {
  const double f = s->it >= 1 ? s->beta / s->oldb : 0.0;
  double acc[1] = {0.0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double y1 = s->it >= 1 ? q[i] - f * r1[i] : q[i];
    acc[0] += v[i] * y1;
  }
  block_sum_store<1>(acc, part);
}

__global__ void k_mr_alpha_fin(const double* __restrict__ part, int nb, MrScalars* __restrict__ s) {
  double r[1];
  reduce_partials<1>(part, nb, r);
  if (threadIdx.x == 0) s->alfa = r[0];
}

// new Lanczos vector rn = (q - (beta/oldb) r1) - (alfa/beta) r2 and z = M^-1 rn;
// partials of rn . z.  Entries of rn needed by the block product are formed
// the same way from q, r1, r2, so no thread waits for another.
__device__ __forceinline__ double mr_next(const MrScalars& s, double f, const double* q, const double* r1,
                                          const double* r2, int64_t j) {
  const double y1 = s.it >= 1 ? q[j] - f * r1[j] : q[j];
  return y1 - (s.alfa / s.beta) * r2[j];
}

__global__ void __launch_bounds__(kThreads) k_mr_lanczos(int64_t n, Precond M, const MrScalars* __restrict__ sp,
                                                         const double* __restrict__ q, const double* __restrict__ r1,
                                                         const double* __restrict__ r2, double* __restrict__ rn,
                                                         double* __restrict__ z, double* __restrict__ part) {
  const MrScalars s = *sp;
  const double f = s.it >= 1 ? s.beta / s.oldb : 0.0;
  double v[1] = {0.0};
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i < n) {
    const double ri = mr_next(s, f, q, r1, r2, i);
    double zi;
    if (!M.binv) {
      zi = ri / M.diag[i];
    } else {
      const int32_t b = M.rowblk[i];
      const int32_t bs = M.bstart[b];
      const int sz = M.bstart[b + 1] - bs;
      const double* row = M.binv + M.boff[b] + static_cast<int64_t>(i - bs) * sz;
      zi = 0.0;
      for (int j = 0; j < sz; ++j) zi += row[j] * mr_next(s, f, q, r1, r2, bs + j);
    }
    rn[i] = ri;
    z[i] = zi;
    v[0] = ri * zi;
  }
  block_sum_store<1>(v, part);
}

// beta of the new vector and one Givens rotation of the tridiagonal matrix
__global__ void k_mr_rotate(const double* __restrict__ part, int nb, MrScalars* __restrict__ s) {
  double r[1];
  reduce_partials<1>(part, nb, r);
  if (threadIdx.x == 0) {
    if (!(r[0] >= 0.0) || !isfinite(r[0])) s->status = 1;
    s->oldb = s->beta;
    s->beta = sqrt(fmax(r[0], 0.0));
    s->oldeps = s->epsln;
    s->delta = s->cs * s->dbar + s->sn * s->alfa;
    const double gbar = s->sn * s->dbar - s->cs * s->alfa;
    s->epsln = s->sn * s->beta;
    s->dbar = -s->cs * s->beta;
    const double gamma = fmax(hypot(gbar, s->beta), 2.2250738585072014e-308);
    s->gamma = gamma;
    s->cs = gbar / gamma;
    s->sn = s->beta / gamma;
    s->phi = s->cs * s->phibar;
    s->phibar = s->sn * s->phibar;
    s->it += 1;
  }
}

// w = (v - oldeps w1 - delta w2) / gamma into the buffer of w1 (oldest);
// x += phi w; next v = z / beta
__global__ void __launch_bounds__(kThreads) k_mr_update(int64_t n, const MrScalars* __restrict__ s,
                                                        double* __restrict__ w1, const double* __restrict__ w2,
                                                        double* __restrict__ x, double* __restrict__ v,
                                                        const double* __restrict__ z) {
  const double oldeps = s->oldeps, delta = s->delta, gamma = s->gamma, phi = s->phi;
  const double sc = s->beta > 0.0 ? 1.0 / s->beta : 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double w = (v[i] - oldeps * w1[i] - delta * w2[i]) / gamma;
    w1[i] = w;
    x[i] += phi * w;
    v[i] = sc * z[i];
  }
}

}  // namespace

SolveResult minres_solve(gp_ctx* c, gp_matrix* m, const double* y, double* x, bool warm, double rtol, int max_iter,
                         int precond) {
  const int64_t n = m->n;
  if (precond == GP_PRECOND_BLOCK_JACOBI) build_block_jacobi(c, m);
  Precond M{m->diag, nullptr, nullptr, nullptr, nullptr};
  if (precond == GP_PRECOND_BLOCK_JACOBI) {
    M.rowblk = m->rowblk;
    M.bstart = m->bstart;
    M.boff = m->boff;
    M.binv = m->binv;
  }
  double* buf[8];
  for (int k = 0; k < 8; ++k) buf[k] = static_cast<double*>(workspace(c, 80 + k, sizeof(double) * n));
  double *r1 = buf[0], *r2 = buf[1], *rn = buf[2], *z = buf[3], *v = buf[4], *q = buf[5];
  double *wa = buf[6], *wb = buf[7];  // w1 (oldest), w2 (newest)
  const unsigned nbp = grid_for(n, kThreads);
  double* part = static_cast<double*>(workspace(c, 88, sizeof(double) * 2 * std::max<unsigned>(nbp, kRedBlocks)));
  MrScalars* s = static_cast<MrScalars*>(workspace(c, 89, sizeof(MrScalars)));
  MrScalars* hs = static_cast<MrScalars*>(pinned(c, sizeof(MrScalars)));
  const dim3 G(kRedBlocks), B(kThreads);
  auto read = [&]() {
    GPS_HIP(hipMemcpyAsync(hs, s, sizeof(MrScalars), hipMemcpyDeviceToHost, c->stream));
    side_pump(c);
    sync(c);
    return *hs;
  };
  // |y|, |y|_{M^-1}: the true-residual check starts once the estimate is
  // below 100 rtol |y|_{M^-1} (the two norms differ by at most sqrt(cond M))
  const double ynorm = std::sqrt(dot_f64(c, y, y, n));
  SolveResult res;
  GPS_REQUIRE(std::isfinite(ynorm), GP_EINVAL, "y holds non-finite values");
  if (ynorm == 0.0) {
    GPS_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, c->stream));
    return res;
  }
  auto residual_into = [&](double* r) {  // r = y - K x
    spmv_f64(c, m, x, q);
    hipLaunchKernelGGL(k_true_resid, G, B, 0, c->stream, n, y, q, r);
  };
  auto apply_m = [&](const double* r) {  // z = M^-1 r, partials of (r.z, r.r)
    hipLaunchKernelGGL(k_precond, dim3(nbp), B, 0, c->stream, n, M, r, z, part);
  };
  // |y|_{M^-1}
  apply_m(y);
  hipLaunchKernelGGL(k_mr_start, dim3(1), B, 0, c->stream, part, static_cast<int>(nbp), s);
  const double ym = read().beta1;
  if (warm) {
    residual_into(r1);
  } else {
    GPS_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, c->stream));
    GPS_HIP(hipMemcpyAsync(r1, y, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  }
  GPS_HIP(hipMemcpyAsync(r2, r1, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  GPS_HIP(hipMemsetAsync(wa, 0, sizeof(double) * n, c->stream));
  GPS_HIP(hipMemsetAsync(wb, 0, sizeof(double) * n, c->stream));
  apply_m(r1);
  hipLaunchKernelGGL(k_mr_start, dim3(1), B, 0, c->stream, part, static_cast<int>(nbp), s);
  hipLaunchKernelGGL(k_mr_first_v, G, B, 0, c->stream, n, s, z, v);
  check_launch("minres start");
  MrScalars sc = read();
  double true_rel = std::sqrt(dot_f64(c, r1, r1, n)) / ynorm;
  int it = 0;
  bool converged = true_rel <= rtol;
  if (!(sc.beta1 > 0.0)) converged = true;
  while (!converged && it < max_iter && sc.status == 0) {
    const int steps = std::min(kCheckEvery, max_iter - it);
    for (int t = 0; t < steps; ++t) {
      spmv_f64(c, m, v, q);
      ProfScope ps(c, "minres_vector_ops");
      hipLaunchKernelGGL(k_mr_alpha, G, B, 0, c->stream, n, s, q, r1, v, part);
      hipLaunchKernelGGL(k_mr_alpha_fin, dim3(1), B, 0, c->stream, part, kRedBlocks, s);
      hipLaunchKernelGGL(k_mr_lanczos, dim3(nbp), B, 0, c->stream, n, M, s, q, r1, r2, rn, z, part);
      hipLaunchKernelGGL(k_mr_rotate, dim3(1), B, 0, c->stream, part, static_cast<int>(nbp), s);
      hipLaunchKernelGGL(k_mr_update, G, B, 0, c->stream, n, s, wa, wb, x, v, z);
      check_launch("minres step");
      side_pump(c);
      // rotate: r1 <- r2, r2 <- rn; w1 <- w2, w2 <- the new w (written over w1)
      double* t1 = r1;
      r1 = r2;
      r2 = rn;
      rn = t1;
      std::swap(wa, wb);
    }
    it += steps;
    sc = read();
    if (sc.status != 0) break;
    if (sc.phibar <= 100.0 * rtol * ym || sc.beta == 0.0) {
      residual_into(rn);
      true_rel = std::sqrt(dot_f64(c, rn, rn, n)) / ynorm;
      if (true_rel <= rtol || sc.beta == 0.0) converged = true;
    }
  }
  if (!converged && sc.status == 0) {
    residual_into(rn);
    true_rel = std::sqrt(dot_f64(c, rn, rn, n)) / ynorm;
    converged = true_rel <= rtol;
  }
  res.iters = it;
  res.relres = true_rel;
  res.st = sc.status != 0 ? GP_ENOTPD : (converged ? GP_OK : GP_ENOTCONV);
  res.quad = dot_f64(c, y, x, n);
  return res;
}

namespace {

// device-driven SLQ pieces: the Lanczos state of a batch of probes, the
// per-probe quadratures collected across batches, and the estimate
// (batched: problem blockIdx.y starts from inv0s[blockIdx.y])
__global__ void k_lz_state_init(LzState* __restrict__ st, int k, double inv0, const double* __restrict__ inv0s) {
  const int l = threadIdx.x;
  if (l >= 32) return;
  st += blockIdx.y;
  if (inv0s) inv0 = inv0s[blockIdx.y];
  st->alpha[l] = st->beta[l] = st->beta_prev[l] = st->inv_prev[l] = st->dcorr[l] = 0.0;
  st->active[l] = l < k ? 1 : 0;
  st->inv_cur[l] = l < k ? inv0 : 0.0;
  st->steps[l] = 0;
}

__global__ void k_slq_collect(const LzState* __restrict__ st, const double* __restrict__ gam, int k, int p0,
                              double* __restrict__ gam_all, int* __restrict__ steps_all, int np) {
  st += blockIdx.y;
  gam += blockIdx.y * 32;
  gam_all += blockIdx.y * np;
  steps_all += blockIdx.y * np;
  const int l = threadIdx.x;
  if (l < k) {
    gam_all[p0 + l] = gam[l];
    steps_all[p0 + l] = st->steps[l];
  }
}

// mean and standard error over the probes, in the host form's order and without
// fused multiply-adds, so the figures equal the synchronous path's bitwise
__global__ void k_slq_final(const double* __restrict__ gam_all, const int* __restrict__ steps_all, int np,
                            const double* __restrict__ jac, const int* __restrict__ bad, DeviceLogdet* __restrict__ out) {
#pragma clang fp contract(off)
  gam_all += blockIdx.y * np;
  steps_all += blockIdx.y * np;
  jac += blockIdx.y;
  bad += blockIdx.y;
  out += blockIdx.y;
  double mean = 0;
  int ms = 0;
  for (int i = 0; i < np; ++i) {
    mean += gam_all[i];
    ms = max(ms, steps_all[i]);
  }
  mean /= static_cast<double>(np);
  double var = 0;
  for (int i = 0; i < np; ++i) var += (gam_all[i] - mean) * (gam_all[i] - mean);
  out->se = np > 1 ? sqrt(var / static_cast<double>(np - 1) / np) : 0.0;
  out->logdet = jac[0] + mean;
  out->steps = ms;
  out->status = (bad[0] & 1) ? GP_EDEVICE : ((bad[0] & 2) ? GP_ENOTPD : GP_OK);
}

}  // namespace

// The work space of an SLQ estimate (R problems stacked in n rows); the
// device-driven form also keeps its Jacobi sums and per-probe results there.
constexpr int kRoBlocks = 256;

template <typename T>
struct SlqBufs {
  double *Qall = nullptr, *ropart = nullptr, *H = nullptr;
  T *V, *Vp, *W, *sc;
  double *part, *Ta, *Tb, *gam;
  LzState* st;
  int* bad;
  double *djac = nullptr, *jpart = nullptr, *gam_all = nullptr;
  int* steps_all = nullptr;
};

template <typename T>
static SlqBufs<T> slq_bufs(gp_ctx* c, int64_t n, int n_probes, int n_steps, bool reorth, int R, bool dev) {
  const int ld = 32;
  const int64_t tstride = static_cast<int64_t>(32) * n_steps;
  SlqBufs<T> b;
  if (reorth) {
    // full re-orthogonalisation keeps every normalised Lanczos block
    b.Qall = static_cast<double*>(workspace(c, 57, sizeof(double) * n * ld * n_steps));
    b.ropart = static_cast<double*>(workspace(c, 58, sizeof(double) * 32 * kRoBlocks * n_steps));
    b.H = static_cast<double*>(workspace(c, 59, sizeof(double) * 32 * n_steps));
  }
  b.V = static_cast<T*>(workspace(c, 30, sizeof(T) * n * ld));
  b.Vp = static_cast<T*>(workspace(c, 31, sizeof(T) * n * ld));
  b.W = static_cast<T*>(workspace(c, 32, sizeof(T) * n * ld));
  b.sc = static_cast<T*>(workspace(c, 33, sizeof(T) * n));
  b.part = static_cast<double*>(workspace(c, 34, sizeof(double) * 64 * kRedBlocks * R));
  b.st = static_cast<LzState*>(workspace(c, 35, sizeof(LzState) * R));
  b.Ta = static_cast<double*>(workspace(c, 36, sizeof(double) * tstride * R));
  b.Tb = static_cast<double*>(workspace(c, 37, sizeof(double) * tstride * R));
  b.gam = static_cast<double*>(workspace(c, 38, sizeof(double) * 32 * R));
  b.bad = static_cast<int*>(workspace(c, 39, sizeof(int) * std::max(R, 2)));
  if (dev) {
    b.djac = static_cast<double*>(workspace(c, 46, sizeof(double) * std::max(R, 2)));
    b.jpart = static_cast<double*>(workspace(c, 47, sizeof(double) * kRedBlocks * R));
    b.gam_all = static_cast<double*>(workspace(c, 48, sizeof(double) * n_probes * R));
    b.steps_all = static_cast<int*>(workspace(c, 49, sizeof(int) * n_probes * R));
  }
  return b;
}

// One SLQ estimate as a sequence of units, each one Lanczos step of the
// current block of (at most 32) probes: the block's start before its first
// step, its quadrature after its last, the estimate after the last block.
// The constructor enqueues the set-up (column scale, Jacobi part).  With
// dev_out every result stays on the device; without, the host reads each
// block's quadratures (a synchronisation per block) and result() forms the
// estimate.
template <typename T>
class SlqRun final : public SideFeed {
 public:
  SlqRun(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, double tol, bool reorth,
         DeviceLogdet* dev_out, const SlqBatch* bt)
      : m_(m), n_(m->n), seed_(seed), n_probes_(n_probes), n_steps_(n_steps), tol_(tol), reorth_(reorth),
        dev_out_(dev_out) {
    // a batch: R problems stacked along the rows, each with its own Lanczos
    // state, coefficients, partial sums and estimate (dev_out[r])
    if (bt) {
      batch_ = true;
      bt_ = *bt;
      R_ = bt->R;
      gl_.off = gj_.off = bt->off;
      gl_.pstride = 32 * kRedBlocks;
      gj_.pstride = kRedBlocks;
    }
    nrow_ = batch_ ? bt_.nmax : n_;
    tstride_ = static_cast<int64_t>(32) * n_steps;
    // the step's kernels: per-problem partial sums 64 x kRedBlocks apart
    if (batch_) gf_ = Seg{bt_.off, 64 * kRedBlocks};
    perm_ = batch_ ? bt_.perm : m->ds->perm;
    const bool dev = dev_out != nullptr;
    bf_ = slq_bufs<T>(c, n_, n_probes, n_steps, reorth, R_, dev);
    V_ = bf_.V;
    Vp_ = bf_.Vp;
    W_ = bf_.W;
    const unsigned Ry = static_cast<unsigned>(R_);
    hipLaunchKernelGGL((k_scale_vec<T>), dim3(grid_for(n_, kThreads)), dim3(kThreads), 0, c->stream, n_, m->diag,
                       bf_.sc);
    check_launch("slq scale");
    if (dev) {
      // Jacobi part, probe results and failure flags stay on the device
      hipLaunchKernelGGL(k_logsum_part, dim3(kRedBlocks, Ry), dim3(kThreads), 0, c->stream, nrow_, m->diag, bf_.jpart,
                         gj_);
      hipLaunchKernelGGL(k_sum_part, dim3(1, Ry), dim3(kThreads), 0, c->stream, bf_.jpart, kRedBlocks, bf_.djac, gj_);
      GPS_HIP(hipMemsetAsync(bf_.bad, 0, sizeof(int) * R_, c->stream));
    } else {
      jac_ = logsum_f64(c, m->diag, n_);
    }
  }

  bool unit(gp_ctx* c) override {
    if (p0_ >= n_probes_) return finish(c);
    const int ld = 32;
    const unsigned Ry = static_cast<unsigned>(R_);
    const bool dev = dev_out_ != nullptr;
    LzState* st = bf_.st;
    if (j_ == 0) {
      k_ = std::min(32, n_probes_ - p0_);
      const double inv0 = 1.0 / std::sqrt(static_cast<double>(n_));  // v_1 = +-1 / sqrt(n)
      if (dev) {
        hipLaunchKernelGGL(k_lz_state_init, dim3(1, Ry), dim3(32), 0, c->stream, st, k_, inv0,
                           batch_ ? bt_.inv0 : nullptr);
      } else {
        LzState init{};
        for (int l = 0; l < 32; ++l) {
          init.active[l] = l < k_ ? 1 : 0;
          init.inv_cur[l] = l < k_ ? inv0 : 0.0;
        }
        LzState* hst = static_cast<LzState*>(pinned_for_write(c, sizeof(LzState)));
        *hst = init;
        h2d_async(c, st, hst, sizeof(LzState));
        GPS_HIP(hipMemsetAsync(bf_.bad, 0, sizeof(int), c->stream));
      }
      hipLaunchKernelGGL((k_lz_init<T>), dim3(grid_for(n_ * ld, kThreads)), dim3(kThreads), 0, c->stream, n_, k_, ld,
                         p0_, seed_, perm_, V_, Vp_);
      check_launch("lanczos init");
    }
    if (j_ < n_steps_) {
      step(c, j_);
      if (++j_ < n_steps_) return true;
    }
    hipLaunchKernelGGL(k_quadrature, dim3((k_ + kQuadProbes - 1) / kQuadProbes, Ry), dim3(kQuadProbes), 0,
                       c->stream, k_, bf_.Ta, bf_.Tb, st, static_cast<double>(n_), bf_.gam, bf_.bad, gl_, tstride_);
    check_launch("quadrature");
    if (dev) {
      hipLaunchKernelGGL(k_slq_collect, dim3(1, Ry), dim3(32), 0, c->stream, st, bf_.gam, k_, p0_, bf_.gam_all,
                         bf_.steps_all, n_probes_);
      check_launch("slq collect");
    } else {
      double* hg = static_cast<double*>(pinned(c, sizeof(double) * 32 + sizeof(LzState) + 16));
      GPS_HIP(hipMemcpyAsync(hg, bf_.gam, sizeof(double) * 32, hipMemcpyDeviceToHost, c->stream));
      LzState* hs2 = reinterpret_cast<LzState*>(hg + 32);
      GPS_HIP(hipMemcpyAsync(hs2, st, sizeof(LzState), hipMemcpyDeviceToHost, c->stream));
      int* hb = reinterpret_cast<int*>(reinterpret_cast<char*>(hs2) + sizeof(LzState));
      GPS_HIP(hipMemcpyAsync(hb, bf_.bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      sync(c);
      for (int l = 0; l < k_; ++l) {
        gammas_.push_back(hg[l]);
        max_steps_ = std::max(max_steps_, hs2->steps[l]);
      }
      nbad_ |= *hb;
    }
    j_ = 0;
    p0_ += 32;
    if (p0_ < n_probes_) return true;
    return finish(c);
  }

  // the steps run beside a solve on the other stream: their products leave
  // wave slots to it
  void beside_solve() { beside_ = true; }

  // the host-driven form's estimate, after the last unit
  LogdetResult result() const {
    LogdetResult res;
    if (dev_out_) return res;
    double mean = 0;
    for (double g : gammas_) mean += g;
    mean /= static_cast<double>(gammas_.size());
    double var = 0;
    for (double g : gammas_) var += (g - mean) * (g - mean);
    res.se = gammas_.size() > 1 ? std::sqrt(var / static_cast<double>(gammas_.size() - 1) / gammas_.size()) : 0.0;
    res.logdet = jac_ + mean;
    res.steps = max_steps_;
    if (nbad_ & 2) res.st = GP_ENOTPD;
    if (nbad_ & 1) res.st = GP_EDEVICE;
    return res;
  }

 private:
  // the estimate from the per-probe results (device-driven form); no units left
  bool finish(gp_ctx* c) {
    if (dev_out_ && !finished_) {
      hipLaunchKernelGGL(k_slq_final, dim3(1, static_cast<unsigned>(R_)), dim3(1), 0, c->stream, bf_.gam_all,
                         bf_.steps_all, n_probes_, bf_.djac, bf_.bad, dev_out_);
      check_launch("slq final");
    }
    finished_ = true;
    return false;
  }

  // Lanczos step j of the current block
  void step(gp_ctx* c, int j) {
    const int ld = 32;
    const unsigned Ry = static_cast<unsigned>(R_);
    const int last = j == n_steps_ - 1;
    LzState* st = bf_.st;
    double* part = bf_.part;
    // W = S K S V; the sums of V W and alpha; one pass applies inv_cur and
    // both subtractions
    spmm<T>(c, m_, ld, ld, V_, W_, bf_.sc, nullptr, beside_);
    ProfScope ps(c, "lanczos_vector_ops");
    hipLaunchKernelGGL((k_lz_vw_part<T>), dim3(kRedBlocks, Ry), dim3(kThreads), 0, c->stream, nrow_, ld, V_, W_, part,
                       gf_);
    hipLaunchKernelGGL(k_lz_fin, dim3(1, Ry), dim3(kFinGroups * 32), 0, c->stream, part, kRedBlocks, k_, 0, j, last,
                       tol_, st, bf_.Ta, bf_.Tb, gf_, tstride_);
    hipLaunchKernelGGL((k_lz_update<T>), dim3(kRedBlocks, Ry), dim3(kThreads), 0, c->stream, nrow_, ld, st, V_, Vp_,
                       W_, part, gf_);
    if (reorth_) {
      // W -= Q Q^T W twice over q_0 .. q_j, then |W|^2 and W . V afresh
      double* Qj = bf_.Qall + static_cast<int64_t>(j) * n_ * ld;
      hipLaunchKernelGGL(k_lz_store_q, dim3(grid_for(n_ * ld, kThreads)), dim3(kThreads), 0, c->stream, n_, V_, st,
                         Qj);
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_ro_dot, dim3(kRoBlocks, j + 1), dim3(kThreads), 0, c->stream, n_, bf_.Qall, W_,
                           bf_.ropart);
        hipLaunchKernelGGL(k_ro_fin, dim3(j + 1), dim3(32), 0, c->stream, bf_.ropart, kRoBlocks, bf_.H);
        hipLaunchKernelGGL(k_ro_update, dim3(grid_for(n_ * ld, kThreads)), dim3(kThreads), 0, c->stream, n_, j + 1,
                           bf_.Qall, bf_.H, W_);
      }
      hipLaunchKernelGGL(k_lz_norm_dot, dim3(kRedBlocks), dim3(kThreads), 0, c->stream, n_, V_, W_, part);
      check_launch("lanczos reorthogonalisation");
    }
    hipLaunchKernelGGL(k_lz_fin, dim3(1, Ry), dim3(kFinGroups * 32), 0, c->stream, part, kRedBlocks, k_, 1, j, last,
                       tol_, st, bf_.Ta, bf_.Tb, gf_, tstride_);
    if (!last) {
      // rotate: the residual block W holds the next (unnormalised) v
      T* old_prev = Vp_;
      Vp_ = V_;
      V_ = W_;
      W_ = old_prev;
    }
    check_launch("lanczos step");
  }

  const gp_matrix* m_;
  int64_t n_, nrow_ = 0, tstride_ = 0;
  uint64_t seed_;
  int n_probes_, n_steps_, R_ = 1;
  double tol_;
  bool reorth_, batch_ = false, finished_ = false, beside_ = false;
  Seg gf_;  // problems of the step's kernels
  DeviceLogdet* dev_out_;
  SlqBatch bt_;
  Seg gl_, gj_;
  const int32_t* perm_ = nullptr;
  SlqBufs<T> bf_;
  T *V_ = nullptr, *Vp_ = nullptr, *W_ = nullptr;
  double jac_ = 0.0;
  std::vector<double> gammas_;
  int max_steps_ = 0, nbad_ = 0;
  int p0_ = 0, j_ = 0, k_ = 0;  // current probe block and step
};

template <typename T>
static LogdetResult slq_impl(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, double tol,
                             bool reorth, DeviceLogdet* dev_out = nullptr, const SlqBatch* bt = nullptr) {
  SlqRun<T> run(c, m, seed, n_probes, n_steps, tol, reorth, dev_out, bt);
  while (run.unit(c)) {
  }
  return run.result();
}

// Lanczos vectors, products and reductions are float64 for both forms; the
// mixed form reads float32 matrix values.  Rounding the product's input or
// accumulating it in float32 perturbs each step by ~1e-7, which the
// recurrence's loss of orthogonality amplifies to ~5e-5 in the quadrature at
// 50 steps; float32 values alone move the estimate by ~5e-8.
LogdetResult slq_logdet(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, bool reorth) {
  return slq_impl<double>(c, m, seed, n_probes, n_steps, 1e-10, reorth);
}

void slq_logdet_device(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, bool reorth,
                       DeviceLogdet* out) {
  slq_impl<double>(c, m, seed, n_probes, n_steps, 1e-10, reorth, out);
}

void slq_logdet_side(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, bool reorth,
                     DeviceLogdet* out) {
  fork_side(c);
  std::unique_ptr<SideFeed> run;
  {
    SideScope side(c);
    auto r = std::make_unique<SlqRun<double>>(c, m, seed, n_probes, n_steps, 1e-10, reorth, out, nullptr);
    r->beside_solve();
    run = std::move(r);
  }
  side_install(c, std::move(run));
}

void slq_batch_side(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, const SlqBatch& b,
                    DeviceLogdet* out) {
  fork_side(c);
  std::unique_ptr<SideFeed> run;
  {
    SideScope side(c);
    auto r = std::make_unique<SlqRun<double>>(c, m, seed, n_probes, n_steps, 1e-10, false, out, &b);
    r->beside_solve();
    run = std::move(r);
  }
  side_install(c, std::move(run));
}

void slq_reserve(gp_ctx* c, const gp_matrix* m, int n_probes, int n_steps, bool reorth, int R) {
  (void)slq_bufs<double>(c, m->n, n_probes, n_steps, reorth, R, true);
  spmm_reserve(c, m);
}

void slq_logdet_batch(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, const SlqBatch& b,
                      DeviceLogdet* out) {
  slq_impl<double>(c, m, seed, n_probes, n_steps, 1e-10, false, out, &b);
}

// Exact log det: Lanczos on the Jacobi-scaled matrix to dimension n with full
// re-orthogonalisation (classical Gram-Schmidt, twice); on breakdown restart
// with a fresh probe orthogonalised against the basis (T splits into blocks).
// log det T from the pivots of T = L D L^T (T is positive definite).
LogdetResult exact_logdet(gp_ctx* c, const gp_matrix* m, uint64_t seed) {
  const int64_t n = m->n;
  GPS_REQUIRE(n <= 8192, GP_EINVAL, "exact log-det mode is limited to n <= 8192");
  double* Vb = static_cast<double*>(workspace(c, 50, sizeof(double) * n * n));
  double* w = static_cast<double*>(workspace(c, 51, sizeof(double) * n));
  double* h = static_cast<double*>(workspace(c, 52, sizeof(double) * n));
  double* sc = static_cast<double*>(workspace(c, 53, sizeof(double) * n));
  const dim3 B(kThreads), Gn(grid_for(n, kThreads));
  hipLaunchKernelGGL((k_scale_vec<double>), Gn, B, 0, c->stream, n, m->diag, sc);
  check_launch("exact scale");
  const double jac = logsum_f64(c, m->diag, n);
  std::vector<double> al, be;  // be[j] couples j and j+1 (0 at restarts)
  uint64_t probe = 0;
  auto orth2 = [&](int nv) {
    for (int pass = 0; pass < 2 && nv > 0; ++pass) {
      hipLaunchKernelGGL(k_gemv_t, dim3(nv), B, 0, c->stream, n, nv, Vb, w, h);
      hipLaunchKernelGGL(k_gemv_n_sub, Gn, B, 0, c->stream, n, nv, Vb, h, w);
    }
    check_launch("reorthogonalise");
  };
  auto start_vector = [&](int nv) -> bool {
    for (int tries = 0; tries < 8; ++tries) {
      hipLaunchKernelGGL(k_probe_vec, Gn, B, 0, c->stream, n, seed, probe++, m->ds->perm, w);
      check_launch("probe");
      const double n0 = std::sqrt(static_cast<double>(n));
      orth2(nv);
      const double nr = std::sqrt(dot_f64(c, w, w, n));
      if (nr > 1e-6 * n0) {
        hipLaunchKernelGGL(k_scale_into, Gn, B, 0, c->stream, n, 1.0 / nr, w, Vb + static_cast<int64_t>(nv) * n);
        check_launch("normalise");
        return true;
      }
    }
    return false;
  };
  LogdetResult res;
  if (!start_vector(0)) throw Error{GP_EDEVICE, "exact log-det: could not start"};
  double beta_prev = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    const double* vj = Vb + j * n;
    spmm<double>(c, m, 1, 1, vj, w, sc);
    const double a = dot_f64(c, vj, w, n);
    const double* vprev = j > 0 ? Vb + (j - 1) * n : vj;
    hipLaunchKernelGGL(k_axpby2, Gn, B, 0, c->stream, n, a, vj, j > 0 ? beta_prev : 0.0, vprev, w);
    check_launch("lanczos axpy");
    orth2(static_cast<int>(j + 1));
    al.push_back(a);
    if (j == n - 1) break;
    const double b = std::sqrt(dot_f64(c, w, w, n));
    if (b > 1e-10) {
      be.push_back(b);
      hipLaunchKernelGGL(k_scale_into, Gn, B, 0, c->stream, n, 1.0 / b, w, Vb + (j + 1) * n);
      check_launch("lanczos normalise");
      beta_prev = b;
    } else {
      be.push_back(0.0);
      if (!start_vector(static_cast<int>(j + 1))) throw Error{GP_EDEVICE, "exact log-det: restart failed"};
      beta_prev = 0.0;
    }
  }
  double ld = 0, piv = 0;
  for (size_t j = 0; j < al.size(); ++j) {
    piv = j == 0 || be[j - 1] == 0.0 ? al[j] : al[j] - be[j - 1] * be[j - 1] / piv;
    if (!(piv > 0)) {
      res.st = GP_ENOTPD;
      break;
    }
    ld += std::log(piv);
  }
  res.logdet = jac + ld;
  res.se = 0;
  res.steps = static_cast<int>(al.size());
  return res;
}

}  // namespace gps
