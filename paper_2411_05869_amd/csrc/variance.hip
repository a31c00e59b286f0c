// Posterior variance of the latent process at test points (Sec. 3.2): the
// diagonal of C_{y|z} = C_y - C_{y,z} C_z^{-1} C_{z,y},
//   v(x*) = C_y(x*, x*) - c^T K^{-1} c,   c = C_{z,y}(., x*),
// for 32 test points at a time:
//   1. the cross-covariance columns c_s are written into an n x 32 block X
//      (rows in binned order): a thread per test point adds the local
//      (Wendland) entries of its cell window, then a wave per test point adds
//      the bump-group entries over the masked training points;
//   2. K W = X is solved by 32 conjugate-gradient recurrences in lockstep
//      (one SpMM per step; block-Jacobi or Jacobi preconditioner; per-column
//      scalars; a column
//      stops changing once |r_s| <= rtol |c_s|), with a float64 true residual
//      X - K W at the end (the recurrences restart from it if it is not small
//      enough);
//   3. v_s = C_y(x*_s, x*_s) - sum_q X[q, s] W[q, s].
// Every reduction adds partial sums in a fixed order, so results are
// reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "device.hpp"

namespace gps {
namespace {

constexpr int kThreads = 256;
constexpr int kC = 32;                 // right-hand sides per batch
constexpr int kRowsPer = kThreads / kC;  // rows handled together by a block
constexpr unsigned kVBlocks = 1024;    // blocks of the column-reduction kernels
constexpr int kRowBatch = 4;           // strided rows a thread loads at once in the column reductions
constexpr int kCheckEvery = 8;
constexpr int kMaxRefresh = 3;

struct CrossArgs {
  KernelTheta kt;
  int64_t n;
  const double* xb;
  const int32_t* cell_start;
  double lo[3], cell[3];
  int32_t g[3], R[3];
  int64_t nm;
  const int32_t* mlist;
  const uint64_t* mmask;
  const double* F;  // nm x n1
};

struct BcgScalars {
  double rz[kC], pq[kC], alpha[kC], beta[kC], rr[kC], cc[kC];
  int32_t active[kC];
  int32_t status;
};

template <int D>
__device__ __forceinline__ void load_train(const CrossArgs& a, int64_t q, double* x) {
  x[0] = a.xb[q];
  if constexpr (D >= 2) x[1] = a.xb[a.n + q];
  if constexpr (D >= 3) x[2] = a.xb[2 * a.n + q];
}

// X[., s] = 0 for the block
__global__ void __launch_bounds__(kThreads) k_zero(int64_t len, double* __restrict__ X) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    X[i] = 0.0;
}

// local part of c_s: C_core(x*, x_q) s0 f0(u) for the training points of the
// cell window with u0^2 < 1 (each q once)
template <int D, int CK>
__global__ void __launch_bounds__(kThreads) k_cross_local(CrossArgs a, CoreBasis cb, int nb,
                                                          const double* __restrict__ xs, double* __restrict__ X) {
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= nb) return;
  double xp[3];
  int c[3] = {0, 0, 0};
  for (int k = 0; k < D; ++k) {
    xp[k] = xs[static_cast<int64_t>(s) * D + k];
    c[k] = cell_coord(xp[k], a.lo[k], a.cell[k]);
  }
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int k = 0; k < D; ++k) {
    lo[k] = max(c[k] - a.R[k], 0);
    hi[k] = min(c[k] + a.R[k], a.g[k] - 1);
    if (lo[k] > hi[k]) return;
  }
  double sp = 0.0, Sp = 0.0;
  if constexpr (CK == 2) core_point_fields<D>(cb, xp, &sp, &Sp);
  for (int z = lo[2]; z <= hi[2]; ++z)
    for (int y = lo[1]; y <= hi[1]; ++y) {
      const int64_t base = (static_cast<int64_t>(z) * a.g[1] + y) * a.g[0];
      const int32_t b = a.cell_start[base + lo[0]];
      const int32_t e = a.cell_start[base + hi[0] + 1];
      for (int32_t q = b; q < e; ++q) {
        double xq[3];
        load_train<D>(a, q, xq);
        const double u2 = scaled_sq<D>(xp, xq, a.kt.inv0);
        if (u2 < 1.0) {
          double v = a.kt.s0 * wendland(u2, a.kt.variant);
          if constexpr (CK == 1) v = core_value<D, 1>(a.kt.core, xp, xq, 0.0, 0.0, 0.0, 0.0) * v;
          if constexpr (CK == 2)
            v = core_value<D, 2>(a.kt.core, xp, xq, sp, Sp, a.kt.core.sig[q], a.kt.core.Sig[q]) * v;
          X[static_cast<int64_t>(q) * kC + s] = v;
        }
      }
    }
}

// bump-group part of c_s and the prior variance C_y(x*, x*): one wave per
// test point; lane i < n1 forms f_i(x*) (bumps of group i in j order)
template <int D, int CK>
__global__ void __launch_bounds__(kThreads) k_cross_groups(CrossArgs a, CoreBasis cb, int nb,
                                                           const double* __restrict__ xs, double* __restrict__ X,
                                                           double* __restrict__ prior) {
  __shared__ double fs[kThreads / kWave][kWave];
  const int s = (blockIdx.x * kThreads + threadIdx.x) / kWave;
  if (s >= nb) return;  // uniform per wave
  const int lane = lane_id();
  double* f = fs[threadIdx.x / kWave];
  double xp[3];
  for (int k = 0; k < D; ++k) xp[k] = xs[static_cast<int64_t>(s) * D + k];
  bool in_group = false;
  double fi = 0.0;
  if (lane < a.kt.n1) {
#pragma clang fp contract(off)
    for (int j = 0; j < a.kt.n2; ++j) {
      const Bump& bp = a.kt.bumps[lane * a.kt.n2 + j];
      const double ub2 = scaled_sq<D>(xp, bp.h, bp.inv);
      if (bp.a > 0.0 && ub2 < 1.0) {
        in_group = true;
        fi = fi + bp.a * exp(bp.b * (1.0 - 1.0 / (1.0 - ub2)));
      }
    }
  }
  const uint64_t mask = __ballot(in_group);
  f[lane] = fi;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double sp = 0.0, Sp = 0.0;
  if constexpr (CK == 2) core_point_fields<D>(cb, xp, &sp, &Sp);
  if (lane == 0) {
#pragma clang fp contract(off)
    double v = a.kt.s0 * wendland(0.0, a.kt.variant);
    uint64_t mm = mask;
    while (mm) {
      const int i = __builtin_ctzll(mm);
      mm &= mm - 1;
      v = v + f[i] * f[i];
    }
    if constexpr (CK == 1) v = core_value<D, 1>(a.kt.core, xp, xp, 0.0, 0.0, 0.0, 0.0) * v;
    if constexpr (CK == 2) v = core_value<D, 2>(a.kt.core, xp, xp, sp, Sp, sp, Sp) * v;
    prior[s] = v;
  }
  if (mask == 0) return;  // uniform
  for (int64_t j = lane; j < a.nm; j += kWave) {
    uint64_t sh = a.mmask[j] & mask;
    if (!sh) continue;
    double bsum = 0.0;
    while (sh) {
      const int i = __builtin_ctzll(sh);
      sh &= sh - 1;
      bsum += f[i] * a.F[j * a.kt.n1 + i];
    }
    const int32_t q = a.mlist[j];
    if constexpr (CK != 0) {
      double xq[3];
      load_train<D>(a, q, xq);
      if constexpr (CK == 1)
        bsum = core_value<D, 1>(a.kt.core, xp, xq, 0.0, 0.0, 0.0, 0.0) * bsum;
      else
        bsum = core_value<D, 2>(a.kt.core, xp, xq, sp, Sp, a.kt.core.sig[q], a.kt.core.Sig[q]) * bsum;
    }
    // one wave owns column s, so these read-modify-writes do not race
    X[static_cast<int64_t>(q) * kC + s] += bsum;
  }
}

// ------------------------------------------------------- column reductions
// Thread (r, col) = (threadIdx.x / 32, threadIdx.x % 32) takes rows r, r + 8,
// ... of the block's share; per block and column the NV partial sums go to
// part[(blockIdx.x * NV + v) * 32 + col].
template <int NV>
__device__ __forceinline__ void col_partials(const double (&v)[NV], double* __restrict__ part) {
  __shared__ double sh[NV][kRowsPer][kC];
  const int col = threadIdx.x % kC, r = threadIdx.x / kC;
#pragma unroll
  for (int i = 0; i < NV; ++i) sh[i][r][col] = v[i];
  __syncthreads();
  if (threadIdx.x < kC) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int rr = 0; rr < kRowsPer; ++rr) s += sh[i][rr][col];
      part[(static_cast<int64_t>(blockIdx.x) * NV + i) * kC + col] = s;
    }
  }
}

// Column totals of the partials of nb blocks, in a fixed order: thread
// (chunk, col) = (threadIdx.x / 32, threadIdx.x % 32) of a kFinThreads-thread
// block adds the partials of its chunk of consecutive blocks, then thread col
// adds the chunks in order.  tot[v] is valid in threads 0..31 (column
// threadIdx.x); every thread of the block must call it.
constexpr int kFinThreads = 1024;
constexpr int kChunks = kFinThreads / kC;

template <int NV>
__device__ __forceinline__ void col_totals(const double* __restrict__ part, int nb, double (&tot)[NV]) {
  __shared__ double sh[NV][kChunks][kC];
  const int col = threadIdx.x % kC, ch = threadIdx.x / kC;
  const int per = (nb + kChunks - 1) / kChunks;
  const int b0 = min(nb, ch * per), b1 = min(nb, b0 + per);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double s = 0.0;
    for (int b = b0; b < b1; ++b) s += part[(static_cast<int64_t>(b) * NV + v) * kC + col];
    sh[v][ch][col] = s;
  }
  __syncthreads();
  if (threadIdx.x < kC) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double s = 0.0;
      for (int c = 0; c < kChunks; ++c) s += sh[v][c][col];
      tot[v] = s;
    }
  }
}

// Preconditioner of the recurrences: the matrix diagonal, or (binv set) the
// block-Jacobi inverses over the binning cells (row-major per block).  Row i of
// z = M^-1 r needs r on the rows of its block; the caller passes a function
// that forms r for any row, so every thread sees the same values without
// waiting for the others.
struct VarPrecond {
  const double* diag;
  const int32_t* rowblk;
  const int32_t* bstart;
  const int64_t* boff;
  const double* binv;
};

template <typename F>
__device__ __forceinline__ double var_precond(const VarPrecond& M, int64_t i, double ri, F&& r_at) {
  if (!M.binv) return ri / M.diag[i];
  const int32_t b = M.rowblk[i];
  const int32_t bs = M.bstart[b];
  const int sz = M.bstart[b + 1] - bs;
  const double* row = M.binv + M.boff[b] + static_cast<int64_t>(i - bs) * sz;
  double z = 0.0;
  for (int j = 0; j < sz; ++j) z += row[j] * r_at(bs + j);
  return z;
}

#define ROW_LOOP(n)                                                                                 \
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRowsPer + threadIdx.x / kC; i < (n);       \
       i += static_cast<int64_t>(gridDim.x) * kRowsPer)

// R = X - KW (KW given, or W = 0 when kw is null); Z = R / diag; P = Z;
// partials of r.z and r.r
__global__ void __launch_bounds__(kThreads) k_bcg_start(int64_t n, const double* __restrict__ X,
                                                        const double* __restrict__ kw, VarPrecond M,
                                                        double* __restrict__ R, double* __restrict__ Z,
                                                        double* __restrict__ P, double* __restrict__ part) {
  const int col = threadIdx.x % kC;
  double v[2] = {0.0, 0.0};
  ROW_LOOP(n) {
    const int64_t e = i * kC + col;
    auto r_at = [&](int64_t q) { return kw ? X[q * kC + col] - kw[q * kC + col] : X[q * kC + col]; };
    const double r = r_at(i);
    const double z = var_precond(M, i, r, r_at);
    R[e] = r;
    Z[e] = z;
    P[e] = z;
    v[0] += r * z;
    v[1] += r * r;
  }
  col_partials<2>(v, part);
}

// mode 0: first start (|c|^2 = r.r, a column with c = 0 is never active);
// mode 1: restart from the true residual (active columns stay active)
__global__ void __launch_bounds__(kFinThreads) k_bcg_start_fin(const double* __restrict__ part, int nb,
                                                               BcgScalars* __restrict__ S, double tol2, int mode) {
  double t[2];
  col_totals<2>(part, nb, t);
  if (threadIdx.x >= kC) return;
  const int col = threadIdx.x;
  const double rz = t[0], rr = t[1];
  S->rz[col] = rz;
  S->rr[col] = rr;
  if (mode == 0) {
    S->cc[col] = rr;
    S->active[col] = rr > 0.0 ? 1 : 0;
    if (col == 0) S->status = 0;
  } else {
    S->active[col] = rr > tol2 * S->cc[col] ? 1 : 0;
  }
}

__global__ void __launch_bounds__(kThreads) k_bcg_pq(int64_t n, const double* __restrict__ P,
                                                     const double* __restrict__ Q, double* __restrict__ part) {
  // four strided rows loaded at once, added in the order of the plain row loop
  const int col = threadIdx.x % kC;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kRowsPer;
  double v[1] = {0.0};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kRowsPer + threadIdx.x / kC; i < n; i += kRowBatch * stride) {
    double pv[kRowBatch], qv[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int64_t k = i + u * stride;
      pv[u] = k < n ? P[k * kC + col] : 0.0;
      qv[u] = k < n ? Q[k * kC + col] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u)
      if (i + u * stride < n) v[0] += pv[u] * qv[u];
  }
  col_partials<1>(v, part);
}

__global__ void __launch_bounds__(kFinThreads) k_bcg_alpha(const double* __restrict__ part, int nb,
                                                           BcgScalars* __restrict__ S) {
  double t[1];
  col_totals<1>(part, nb, t);
  if (threadIdx.x >= kC) return;
  const int col = threadIdx.x;
  const double pq = t[0];
  S->pq[col] = pq;
  double a = 0.0;
  if (S->active[col]) {
    if (pq > 0.0 && isfinite(pq)) {
      a = S->rz[col] / pq;
    } else {
      S->status = 1;  // non-positive curvature
      S->active[col] = 0;
    }
  }
  S->alpha[col] = a;
}

// W += alpha P; Rout = Rin - alpha Q; Z = M^-1 Rout; partials of r.z and r.r.
// The residual alternates between two buffers: the block product reads the
// old residual of the neighbouring rows, which no thread overwrites.
__global__ void __launch_bounds__(kThreads) k_bcg_update(int64_t n, const BcgScalars* __restrict__ S,
                                                         const double* __restrict__ P, const double* __restrict__ Q,
                                                         VarPrecond M, double* __restrict__ W,
                                                         const double* __restrict__ Rin, double* __restrict__ Rout,
                                                         double* __restrict__ Z, double* __restrict__ part) {
  const int col = threadIdx.x % kC;
  const double a = S->alpha[col];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kRowsPer;
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kRowsPer + threadIdx.x / kC;
  // the next row's R, Q, W and P are requested before the current row is
  // processed (same arithmetic, same order)
  double rn = 0.0, qn = 0.0, wn = 0.0, pn = 0.0;
  if (i0 < n) {
    const int64_t e = i0 * kC + col;
    rn = Rin[e], qn = Q[e], wn = W[e], pn = P[e];
  }
  double v[2] = {0.0, 0.0};
  for (int64_t i = i0; i < n; i += stride) {
    const int64_t e = i * kC + col;
    const double ri = rn, qi = qn, wi = wn, pi = pn;
    if (i + stride < n) {
      const int64_t f = (i + stride) * kC + col;
      rn = Rin[f], qn = Q[f], wn = W[f], pn = P[f];
    }
    // the new residual of any row of the block, formed as for the row itself
    auto r_at = [&](int64_t q) { return Rin[q * kC + col] - a * Q[q * kC + col]; };
    const double r = ri - a * qi;
    const double z = var_precond(M, i, r, r_at);
    W[e] = wi + a * pi;
    Rout[e] = r;
    Z[e] = z;
    v[0] += r * z;
    v[1] += r * r;
  }
  col_partials<2>(v, part);
}

__global__ void __launch_bounds__(kFinThreads) k_bcg_beta(const double* __restrict__ part, int nb,
                                                          BcgScalars* __restrict__ S, double tol2) {
  double t[2];
  col_totals<2>(part, nb, t);
  if (threadIdx.x >= kC) return;
  const int col = threadIdx.x;
  const double rz = t[0], rr = t[1];
  const bool act = S->active[col] != 0;
  S->beta[col] = act ? rz / S->rz[col] : 0.0;
  S->rz[col] = rz;
  S->rr[col] = rr;
  S->active[col] = (act && rr > tol2 * S->cc[col]) ? 1 : 0;
}

// P = Z + beta P for the active columns
__global__ void __launch_bounds__(kThreads) k_bcg_dir(int64_t n, const BcgScalars* __restrict__ S,
                                                      const double* __restrict__ Z, double* __restrict__ P) {
  const int col = threadIdx.x % kC;
  if (!S->active[col]) return;  // the whole column; no block-level synchronisation follows
  const double b = S->beta[col];
  ROW_LOOP(n) {
    const int64_t e = i * kC + col;
    P[e] = Z[e] + b * P[e];
  }
}

// partials of the true residual |X - KW|^2 and of X.W per column
__global__ void __launch_bounds__(kThreads) k_bcg_final(int64_t n, const double* __restrict__ X,
                                                        const double* __restrict__ kw, const double* __restrict__ W,
                                                        double* __restrict__ part) {
  const int col = threadIdx.x % kC;
  double v[2] = {0.0, 0.0};
  ROW_LOOP(n) {
    const int64_t e = i * kC + col;
    const double r = X[e] - kw[e];
    v[0] += r * r;
    v[1] += X[e] * W[e];
  }
  col_partials<2>(v, part);
}

// true residual per column into S->rr; v_s = prior_s - c_s . w_s for s < nbatch
__global__ void __launch_bounds__(kFinThreads) k_bcg_var(const double* __restrict__ part, int nb,
                                                         BcgScalars* __restrict__ S, const double* __restrict__ prior,
                                                         int nbatch, double* __restrict__ var) {
  double t[2];
  col_totals<2>(part, nb, t);
  if (threadIdx.x >= kC) return;
  const int col = threadIdx.x;
  const double rr = t[0], cw = t[1];
  S->rr[col] = rr;
  if (col < nbatch) var[col] = prior[col] - cw;
}

#undef ROW_LOOP

template <typename F3>
void dispatch_dk(int d, int kind, F3&& f) {
  auto with_d = [&](auto DD) {
    if (kind == GP_CORE_MATERN)
      f(DD, std::integral_constant<int, 1>{});
    else if (kind == GP_CORE_PACIOREK)
      f(DD, std::integral_constant<int, 2>{});
    else
      f(DD, std::integral_constant<int, 0>{});
  };
  if (d == 1)
    with_d(std::integral_constant<int, 1>{});
  else if (d == 2)
    with_d(std::integral_constant<int, 2>{});
  else
    with_d(std::integral_constant<int, 3>{});
}

}  // namespace

VarResult predict_variance(gp_ctx* c, const gp_matrix* m, const gp_theta* th, int64_t ntest, const double* xs,
                           double rtol, int max_iter, int precond, double* var) {
  VarResult res;
  if (ntest == 0) return res;
  VarPrecond M{m->diag, nullptr, nullptr, nullptr, nullptr};
  if (precond == GP_PRECOND_BLOCK_JACOBI) {
    // the inverses are cached in the matrix object on first use
    gp_matrix* mm = const_cast<gp_matrix*>(m);
    build_block_jacobi(c, mm);
    M.rowblk = mm->rowblk;
    M.bstart = mm->bstart;
    M.boff = mm->boff;
    M.binv = mm->binv;
  }
  const gp_dataset* ds = m->ds;
  const int64_t n = m->n;
  const int d = ds->d;
  Bump* bumps = nullptr;
  KernelTheta kt{};
  upload_theta(c, th, &bumps, &kt);
  CoreBasis cb{};
  core_params(th, &kt.core, &cb);
  if (kt.core.kind == GP_CORE_PACIOREK) {
    double* sig = static_cast<double*>(workspace(c, 92, sizeof(double) * n));
    double* Sig = static_cast<double*>(workspace(c, 93, sizeof(double) * n));
    core_fields(c, ds, cb, sig, Sig);
    kt.core.sig = sig;
    kt.core.Sig = Sig;
  }
  Features f;
  if (th->n1 > 0) compute_features(c, ds, kt, &f, 100);
  const Grid grid = make_grid(ds, th);
  CrossArgs a{};
  a.kt = kt;
  a.n = n;
  a.xb = ds->xb;
  a.cell_start = ds->cell_start;
  for (int k = 0; k < 3; ++k) {
    a.lo[k] = ds->lo[k];
    a.cell[k] = ds->cell[k];
    a.g[k] = ds->g[k];
    a.R[k] = grid.R[k];
  }
  a.nm = f.nm;
  a.mlist = f.mlist;
  a.mmask = f.mmask;
  a.F = f.F;

  const size_t blk = sizeof(double) * n * kC;
  double* X = static_cast<double*>(workspace(c, 110, blk));
  double* R = static_cast<double*>(workspace(c, 111, blk));
  double* R2 = static_cast<double*>(workspace(c, 119, blk));  // the residual alternates between R and R2
  double* Z = static_cast<double*>(workspace(c, 112, blk));
  double* P = static_cast<double*>(workspace(c, 113, blk));
  double* Q = static_cast<double*>(workspace(c, 114, blk));
  double* W = static_cast<double*>(workspace(c, 115, blk));
  double* part = static_cast<double*>(workspace(c, 116, sizeof(double) * kVBlocks * 2 * kC));
  BcgScalars* S = static_cast<BcgScalars*>(workspace(c, 117, sizeof(BcgScalars)));
  double* prior = static_cast<double*>(workspace(c, 118, sizeof(double) * kC));
  BcgScalars* hs = static_cast<BcgScalars*>(pinned(c, sizeof(BcgScalars)));
  const unsigned nbv = static_cast<unsigned>(std::min<int64_t>(kVBlocks, (n + kRowsPer - 1) / kRowsPer));
  const dim3 B(kThreads), G(nbv), FB(kFinThreads);
  // element-wise kernels without a reduction take a row per thread
  const dim3 Gfull(static_cast<unsigned>((n + kRowsPer - 1) / kRowsPer));
  const double tol2 = rtol * rtol;
  auto read = [&]() {
    GPS_HIP(hipMemcpyAsync(hs, S, sizeof(BcgScalars), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    return *hs;
  };
  for (int64_t m0 = 0; m0 < ntest; m0 += kC) {
    const int nb = static_cast<int>(std::min<int64_t>(kC, ntest - m0));
    const double* xb = xs + m0 * d;
    {
      ProfScope ps(c, "var_cross");
      hipLaunchKernelGGL(k_zero, dim3(grid_for(n * kC, kThreads)), B, 0, c->stream, n * kC, X);
      dispatch_dk(d, kt.core.kind, [&](auto DD, auto CC) {
        constexpr int D = decltype(DD)::value;
        constexpr int CK = decltype(CC)::value;
        hipLaunchKernelGGL((k_cross_local<D, CK>), dim3(1), B, 0, c->stream, a, cb, nb, xb, X);
        hipLaunchKernelGGL((k_cross_groups<D, CK>), dim3((nb * kWave + kThreads - 1) / kThreads), B, 0, c->stream,
                           a, cb, nb, xb, X, prior);
      });
      check_launch("variance cross-covariance");
    }
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n * kC, kThreads)), B, 0, c->stream, n * kC, W);
    hipLaunchKernelGGL(k_bcg_start, G, B, 0, c->stream, n, X, nullptr, M, R, Z, P, part);
    hipLaunchKernelGGL(k_bcg_start_fin, dim3(1), FB, 0, c->stream, part, static_cast<int>(nbv), S, tol2, 0);
    check_launch("variance start");
    BcgScalars hsc = read();
    int it = 0, refresh = 0;
    auto any_active = [](const BcgScalars& s) {
      for (int j = 0; j < kC; ++j)
        if (s.active[j]) return true;
      return false;
    };
    while (hsc.status == 0 && it < max_iter) {
      if (!any_active(hsc)) {
        // recurrences done: check the float64 true residual, restart once it is not small enough
        if (refresh >= kMaxRefresh) break;
        spmm<double>(c, m, kC, kC, W, Q, nullptr);
        hipLaunchKernelGGL(k_bcg_start, G, B, 0, c->stream, n, X, Q, M, R, Z, P, part);
        hipLaunchKernelGGL(k_bcg_start_fin, dim3(1), FB, 0, c->stream, part, static_cast<int>(nbv), S, tol2, 1);
        check_launch("variance restart");
        ++refresh;
        hsc = read();
        if (!any_active(hsc)) break;
        continue;
      }
      const int steps = std::min(kCheckEvery, max_iter - it);
      for (int t = 0; t < steps; ++t) {
        spmm<double>(c, m, kC, kC, P, Q, nullptr);
        ProfScope ps(c, "var_vector_ops");
        hipLaunchKernelGGL(k_bcg_pq, G, B, 0, c->stream, n, P, Q, part);
        hipLaunchKernelGGL(k_bcg_alpha, dim3(1), FB, 0, c->stream, part, static_cast<int>(nbv), S);
        hipLaunchKernelGGL(k_bcg_update, G, B, 0, c->stream, n, S, P, Q, M, W, R, R2, Z, part);
        std::swap(R, R2);
        hipLaunchKernelGGL(k_bcg_beta, dim3(1), FB, 0, c->stream, part, static_cast<int>(nbv), S, tol2);
        hipLaunchKernelGGL(k_bcg_dir, Gfull, B, 0, c->stream, n, S, Z, P);
        check_launch("variance step");
      }
      it += steps;
      hsc = read();
    }
    // true residual and the variances of this batch
    spmm<double>(c, m, kC, kC, W, Q, nullptr);
    hipLaunchKernelGGL(k_bcg_final, G, B, 0, c->stream, n, X, Q, W, part);
    hipLaunchKernelGGL(k_bcg_var, dim3(1), FB, 0, c->stream, part, static_cast<int>(nbv), S, prior, nb, var + m0);
    check_launch("variance final");
    hsc = read();
    res.iters += it;
    res.max_batch_iters = std::max(res.max_batch_iters, it);
    bool ok = hsc.status == 0;
    for (int j = 0; j < nb; ++j) {
      const double rel = hsc.cc[j] > 0.0 ? std::sqrt(hsc.rr[j] / hsc.cc[j]) : 0.0;
      res.relres = std::max(res.relres, rel);
      if (!(rel <= rtol)) ok = false;
    }
    if (hsc.status != 0)
      res.st = GP_ENOTPD;
    else if (!ok && res.st == GP_OK)
      res.st = GP_ENOTCONV;
  }
  return res;
}

}  // namespace gps
