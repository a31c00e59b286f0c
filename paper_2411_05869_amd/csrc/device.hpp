// Device-side building blocks shared by the assembly and prediction kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace gps {

__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ uint64_t lanes_below() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Support test of Eq. compSupp / Eq. bumpFcn: u^2 = sum_k ((p_k - q_k) * inv_k)^2,
// every operation rounded on its own, k increasing, no fused multiply-add.
// The caller compares with < 1.0.  Identical for (p, q) and (q, p).
template <int D>
__device__ __forceinline__ double scaled_sq(const double* p, const double* q, const double* inv) {
#pragma clang fp contract(off)
  double t = (p[0] - q[0]) * inv[0];
  double acc = t * t;
  if constexpr (D >= 2) {
    double t1 = (p[1] - q[1]) * inv[1];
    acc = acc + t1 * t1;
  }
  if constexpr (D >= 3) {
    double t2 = (p[2] - q[2]) * inv[2];
    acc = acc + t2 * t2;
  }
  return acc;
}

// Wendland part f0 (Eq. compSupp) from u^2 < 1: (1-u)^8 (c3 u^3 + 25 u^2 + 8 u + 1).
// Contraction is off so that every kernel rounds the same way: this keeps the
// matrix bitwise symmetric whichever kernel produced an entry.
__device__ __forceinline__ double wendland(double u2, int variant) {
#pragma clang fp contract(off)
  const double u = __builtin_sqrt(u2);
  const double t = 1.0 - u;
  const double t2 = t * t;
  const double t4 = t2 * t2;
  const double t8 = t4 * t4;
  const double c3 = variant ? 32.0 : 35.0;
  const double poly = ((c3 * u + 25.0) * u + 8.0) * u + 1.0;
  return t8 * poly;
}

// The three steps of an entry (entry_value below): the local term, one group
// term added (the caller adds them in increasing i), the core and diagonal.
__device__ __forceinline__ double entry_local(const KernelTheta& kt, double u2) {
#pragma clang fp contract(off)
  return (u2 < 1.0) ? kt.s0 * wendland(u2, kt.variant) : 0.0;
}
__device__ __forceinline__ double entry_add_group(double acc, double fp, double fq) {
#pragma clang fp contract(off)
  return acc + fp * fq;
}
__device__ __forceinline__ double entry_finish(const KernelTheta& kt, double acc, double core, bool diag,
                                               int64_t row) {
#pragma clang fp contract(off)
  acc = core * acc;
  if (diag) {
    acc = acc + kt.nugget;
    if (kt.tau2) acc = acc + kt.tau2[row];  // Delta_pp = sigma^2 + tau2[p] (Eq. Zcov)
  }
  return acc;
}

// Entry K_pq (Eq. sparseCov, Eq. C_sparse, Eq. Zcov): core x (s0 f0 [local] +
// sum over shared groups in increasing i of f_i(p) f_i(q)) + sigma^2 [p = q].
// f_i(p) = Fp[i * sp], f_i(q) = Fq[i * sq]; core = C_core(x_p, x_q), 1 without
// a core kernel (a product with 1 is exact).
__device__ __forceinline__ double entry_value(const KernelTheta& kt, double u2, uint64_t shared,
                                              const double* Fp, const double* Fq, bool diag, int64_t sp = 1,
                                              int64_t sq = 1, double core = 1.0, int64_t row = 0) {
  double acc = entry_local(kt, u2);
  while (shared) {
    const int i = __builtin_ctzll(shared);
    shared &= shared - 1;
    acc = entry_add_group(acc, Fp[i * sp], Fq[i * sq]);
  }
  return entry_finish(kt, acc, core, diag, row);
}

// Matern correlation M_nu(t) (Rasmussen-Williams scaling sqrt(2 nu) t) at
// nu = nu2 / 2 from t and t2 = t^2; nu2 = 0 is the limit exp(-t^2 / 2).
__device__ __forceinline__ double matern(double t, double t2, int nu2) {
#pragma clang fp contract(off)
  if (nu2 == 0) return exp(-0.5 * t2);
  if (nu2 == 1) return exp(-t);
  if (nu2 == 3) {
    const double a = 1.7320508075688772 * t;
    return (1.0 + a) * exp(-a);
  }
  const double a = 2.23606797749979 * t;
  return (1.0 + a + a * a / 3.0) * exp(-a);
}

// Core kernel value C_core(x_p, x_q) (Eq. sparseCov): CK = 1 stationary
// Matern sigma0^2 M_nu(|(x_p - x_q) / ell|); CK = 2 the nonstationary kernel
// of Eq. PScov from the fields (sp, Sp) at x_p and (sq, Sq) at x_q, its
// prefactor (Sp Sq)^(d/4) / ((Sp + Sq)/2)^(d/2) written as g^(d/2) with
// g = 2 sqrt(Sp Sq) / (Sp + Sq).  Every operation is symmetric in p and q, so
// the value is bitwise the same for (p, q) and (q, p).
template <int D, int CK>
__device__ __forceinline__ double core_value(const KernelCore& kc, const double* xp, const double* xq, double sp,
                                             double Sp, double sq, double Sq) {
#pragma clang fp contract(off)
  const double r2 = scaled_sq<D>(xp, xq, kc.inv_ell);
  if constexpr (CK == 1) {
    return kc.s2 * matern(__builtin_sqrt(r2), r2, kc.nu2);
  } else {
    const double sum = Sp + Sq;
    const double avg = 0.5 * sum;
    const double g = 2.0 * __builtin_sqrt(Sp * Sq) / sum;
    double pre;
    if constexpr (D == 1) pre = __builtin_sqrt(g);
    else if constexpr (D == 2) pre = g;
    else pre = g * __builtin_sqrt(g);
    const double q2 = r2 / avg;
    return (sp * sq) * pre * matern(__builtin_sqrt(q2), q2, kc.nu2);
  }
}

// sigma(x), Sigma(x) of the nonstationary core: basis functions and
// coefficients summed in increasing m.
template <int D>
__device__ __forceinline__ void core_point_fields(const CoreBasis& cb, const double* x, double* sig, double* Sig) {
#pragma clang fp contract(off)
  double ls = cb.log_sigma0, lS = cb.log_Sigma0;
  for (int m = 0; m < cb.nb; ++m) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double z = (x[k] - cb.c[m][k]) / cb.w[k];
      acc = acc + z * z;
    }
    const double s = exp(-0.5 * acc);
    ls = ls + s * cb.phi_s[m];
    lS = lS + s * cb.phi_S[m];
  }
  *sig = exp(ls);
  *Sig = exp(lS);
}

// Point features: group mask and (optionally) the bump sums f_i (Eq. bumpFcn,
// Eq. sumOfBumps), bumps of a group summed in j order.
template <int D, bool VALUES>
__device__ __forceinline__ uint64_t point_features(const KernelTheta& kt, const double* x,
                                                   double* F /* n1 values, VALUES only */) {
#pragma clang fp contract(off)
  uint64_t mask = 0;
  for (int i = 0; i < kt.n1; ++i) {
    double f = 0.0;
    bool in_group = false;
    for (int j = 0; j < kt.n2; ++j) {
      const Bump& bp = kt.bumps[i * kt.n2 + j];
      const double ub2 = scaled_sq<D>(x, bp.h, bp.inv);
      const bool inside = (bp.a > 0.0) && (ub2 < 1.0);
      if (inside) {
        in_group = true;
        if constexpr (VALUES) f = f + bp.a * exp(bp.b * (1.0 - 1.0 / (1.0 - ub2)));
      }
    }
    if (in_group) mask |= (1ull << i);
    if constexpr (VALUES) F[i] = f;
  }
  return mask;
}

// Raises the issue priority of the calling wave over other waves on its SIMD.
// The solver's kernels call it: with the log det's launches on a second
// stream sharing the CUs, the solve is the longer chain of the two.
__device__ __forceinline__ void solve_wave_priority() { __builtin_amdgcn_s_setprio(3); }

// Workgroup b of a launch runs on XCD b % 8 (each XCD has its own L2).  This
// maps b to a logical block index such that every XCD receives one contiguous
// range of logical blocks; it is a bijection on [0, nb).
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
  const unsigned q = nb / kXcds, r = nb % kXcds;
  const unsigned x = b % kXcds, i = b / kXcds;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

__device__ __forceinline__ void decode_key(int32_t key, const int32_t* g, int* c) {
  c[0] = key % g[0];
  const int32_t r = key / g[0];
  c[1] = r % g[1];
  c[2] = r / g[1];
}

// Cell coordinate of value v on an axis; clamped far outside the grid so that
// integer conversion cannot overflow (windows are clipped to the grid later).
__device__ __forceinline__ int cell_coord(double v, double lo, double cell) {
  double t = floor((v - lo) / cell);
  t = fmin(fmax(t, -1.0e9), 1.0e9);
  return static_cast<int>(t);
}

}  // namespace gps
