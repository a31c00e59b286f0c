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

// Entry K_pq (Eq. C_sparse + Eq. Zcov): s0 f0 [local] + sum over shared groups
// in increasing i of f_i(p) f_i(q) + sigma^2 [p = q].  f_i(p) = Fp[i * sp],
// f_i(q) = Fq[i * sq].
__device__ __forceinline__ double entry_value(const KernelTheta& kt, double u2, uint64_t shared,
                                              const double* Fp, const double* Fq, bool diag, int64_t sp = 1,
                                              int64_t sq = 1) {
#pragma clang fp contract(off)
  double acc = (u2 < 1.0) ? kt.s0 * wendland(u2, kt.variant) : 0.0;
  while (shared) {
    const int i = __builtin_ctzll(shared);
    shared &= shared - 1;
    acc = acc + Fp[i * sp] * Fq[i * sq];
  }
  if (diag) acc = acc + kt.nugget;
  return acc;
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
