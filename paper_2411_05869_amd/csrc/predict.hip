// Kriging mean at test points (Sec. 3.2): m(x*) = sum_q C_y(x*, x_q) alpha_q.
//
// The cross-covariance is evaluated and applied in one pass (never stored):
//   local part: each test point searches the training cells within R rings of
//     its cell and adds s0 f0(u) alpha_q for every q with u0^2 < 1;
//   bump part: sum_q [M_i(x*) M_i(q)] f_i(x*) f_i(q) alpha_q
//            = sum_{i in M(x*)} f_i(x*) c_i,   c_i = sum_q f_i(x_q) alpha_q,
//     the rank-n1 structure of the bump term (Proposition 1's proof), with
//     c_i computed once per (theta, alpha) when the predictor is created.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "device.hpp"

struct gp_predictor {
  const gp_dataset* ds = nullptr;
  gps::Bump* bumps = nullptr;
  int nbumps = 0;
  gps::KernelTheta kt{};
  gps::Grid grid{};
  double* alpha_b = nullptr;  // n, binned order
  double* coef = nullptr;     // n1 (at least 1)
  float* alpha32 = nullptr;   // n, float32 copy for the mixed form
};

namespace gps {
namespace {

constexpr int kThreads = 256;

// c_i = sum over masked points k of F[k, i] * alpha[mlist[k]]; one block per group.
__global__ void __launch_bounds__(kThreads) k_group_coef(int64_t nm, int n1, const double* __restrict__ F,
                                                         const int32_t* __restrict__ mlist,
                                                         const double* __restrict__ alpha, double* __restrict__ coef) {
  const int i = blockIdx.x;
  double s = 0;
  for (int64_t k = threadIdx.x; k < nm; k += kThreads) s += F[k * n1 + i] * alpha[mlist[k]];
  __shared__ double sh[kThreads];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) coef[i] = sh[0];
}

__global__ void k_to_f32(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i < n) b[i] = static_cast<float>(a[i]);
}

struct PredArgs {
  KernelTheta kt;
  int64_t n;
  const double* xb;
  const int32_t* cell_start;
  double lo[3], cell[3];
  int32_t g[3], R[3];
  const double* alpha;
  const float* alpha32;
  const double* coef;
};

template <int D, bool MIXED>
__global__ void __launch_bounds__(kThreads) k_predict(PredArgs a, int64_t m, const double* __restrict__ xs,
                                                      double* __restrict__ out) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (t >= m) return;
  double xp[3];
  int c[3] = {0, 0, 0};
  for (int k = 0; k < D; ++k) {
    xp[k] = xs[t * D + k];
    c[k] = cell_coord(xp[k], a.lo[k], a.cell[k]);
  }
  int lo_[3] = {0, 0, 0}, hi_[3] = {0, 0, 0};
  bool empty = false;
  for (int k = 0; k < D; ++k) {
    lo_[k] = max(c[k] - a.R[k], 0);
    hi_[k] = min(c[k] + a.R[k], a.g[k] - 1);
    if (lo_[k] > hi_[k]) empty = true;
  }
  double acc = 0.0;
  if (!empty) {
    for (int z = lo_[2]; z <= hi_[2]; ++z)
      for (int y = lo_[1]; y <= hi_[1]; ++y) {
        const int64_t base = (static_cast<int64_t>(z) * a.g[1] + y) * a.g[0];
        const int32_t s = a.cell_start[base + lo_[0]];
        const int32_t e = a.cell_start[base + hi_[0] + 1];
        for (int32_t q = s; q < e; ++q) {
          double xq[3];
          xq[0] = a.xb[q];
          if constexpr (D >= 2) xq[1] = a.xb[a.n + q];
          if constexpr (D >= 3) xq[2] = a.xb[2 * a.n + q];
          const double u2 = scaled_sq<D>(xp, xq, a.kt.inv0);
          if (u2 < 1.0) {
            const double v = a.kt.s0 * wendland(u2, a.kt.variant);
            if constexpr (MIXED)
              acc += static_cast<double>(static_cast<float>(v) * a.alpha32[q]);
            else
              acc += v * a.alpha[q];
          }
        }
      }
  }
  // bump groups of the test point
  double gsum = 0.0;
  for (int i = 0; i < a.kt.n1; ++i) {
    double f = 0.0;
    bool in_group = false;
    for (int j = 0; j < a.kt.n2; ++j) {
      const Bump& bp = a.kt.bumps[i * a.kt.n2 + j];
      const double ub2 = scaled_sq<D>(xp, bp.h, bp.inv);
      if (bp.a > 0.0 && ub2 < 1.0) {
        in_group = true;
        f = f + bp.a * exp(bp.b * (1.0 - 1.0 / (1.0 - ub2)));
      }
    }
    if (in_group) gsum += f * a.coef[i];
  }
  out[t] = acc + gsum;
}

}  // namespace

gp_predictor* make_predictor(gp_ctx* c, const gp_dataset* ds, const gp_theta* th, const double* alpha) {
  std::unique_ptr<gp_predictor> p(new gp_predictor());
  p->ds = ds;
  Bump* tmp_bumps = nullptr;
  KernelTheta kt{};
  upload_theta(c, th, &tmp_bumps, &kt);
  const int nb = std::max(th->n1 * th->n2, 1);
  p->nbumps = nb;
  p->bumps = dev_new<Bump>(c, nb);
  GPS_HIP(hipMemcpyAsync(p->bumps, tmp_bumps, sizeof(Bump) * nb, hipMemcpyDeviceToDevice, c->stream));
  kt.bumps = p->bumps;
  p->kt = kt;
  p->grid = make_grid(ds, th);
  const int64_t n = ds->n;
  p->alpha_b = dev_new<double>(c, n);
  p->alpha32 = dev_new<float>(c, n);
  p->coef = dev_new<double>(c, std::max(th->n1, 1));
  permute_to_binned<double>(c, ds, 1, alpha, p->alpha_b);
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, n, p->alpha_b, p->alpha32);
  check_launch("alpha f32");
  if (th->n1 > 0) {
    Features f;
    compute_features(c, ds, kt, &f, 60);
    hipLaunchKernelGGL(k_group_coef, dim3(th->n1), dim3(kThreads), 0, c->stream, f.nm, th->n1, f.F, f.mlist,
                       p->alpha_b, p->coef);
    check_launch("group coefficients");
  }
  sync(c);
  return p.release();
}

void destroy_predictor(gp_ctx* c, gp_predictor* p) {
  if (!p) return;
  const int64_t n = p->ds->n;
  dev_free(c, p->bumps, sizeof(Bump) * p->nbumps);
  dev_free(c, p->alpha_b, sizeof(double) * n);
  dev_free(c, p->alpha32, sizeof(float) * n);
  dev_free(c, p->coef, sizeof(double) * std::max(p->kt.n1, 1));
  delete p;
}

void predict(gp_ctx* c, const gp_predictor* p, int64_t m, const double* xs, int prec, double* out) {
  if (m == 0) return;
  const gp_dataset* ds = p->ds;
  PredArgs a{};
  a.kt = p->kt;
  a.n = ds->n;
  a.xb = ds->xb;
  a.cell_start = ds->cell_start;
  for (int k = 0; k < 3; ++k) {
    a.lo[k] = ds->lo[k];
    a.cell[k] = ds->cell[k];
    a.g[k] = ds->g[k];
    a.R[k] = p->grid.R[k];
  }
  a.alpha = p->alpha_b;
  a.alpha32 = p->alpha32;
  a.coef = p->coef;
  const dim3 G(grid_for(m, kThreads)), B(kThreads);
  ProfScope ps(c, prec == GP_MIXED ? "predict_f32" : "predict_f64");
  auto go = [&](auto DD) {
    constexpr int D = decltype(DD)::value;
    if (prec == GP_MIXED)
      hipLaunchKernelGGL((k_predict<D, true>), G, B, 0, c->stream, a, m, xs, out);
    else
      hipLaunchKernelGGL((k_predict<D, false>), G, B, 0, c->stream, a, m, xs, out);
  };
  if (ds->d == 1)
    go(std::integral_constant<int, 1>{});
  else if (ds->d == 2)
    go(std::integral_constant<int, 2>{});
  else
    go(std::integral_constant<int, 3>{});
  check_launch("predict");
}

}  // namespace gps
