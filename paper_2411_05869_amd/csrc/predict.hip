// Kriging mean at test points (Sec. 3.2): m(x*) = sum_q C_y(x*, x_q) alpha_q.
//
// The cross-covariance is evaluated and applied in one pass (never stored):
//   local part: each test point searches the training cells within R rings of
//     its cell and adds s0 f0(u) alpha_q for every q with u0^2 < 1;
//   bump part: sum_q [M_i(x*) M_i(q)] f_i(x*) f_i(q) alpha_q
//            = sum_{i in M(x*)} f_i(x*) c_i,   c_i = sum_q f_i(x_q) alpha_q,
//     the rank-n1 structure of the bump term (Proposition 1's proof), with
//     c_i computed once per (theta, alpha) when the predictor is created.
// With a core kernel (Eq. sparseCov) both parts are multiplied by
// C_core(x*, x_q) inside the sums.  The bump part then no longer factors
// through c_i: a wave per test point with a group bit sums
//   sum_q C_core(x*, x_q) sum_{i in M(x*) & M(q)} f_i(x*) f_i(x_q) alpha_q
// over the masked training points (their data copied when the predictor is
// created).
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
  // core kernel: basis of the nonstationary fields, the fields of the training
  // points (binned order), and the masked training points' data
  gps::CoreBasis cb{};
  double* sig = nullptr;      // n (nonstationary core)
  double* Sig = nullptr;      // n
  int64_t nm = 0;
  int32_t* mlist = nullptr;   // nm binned ids of the masked training points
  uint64_t* mmask = nullptr;  // nm group masks
  double* mF = nullptr;       // nm x n1 values f_i
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
  // core kernel: masked training points
  int64_t nm;
  const int32_t* mlist;
  const uint64_t* mmask;
  const double* mF;
};

// The mean at one test point xp (local part over the cell window, plus the
// bump groups through c_i when there is no core kernel).
template <int D, bool MIXED, int CK>
__device__ __forceinline__ double predict_point(const PredArgs& a, const CoreBasis& cb, const double* xp) {
  int c[3] = {0, 0, 0};
  for (int k = 0; k < D; ++k) c[k] = cell_coord(xp[k], a.lo[k], a.cell[k]);
  double sp = 0.0, Sp = 0.0;
  if constexpr (CK == 2) core_point_fields<D>(cb, xp, &sp, &Sp);
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
            double v = a.kt.s0 * wendland(u2, a.kt.variant);
            if constexpr (CK == 1) v = core_value<D, 1>(a.kt.core, xp, xq, 0.0, 0.0, 0.0, 0.0) * v;
            if constexpr (CK == 2)
              v = core_value<D, 2>(a.kt.core, xp, xq, sp, Sp, a.kt.core.sig[q], a.kt.core.Sig[q]) * v;
            if constexpr (MIXED)
              acc += static_cast<double>(static_cast<float>(v) * a.alpha32[q]);
            else
              acc += v * a.alpha[q];
          }
        }
      }
  }
  // bump groups of the test point (with a core kernel: k_predict_groups)
  double gsum = 0.0;
  for (int i = 0; CK == 0 && i < a.kt.n1; ++i) {
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
  return acc + gsum;
}

template <int D, bool MIXED, int CK>
__global__ void __launch_bounds__(kThreads) k_predict(PredArgs a, CoreBasis cb, int64_t m,
                                                      const double* __restrict__ xs, double* __restrict__ out) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (t >= m) return;
  double xp[3];
  for (int k = 0; k < D; ++k) xp[k] = xs[t * D + k];
  out[t] = predict_point<D, MIXED, CK>(a, cb, xp);
}

// Request of row t of a batch: the last r with roff[r] <= t (empty requests
// share their offset with the next one).
__device__ __forceinline__ int batch_request(const int64_t* __restrict__ roff, int nreq, int64_t t) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (roff[mid] <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Batched form: the rows of all requests in one launch, each row with the
// arguments of its request's predictor.
template <int D, bool MIXED, int CK>
__global__ void __launch_bounds__(kThreads) k_predict_batch(const PredArgs* __restrict__ args,
                                                            const CoreBasis* __restrict__ cbs,
                                                            const int32_t* __restrict__ req_pred,
                                                            const int64_t* __restrict__ roff, int nreq, int64_t m,
                                                            const double* __restrict__ xs, double* __restrict__ out) {
  const int64_t t = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (t >= m) return;
  const int pi = req_pred[batch_request(roff, nreq, t)];
  double xp[3];
  for (int k = 0; k < D; ++k) xp[k] = xs[t * D + k];
  out[t] = predict_point<D, MIXED, CK>(args[pi], cbs[pi], xp);
}

// Bump part with a core kernel: one wave per test point.  Lane i < n1 forms
// f_i(x*) (bumps of group i in j order) into LDS; the lanes then stride over
// the masked training points and the wave adds its lanes in a fixed order.
template <int D, int CK>
__device__ __forceinline__ void predict_groups_point(const PredArgs& a, const CoreBasis& cb, int64_t t,
                                                     const double* __restrict__ xs, double* __restrict__ out,
                                                     double* f) {
  const int lane = lane_id();
  double xp[3];
  for (int k = 0; k < D; ++k) xp[k] = xs[t * D + k];
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
  if (mask == 0) return;  // uniform
  f[lane] = fi;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double sp = 0.0, Sp = 0.0;
  if constexpr (CK == 2) core_point_fields<D>(cb, xp, &sp, &Sp);
  double acc = 0.0;
  for (int64_t j = lane; j < a.nm; j += kWave) {
    uint64_t sh = a.mmask[j] & mask;
    if (!sh) continue;
    double bsum = 0.0;
    while (sh) {
      const int i = __builtin_ctzll(sh);
      sh &= sh - 1;
      bsum += f[i] * a.mF[j * a.kt.n1 + i];
    }
    const int32_t q = a.mlist[j];
    double xq[3];
    xq[0] = a.xb[q];
    if constexpr (D >= 2) xq[1] = a.xb[a.n + q];
    if constexpr (D >= 3) xq[2] = a.xb[2 * a.n + q];
    double cv;
    if constexpr (CK == 1)
      cv = core_value<D, 1>(a.kt.core, xp, xq, 0.0, 0.0, 0.0, 0.0);
    else
      cv = core_value<D, 2>(a.kt.core, xp, xq, sp, Sp, a.kt.core.sig[q], a.kt.core.Sig[q]);
    acc += cv * bsum * a.alpha[q];
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
  if (lane == 0) out[t] += acc;
}

template <int D, int CK>
__global__ void __launch_bounds__(kThreads) k_predict_groups(PredArgs a, CoreBasis cb, int64_t m,
                                                             const double* __restrict__ xs, double* __restrict__ out) {
  __shared__ double fs[kThreads / kWave][kWave];
  const int64_t t = (blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x) / kWave;
  if (t >= m) return;  // uniform per wave
  predict_groups_point<D, CK>(a, cb, t, xs, out, fs[threadIdx.x / kWave]);
}

template <int D, int CK>
__global__ void __launch_bounds__(kThreads) k_predict_groups_batch(const PredArgs* __restrict__ args,
                                                                   const CoreBasis* __restrict__ cbs,
                                                                   const int32_t* __restrict__ req_pred,
                                                                   const int64_t* __restrict__ roff, int nreq,
                                                                   int64_t m, const double* __restrict__ xs,
                                                                   double* __restrict__ out) {
  __shared__ double fs[kThreads / kWave][kWave];
  const int64_t t = (blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x) / kWave;
  if (t >= m) return;  // uniform per wave
  const int pi = req_pred[batch_request(roff, nreq, t)];
  if (args[pi].nm == 0) return;  // no masked training points: no group part (uniform per wave)
  predict_groups_point<D, CK>(args[pi], cbs[pi], t, xs, out, fs[threadIdx.x / kWave]);
}

}  // namespace

void destroy_predictor(gp_ctx* c, gp_predictor* p);

gp_predictor* make_predictor(gp_ctx* c, const gp_dataset* ds, const gp_theta* th, const double* alpha) {
  // a failure part-way releases whatever device memory the predictor holds by then
  auto release = [c](gp_predictor* x) { destroy_predictor(c, x); };
  std::unique_ptr<gp_predictor, decltype(release)> p(new gp_predictor(), release);
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
  KernelCore kc;
  core_params(th, &kc, &p->cb);
  if (kc.kind == GP_CORE_PACIOREK) {
    p->sig = dev_new<double>(c, n);
    p->Sig = dev_new<double>(c, n);
    core_fields(c, ds, p->cb, p->sig, p->Sig);
    kc.sig = p->sig;
    kc.Sig = p->Sig;
  }
  p->kt.core = kc;
  if (th->n1 > 0) {
    Features f;
    compute_features(c, ds, kt, &f, 60);
    hipLaunchKernelGGL(k_group_coef, dim3(th->n1), dim3(kThreads), 0, c->stream, f.nm, th->n1, f.F, f.mlist,
                       p->alpha_b, p->coef);
    check_launch("group coefficients");
    if (kc.kind != GP_CORE_NONE && f.nm > 0) {
      // the feature arrays live in workspace slots: keep copies
      p->nm = f.nm;
      p->mlist = dev_new<int32_t>(c, f.nm);
      p->mmask = dev_new<uint64_t>(c, f.nm);
      p->mF = dev_new<double>(c, f.nm * th->n1);
      GPS_HIP(hipMemcpyAsync(p->mlist, f.mlist, sizeof(int32_t) * f.nm, hipMemcpyDeviceToDevice, c->stream));
      GPS_HIP(hipMemcpyAsync(p->mmask, f.mmask, sizeof(uint64_t) * f.nm, hipMemcpyDeviceToDevice, c->stream));
      GPS_HIP(hipMemcpyAsync(p->mF, f.F, sizeof(double) * f.nm * th->n1, hipMemcpyDeviceToDevice, c->stream));
    }
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
  if (p->sig) dev_free(c, p->sig, sizeof(double) * n);
  if (p->Sig) dev_free(c, p->Sig, sizeof(double) * n);
  if (p->mlist) dev_free(c, p->mlist, sizeof(int32_t) * p->nm);
  if (p->mmask) dev_free(c, p->mmask, sizeof(uint64_t) * p->nm);
  if (p->mF) dev_free(c, p->mF, sizeof(double) * p->nm * p->kt.n1);
  delete p;
}

static PredArgs pred_args(const gp_predictor* p) {
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
  a.nm = p->nm;
  a.mlist = p->mlist;
  a.mmask = p->mmask;
  a.mF = p->mF;
  return a;
}

void predict(gp_ctx* c, const gp_predictor* p, int64_t m, const double* xs, int prec, double* out) {
  if (m == 0) return;
  const gp_dataset* ds = p->ds;
  const PredArgs a = pred_args(p);
  const dim3 G(grid_for(m, kThreads)), B(kThreads);
  ProfScope ps(c, prec == GP_MIXED ? "predict_f32" : "predict_f64");
  auto go = [&](auto DD) {
    constexpr int D = decltype(DD)::value;
    auto with_core = [&](auto CC) {
      constexpr int CK = decltype(CC)::value;
      if (prec == GP_MIXED)
        hipLaunchKernelGGL((k_predict<D, true, CK>), G, B, 0, c->stream, a, p->cb, m, xs, out);
      else
        hipLaunchKernelGGL((k_predict<D, false, CK>), G, B, 0, c->stream, a, p->cb, m, xs, out);
      if constexpr (CK != 0) {
        if (p->nm > 0)
          hipLaunchKernelGGL((k_predict_groups<D, CK>), dim3(grid_for(m * kWave, kThreads)), B, 0, c->stream, a,
                             p->cb, m, xs, out);
      }
    };
    if (p->kt.core.kind == GP_CORE_MATERN)
      with_core(std::integral_constant<int, 1>{});
    else if (p->kt.core.kind == GP_CORE_PACIOREK)
      with_core(std::integral_constant<int, 2>{});
    else
      with_core(std::integral_constant<int, 0>{});
  };
  if (ds->d == 1)
    go(std::integral_constant<int, 1>{});
  else if (ds->d == 2)
    go(std::integral_constant<int, 2>{});
  else
    go(std::integral_constant<int, 3>{});
  check_launch("predict");
}

void predict_batch(gp_ctx* c, int32_t nreq, const gp_predictor* const* preds, const int64_t* roff_host,
                   const double* xs, int prec, double* out) {
  for (int32_t r = 0; r < nreq; ++r) {
    GPS_REQUIRE(preds[r]->ds->d == preds[0]->ds->d, GP_EINVAL,
                "gp_predict_batch: all predictors must have the same dimension");
    GPS_REQUIRE(preds[r]->kt.core.kind == preds[0]->kt.core.kind, GP_EINVAL,
                "gp_predict_batch: all predictors must have the same core kernel kind");
  }
  const int64_t m = roff_host[nreq];
  if (m == 0) return;
  // distinct predictors, in order of first appearance
  std::vector<const gp_predictor*> uniq;
  std::vector<int32_t> req_pred(nreq);
  for (int32_t r = 0; r < nreq; ++r) {
    int32_t k = 0;
    while (k < static_cast<int32_t>(uniq.size()) && uniq[k] != preds[r]) ++k;
    if (k == static_cast<int32_t>(uniq.size())) uniq.push_back(preds[r]);
    req_pred[r] = k;
  }
  const int d = uniq[0]->ds->d;
  const int ck = uniq[0]->kt.core.kind;
  bool any_nm = false;
  for (const gp_predictor* p : uniq) any_nm = any_nm || p->nm > 0;
  const size_t np = uniq.size();
  const size_t b_args = sizeof(PredArgs) * np, b_cb = sizeof(CoreBasis) * np;
  const size_t b_req = sizeof(int32_t) * nreq, b_off = sizeof(int64_t) * (nreq + 1);
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t total = up(b_args) + up(b_cb) + up(b_req) + up(b_off);
  char* dbuf = static_cast<char*>(workspace(c, 123, total));
  char* hbuf = static_cast<char*>(pinned_for_write(c, total));
  PredArgs* ha = reinterpret_cast<PredArgs*>(hbuf);
  CoreBasis* hc = reinterpret_cast<CoreBasis*>(hbuf + up(b_args));
  for (size_t k = 0; k < np; ++k) {
    ha[k] = pred_args(uniq[k]);
    hc[k] = uniq[k]->cb;
  }
  std::memcpy(hbuf + up(b_args) + up(b_cb), req_pred.data(), b_req);
  std::memcpy(hbuf + up(b_args) + up(b_cb) + up(b_req), roff_host, b_off);
  h2d_async(c, dbuf, hbuf, total);
  const PredArgs* da = reinterpret_cast<const PredArgs*>(dbuf);
  const CoreBasis* dc = reinterpret_cast<const CoreBasis*>(dbuf + up(b_args));
  const int32_t* dreq = reinterpret_cast<const int32_t*>(dbuf + up(b_args) + up(b_cb));
  const int64_t* droff = reinterpret_cast<const int64_t*>(dbuf + up(b_args) + up(b_cb) + up(b_req));
  const dim3 G(grid_for(m, kThreads)), B(kThreads);
  ProfScope ps(c, prec == GP_MIXED ? "predict_batch_f32" : "predict_batch_f64");
  auto go = [&](auto DD) {
    constexpr int D = decltype(DD)::value;
    auto with_core = [&](auto CC) {
      constexpr int CK = decltype(CC)::value;
      if (prec == GP_MIXED)
        hipLaunchKernelGGL((k_predict_batch<D, true, CK>), G, B, 0, c->stream, da, dc, dreq, droff, nreq, m, xs, out);
      else
        hipLaunchKernelGGL((k_predict_batch<D, false, CK>), G, B, 0, c->stream, da, dc, dreq, droff, nreq, m, xs,
                           out);
      if constexpr (CK != 0) {
        if (any_nm)
          hipLaunchKernelGGL((k_predict_groups_batch<D, CK>), dim3(grid_for(m * kWave, kThreads)), B, 0, c->stream,
                             da, dc, dreq, droff, nreq, m, xs, out);
      }
    };
    if (ck == GP_CORE_MATERN)
      with_core(std::integral_constant<int, 1>{});
    else if (ck == GP_CORE_PACIOREK)
      with_core(std::integral_constant<int, 2>{});
    else
      with_core(std::integral_constant<int, 0>{});
  };
  if (d == 1)
    go(std::integral_constant<int, 1>{});
  else if (d == 2)
    go(std::integral_constant<int, 2>{});
  else
    go(std::integral_constant<int, 3>{});
  check_launch("predict batch");
}

}  // namespace gps
