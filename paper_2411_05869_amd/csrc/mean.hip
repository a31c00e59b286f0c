// Residual of the prior mean (Sec. 3.1, Eq. Zmarg: z ~ N(W beta, C_z)):
// y = z - W beta for an n x p covariate matrix W stored column by column, so
// that a thread per row reads each column coalesced across the wave.
#include "device.hpp"

namespace gps {
namespace {

constexpr int kThreads = 256;
constexpr int kBetaChunk = 1024;  // coefficients staged in LDS at a time

__global__ void __launch_bounds__(kThreads) k_residual(int64_t n, int p, const double* __restrict__ W,
                                                       const double* __restrict__ beta, const double* __restrict__ z,
                                                       double* __restrict__ y) {
  __shared__ double bs[kBetaChunk];
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  double acc = 0.0;
  for (int k0 = 0; k0 < p; k0 += kBetaChunk) {
    const int kn = min(kBetaChunk, p - k0);
    __syncthreads();
    for (int k = threadIdx.x; k < kn; k += kThreads) bs[k] = beta[k0 + k];
    __syncthreads();
    if (i < n)
      for (int k = 0; k < kn; ++k) acc += W[static_cast<int64_t>(k0 + k) * n + i] * bs[k];
  }
  if (i < n) y[i] = z[i] - acc;
}

}  // namespace

void mean_residual(gp_ctx* c, int64_t n, int p, const double* W, const double* beta_host, const double* z,
                   double* y) {
  double* bd = nullptr;
  if (p > 0) {
    bd = static_cast<double*>(workspace(c, 120, sizeof(double) * p));
    double* st = static_cast<double*>(pinned_for_write(c, sizeof(double) * p));
    for (int k = 0; k < p; ++k) st[k] = beta_host[k];
    h2d_async(c, bd, st, sizeof(double) * p);
  }
  hipLaunchKernelGGL(k_residual, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, n, p, W, bd, z, y);
  check_launch("mean residual");
}

}  // namespace gps
