// Spatial-hash binning of a dataset (once per dataset; theta-independent).
//
// Points are sorted by the key of their cell on a regular grid with cell edge
// c_k per coordinate (key = (cz * gy + cy) * gx + cx, x fastest), ties kept in
// original index order.  Cells only bound the candidate search of the
// assembly: every membership decision is made on the raw coordinates.
#include <algorithm>
#include <cmath>

#include "device.hpp"

namespace gps {
namespace {

constexpr int kThreads = 256;

__global__ void k_bbox_partial(const double* __restrict__ x, int64_t n, int d, double* __restrict__ part) {
  // part[blockIdx.x * 6 + k] = min_k, part[... + 3 + k] = max_k
  __shared__ double smin[3][kThreads];
  __shared__ double smax[3][kThreads];
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    for (int k = 0; k < d; ++k) {
      const double v = x[i * d + k];
      if (!isfinite(v)) bad = true;
      mn[k] = fmin(mn[k], v);
      mx[k] = fmax(mx[k], v);
    }
  }
  for (int k = 0; k < 3; ++k) {
    smin[k][threadIdx.x] = bad ? NAN : mn[k];
    smax[k][threadIdx.x] = bad ? NAN : mx[k];
  }
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      for (int k = 0; k < 3; ++k) {
        const double a = smin[k][threadIdx.x], b = smin[k][threadIdx.x + s];
        smin[k][threadIdx.x] = (isnan(a) || isnan(b)) ? NAN : fmin(a, b);
        const double c = smax[k][threadIdx.x], e = smax[k][threadIdx.x + s];
        smax[k][threadIdx.x] = (isnan(c) || isnan(e)) ? NAN : fmax(c, e);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) {
      part[blockIdx.x * 6 + k] = smin[k][0];
      part[blockIdx.x * 6 + 3 + k] = smax[k][0];
    }
}

struct BinGrid {
  double lo[3];
  double cell[3];
  int32_t g[3];
};

__global__ void k_keys_hist(const double* __restrict__ x, int64_t n, int d, BinGrid bg,
                            int32_t* __restrict__ key_orig, int32_t* __restrict__ count) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i >= n) return;
  int c[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) {
    int v = cell_coord(x[i * d + k], bg.lo[k], bg.cell[k]);
    v = v < 0 ? 0 : (v >= bg.g[k] ? bg.g[k] - 1 : v);
    c[k] = v;
  }
  const int32_t key = (c[2] * bg.g[1] + c[1]) * bg.g[0] + c[0];
  key_orig[i] = key;
  atomicAdd(&count[key], 1);
}

__global__ void k_scatter(const int32_t* __restrict__ key_orig, int64_t n, const int32_t* __restrict__ cell_start,
                          int32_t* __restrict__ cursor, int32_t* __restrict__ perm) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i >= n) return;
  const int32_t k = key_orig[i];
  const int32_t slot = cell_start[k] + atomicAdd(&cursor[k], 1);
  perm[slot] = static_cast<int32_t>(i);
}

// One wave per cell: order the cell's original indices ascending by rank
// (rank = number of smaller indices; indices are unique, so ranks are a
// permutation).  Deterministic whatever order the scatter produced.
__global__ void k_sort_cells(const int32_t* __restrict__ cell_start, int64_t ncells, int32_t* __restrict__ perm,
                             int32_t* __restrict__ tmp) {
  const int64_t cell = (blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x) / kWave;
  if (cell >= ncells) return;
  const int lane = lane_id();
  const int32_t s = cell_start[cell], e = cell_start[cell + 1];
  const int32_t len = e - s;
  if (len < 2) return;
  // tmp holds a copy of perm made by an earlier operation on the stream
  for (int32_t a = lane; a < len; a += kWave) {
    const int32_t v = tmp[s + a];
    int32_t rank = 0;
    for (int32_t b = 0; b < len; ++b) rank += tmp[s + b] < v ? 1 : 0;
    perm[s + rank] = v;
  }
}

__global__ void k_gather(const double* __restrict__ x, int64_t n, int d, const int32_t* __restrict__ perm,
                         const int32_t* __restrict__ key_orig, double* __restrict__ xb, int32_t* __restrict__ iperm,
                         int32_t* __restrict__ key) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i >= n) return;
  const int32_t o = perm[i];
  for (int k = 0; k < d; ++k) xb[k * n + i] = x[static_cast<int64_t>(o) * d + k];
  iperm[o] = static_cast<int32_t>(i);
  key[i] = key_orig[o];
}

__global__ void k_max_count(const int32_t* __restrict__ count, int64_t ncells, int32_t* __restrict__ out) {
  int32_t m = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < ncells;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    m = max(m, count[i]);
  for (int off = kWave / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, kWave));
  if (lane_id() == 0) atomicMax(out, m);
}

}  // namespace

void bin_dataset(gp_ctx* c, gp_dataset* ds, const double* x_dev, const double* cell) {
  const int64_t n = ds->n;
  const int d = ds->d;
  // bounding box
  const unsigned nb = std::min<int64_t>(grid_for(n, kThreads), 1024);
  TmpBuf part(c, sizeof(double) * 6 * nb);
  hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kThreads), 0, c->stream, x_dev, n, d, part.as<double>());
  check_launch("bbox");
  std::vector<double> hp(6 * nb);
  GPS_HIP(hipMemcpyAsync(hp.data(), part.p, sizeof(double) * 6 * nb, hipMemcpyDeviceToHost, c->stream));
  sync(c);
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) {
    lo[k] = INFINITY;
    hi[k] = -INFINITY;
    for (unsigned b = 0; b < nb; ++b) {
      const double a = hp[b * 6 + k], e = hp[b * 6 + 3 + k];
      GPS_REQUIRE(std::isfinite(a) && std::isfinite(e), GP_EINVAL, "gp_dataset_create: non-finite coordinate");
      lo[k] = std::min(lo[k], a);
      hi[k] = std::max(hi[k], e);
    }
  }
  // cell edges: caller's, or about eight points per cell over the bounding box
  double cs[3] = {1, 1, 1};
  for (int k = 0; k < d; ++k) {
    if (cell) {
      GPS_REQUIRE(std::isfinite(cell[k]) && cell[k] > 0, GP_EINVAL, "gp_dataset_create: cell must be > 0");
      cs[k] = cell[k];
    } else {
      double vol = 1.0;
      int nz = 0;
      for (int j = 0; j < d; ++j)
        if (hi[j] > lo[j]) {
          vol *= hi[j] - lo[j];
          ++nz;
        }
      const double per = nz ? std::pow(vol * 8.0 / static_cast<double>(n), 1.0 / nz) : 1.0;
      cs[k] = hi[k] > lo[k] ? per : 1.0;
    }
  }
  // keep the grid modest: at most max(4n, 1024) cells, at most 2^30
  for (int iter = 0; iter < 64; ++iter) {
    double total = 1.0;
    for (int k = 0; k < d; ++k) total *= std::floor((hi[k] - lo[k]) / cs[k]) + 2.0;
    const double cap = std::min<double>(std::max<double>(4.0 * n, 1024.0), 1073741824.0);
    if (total <= cap) break;
    const double f = std::pow(total / cap, 1.0 / d) * 1.0001;
    for (int k = 0; k < d; ++k) cs[k] *= f;
  }
  BinGrid bg{};
  int64_t ncells = 1;
  for (int k = 0; k < 3; ++k) {
    bg.lo[k] = k < d ? lo[k] : 0.0;
    bg.cell[k] = k < d ? cs[k] : 1.0;
    // one slack cell above the box: a rounded cell index of a point never needs clamping
    bg.g[k] = k < d ? static_cast<int32_t>(std::floor((hi[k] - lo[k]) / cs[k]) + 2.0) : 1;
    ncells *= bg.g[k];
    ds->lo[k] = bg.lo[k];
    ds->cell[k] = bg.cell[k];
    ds->g[k] = bg.g[k];
  }
  ds->ncells = ncells;

  ds->xb = dev_new<double>(c, static_cast<size_t>(d) * n);
  ds->perm = dev_new<int32_t>(c, n);
  ds->iperm = dev_new<int32_t>(c, n);
  ds->key = dev_new<int32_t>(c, n);
  ds->cell_start = dev_new<int32_t>(c, ncells + 1);
  ds->bytes = sizeof(double) * d * n + 3 * sizeof(int32_t) * n + sizeof(int32_t) * (ncells + 1);

  TmpBuf key_orig(c, sizeof(int32_t) * n);
  TmpBuf count(c, sizeof(int32_t) * ncells);
  TmpBuf tmp(c, sizeof(int32_t) * n);
  TmpBuf mx(c, sizeof(int32_t));
  GPS_HIP(hipMemsetAsync(count.p, 0, sizeof(int32_t) * ncells, c->stream));
  GPS_HIP(hipMemsetAsync(mx.p, 0, sizeof(int32_t), c->stream));
  hipLaunchKernelGGL(k_keys_hist, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, x_dev, n, d, bg,
                     key_orig.as<int32_t>(), count.as<int32_t>());
  check_launch("keys");
  scan_i32_to_i32(c, count.as<int32_t>(), ds->cell_start, ncells);
  hipLaunchKernelGGL(k_max_count, dim3(std::min<int64_t>(grid_for(ncells, kThreads), 1024)), dim3(kThreads), 0,
                     c->stream, count.as<int32_t>(), ncells, mx.as<int32_t>());
  check_launch("max count");
  GPS_HIP(hipMemsetAsync(count.p, 0, sizeof(int32_t) * ncells, c->stream));
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, key_orig.as<int32_t>(),
                     n, ds->cell_start, count.as<int32_t>(), ds->perm);
  check_launch("scatter");
  GPS_HIP(hipMemcpyAsync(tmp.p, ds->perm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c->stream));
  hipLaunchKernelGGL(k_sort_cells, dim3(grid_for(ncells * kWave, kThreads)), dim3(kThreads), 0, c->stream,
                     ds->cell_start, ncells, ds->perm, tmp.as<int32_t>());
  check_launch("sort cells");
  hipLaunchKernelGGL(k_gather, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, x_dev, n, d, ds->perm,
                     key_orig.as<int32_t>(), ds->xb, ds->iperm, ds->key);
  check_launch("gather");
  int32_t* h = static_cast<int32_t*>(pinned(c, sizeof(int32_t)));
  GPS_HIP(hipMemcpyAsync(h, mx.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  ds->max_cell = *h;
}

}  // namespace gps
