// y = K x without any device allocation, for callers that cannot allocate
// (code under stream capture, tight serving loops).  The two n-vectors that
// gp_matvec stages in binned order live in a fixed array of device memory
// owned by the library; the product itself is the one-column product of
// gp_matvec, reading only the caches the matrix already holds.
#include <mutex>

#include "internal.hpp"

namespace gps {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  In host code this name is
// not a device address: the per-device address comes from
// hipGetSymbolAddress below and is the only one passed to kernels.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Looks up this device's copy of the array once (the device must be current).
void noalloc_init(int device) {
  GPS_REQUIRE(device >= 0 && device < kMaxDevices, GP_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return;
  void* p = nullptr;
  GPS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  GPS_REQUIRE(p != nullptr, GP_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch[device] = p;
}

void matvec_noalloc(gp_ctx* c, const gp_matrix* m, const double* x, double* y) {
  const int64_t n = m->n;
  GPS_REQUIRE(static_cast<size_t>(n) * 2 * sizeof(double) <= kScratchBytes, GP_EINVAL,
              "gp_matvec_noalloc: n = " + std::to_string(n) + " exceeds the " + std::to_string(kScratchBytes >> 20) +
                  " MiB scratch (at most " + std::to_string(kScratchBytes / (2 * sizeof(double))) + " points)");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    base = g_scratch[c->device];
  }
  GPS_REQUIRE(base != nullptr, GP_EDEVICE, "gp_matvec_noalloc: scratch address not set up for this device");
  double* xb = static_cast<double*>(base);
  double* yb = xb + n;
  // every entry of xb and yb is written before it is read, so nothing from an
  // earlier call needs clearing
  permute_to_binned<double>(c, m->ds, 1, x, xb);
  spmv_f64_enqueue(c, m, xb, yb);
  permute_to_orig<double>(c, m->ds, 1, yb, y);
}

}  // namespace gps
