// Assembly of K(theta) + sigma^2 I as CSR (binned order, ascending columns).
//
// The pattern is   P = {(p,q): u0^2(p,q) < 1}  U  {(p,q): M(p) & M(q) != 0}
// (local Wendland support of Eq. compSupp, or a shared bump group of
// Eq. C_sparse; the diagonal is in both).  For a fixed theta both supports are
// explicit balls, so the pattern is found without testing all pairs:
//   * local pairs: each row searches the cells within R_k rings of its own
//     cell; cells in key order and points in binned order visit candidate
//     columns in ascending order;
//   * group pairs: rows with a group mask M take every point of
//     U_M = {q : M(q) & M != 0}, a sorted list shared by all rows with mask M.
// A row with group mask M (M = 0 for most rows) holds first the |U_M| group
// entries (ascending), then its local-only entries L'(p) = {q : u0^2 < 1,
// M(q) & M = 0} (ascending; all local entries when M = 0).  The local parts
// are found one row per lane; the group parts are written tile by tile for
// the rows sharing a mask.  Count and fill run the same candidate loops; the
// fill checks that it wrote exactly the counted number of entries.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "device.hpp"

namespace gps {
namespace {

constexpr int kThreads = 256;

struct AsmArgs {
  KernelTheta kt;
  int64_t n;
  const double* xb;
  const int32_t* key;
  const int32_t* cell_start;
  int32_t g[3];
  int32_t R[3];
  const uint64_t* mask;
  const int32_t* midx;
  const int32_t* mlist;
  const double* F;
  int64_t nm;
  // group lists
  const int32_t* did;       // nm: distinct-mask id of each masked row
  const int64_t* uoff;      // nD + 1
  const int32_t* ulist;     // concatenated U_M lists
  int64_t utotal;           // their total length
  const double* ux;         // D x utotal coordinates of the U list entries
  const uint64_t* umask;    // utotal group masks
  const double* uF;         // n1 x utotal values f_i
  // counts / outputs
  int32_t* counts;          // n
  int32_t* gskip;           // n: leading group entries of each row (|U_M| or 0)
  const int64_t* row_ptr;   // n + 1
  int32_t* col;
  void* val;
  double* diag;
  int* err;
};

template <int D>
__device__ __forceinline__ void load_point(const double* xb, int64_t n, int64_t i, double* x) {
  x[0] = xb[i];
  if constexpr (D >= 2) x[1] = xb[n + i];
  if constexpr (D >= 3) x[2] = xb[2 * n + i];
}

// Window bounds of the local search around cell c: for each (z, y) pencil, the
// binned range of cells x0..x1.
struct Window {
  int x0, x1, y0, y1, z0, z1;
};

template <int D>
__device__ __forceinline__ Window make_window(const AsmArgs& a, const int* c) {
  Window w;
  w.x0 = max(c[0] - a.R[0], 0);
  w.x1 = min(c[0] + a.R[0], a.g[0] - 1);
  w.y0 = D >= 2 ? max(c[1] - a.R[1], 0) : 0;
  w.y1 = D >= 2 ? min(c[1] + a.R[1], a.g[1] - 1) : 0;
  w.z0 = D >= 3 ? max(c[2] - a.R[2], 0) : 0;
  w.z1 = D >= 3 ? min(c[2] + a.R[2], a.g[2] - 1) : 0;
  return w;
}

// ---------------------------------------------------------------- features
// Group mask of every point (the support tests of point_features, bump j of
// group i is bump i * n2 + j): the bumps are staged in LDS kThreads at a
// time and every thread tests its point against the staged ones.
template <int D>
__global__ void __launch_bounds__(kThreads) k_mask(KernelTheta kt, int64_t n, const double* __restrict__ xb,
                                                   uint64_t* __restrict__ mask, int32_t* __restrict__ flag) {
  __shared__ double sh[3][kThreads], si[3][kThreads];
  __shared__ int32_t sact[kThreads];
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  double x[3] = {0, 0, 0};
  if (p < n) load_point<D>(xb, n, p, x);
  uint64_t m = 0;
  const int nb = kt.n1 * kt.n2;
  for (int b0 = 0; b0 < nb; b0 += kThreads) {
    __syncthreads();  // the previous chunk has been read
    const int b = b0 + static_cast<int>(threadIdx.x);
    if (b < nb) {
      const Bump& bp = kt.bumps[b];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sh[k][threadIdx.x] = bp.h[k];
        si[k][threadIdx.x] = bp.inv[k];
      }
      sact[threadIdx.x] = bp.a > 0.0 ? 1 : 0;
    }
    __syncthreads();
    const int cnt = min(kThreads, nb - b0);
    int gi = b0 / kt.n2, jj = b0 % kt.n2;
    for (int j = 0; j < cnt; ++j) {
      const double h[3] = {sh[0][j], sh[1][j], sh[2][j]};
      const double inv[3] = {si[0][j], si[1][j], si[2][j]};
      const double ub2 = scaled_sq<D>(x, h, inv);
      if (sact[j] && ub2 < 1.0) m |= 1ull << gi;
      if (++jj == kt.n2) {
        jj = 0;
        ++gi;
      }
    }
  }
  if (p < n) {
    mask[p] = m;
    flag[p] = m != 0 ? 1 : 0;
  }
}

__global__ void __launch_bounds__(kThreads) k_compact_masked(int64_t n, const int32_t* __restrict__ flag,
                                                             const int32_t* __restrict__ pos,
                                                             const uint64_t* __restrict__ mask,
                                                             int32_t* __restrict__ midx, int32_t* __restrict__ mlist,
                                                             uint64_t* __restrict__ mmask) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (p >= n) return;
  if (flag[p]) {
    const int32_t k = pos[p];
    midx[p] = k;
    mlist[k] = static_cast<int32_t>(p);
    mmask[k] = mask[p];
  } else {
    midx[p] = -1;
  }
}

template <int D>
__global__ void __launch_bounds__(kThreads) k_fvals(KernelTheta kt, int64_t n, int64_t nm, const double* __restrict__ xb,
                                                    const int32_t* __restrict__ mlist, double* __restrict__ F) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (k >= nm) return;
  double x[3];
  load_point<D>(xb, n, mlist[k], x);
  point_features<D, true>(kt, x, F + k * kt.n1);
}

// One block per distinct mask M: U_M = masked points q (ascending) with M(q) & M != 0.
constexpr int kUlThreads = 1024;
__global__ void __launch_bounds__(kUlThreads) k_ulists(int64_t nm, const uint64_t* __restrict__ mmask,
                                                       const int32_t* __restrict__ mlist,
                                                       const uint64_t* __restrict__ dmask,
                                                       const int64_t* __restrict__ uoff, int32_t* __restrict__ ulist) {
  __shared__ int32_t wcount[kUlThreads / kWave];
  const uint64_t M = dmask[blockIdx.x];
  int32_t* out = ulist + uoff[blockIdx.x];
  const int w = threadIdx.x / kWave;
  int64_t running = 0;
  for (int64_t b = 0; b < nm; b += kUlThreads) {
    const int64_t k = b + threadIdx.x;
    const bool hit = k < nm && (mmask[k] & M) != 0;
    const uint64_t bal = __ballot(hit);
    if (lane_id() == 0) wcount[w] = __popcll(bal);
    __syncthreads();
    int64_t before = 0, total = 0;
    for (int i = 0; i < kUlThreads / kWave; ++i) {
      if (i < w) before += wcount[i];
      total += wcount[i];
    }
    if (hit) out[running + before + __popcll(bal & lanes_below())] = mlist[k];
    running += total;
    __syncthreads();
  }
}

// Point data of the concatenated U_M lists in list order (coordinates, mask,
// f_i as one array per i), so that rows read their group columns contiguously.
template <int D>
__global__ void __launch_bounds__(kThreads) k_ugather(AsmArgs a, double* __restrict__ ux,
                                                      uint64_t* __restrict__ umask, double* __restrict__ uF) {
  const int64_t j = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (j >= a.utotal) return;
  const int32_t u = a.ulist[j];
#pragma unroll
  for (int k = 0; k < D; ++k) ux[k * a.utotal + j] = a.xb[k * a.n + u];
  umask[j] = a.mask[u];
  const double* f = a.F + static_cast<int64_t>(a.midx[u]) * a.kt.n1;
  for (int i = 0; i < a.kt.n1; ++i) uF[i * a.utotal + j] = f[i];
}

// flags a per-point error variance that is not finite or is negative
__global__ void __launch_bounds__(kThreads) k_check_tau2(int64_t n, const double* __restrict__ t,
                                                         int* __restrict__ err) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (i < n && !(t[i] >= 0.0 && t[i] <= 1.7976931348623157e308)) atomicOr(err, 1);
}

// ------------------------------------------------------------- local entries
// Every row's local entries: for a row without a group bit all pairs with
// u0^2 < 1; for a row with group mask M(p) only the local-only ones L'(p)
// (u0^2 < 1 and M(q) & M(p) = 0), which follow the row's |U_M| group entries
// (written by k_group_tile_fill).  One row per lane.
//
// A row's window is a set of pencils (cell rows along x within R rings),
// each a contiguous range of binned points; visited in key order they give
// the candidate columns in ascending order.  The wave's rows (consecutive in
// binned order, so mostly in neighbouring cells) need, per pencil, one
// contiguous range of points, the union of their own ranges.  When it holds
// at most kStage points the wave stages their coordinates in its LDS slice
// with coalesced loads and every lane scans its own range there; otherwise
// the lanes read the points from global memory.  A row with a group bit reads
// its candidates' masks from global memory (few rows have one).
constexpr int kBuf = 4;
constexpr int kStage = 256;
constexpr int kCu = 2;  // candidates whose global loads are in flight together

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// COUNT (FILL = false): counts[p] = number of local (local-only) entries of
// row p; gskip[p] = 0 for a row without a group bit (set for the others once
// the group lists are known).  FILL: writes them at row_ptr[p] + gskip[p] and
// checks that they are exactly the rest of the row.
template <int D, bool FILL, typename VT, int CK = 0>
__global__ void __launch_bounds__(kThreads) k_local_rows(AsmArgs a) {
  __shared__ double stage[kThreads / kWave][D][kStage];
  // each XCD takes a contiguous range of rows: their candidates and output
  // cache lines stay within its L2
  const int64_t p = xcd_remap(blockIdx.x, gridDim.x) * static_cast<int64_t>(kThreads) + threadIdx.x;
  const int lane = lane_id();
  double (*st)[kStage] = stage[threadIdx.x / kWave];
  const uint64_t mp = p < a.n ? a.mask[p] : 0;
  const int64_t out = (FILL && p < a.n) ? a.row_ptr[p] + (mp ? a.gskip[p] : 0) : 0;
  const int64_t len = (FILL && p < a.n) ? a.row_ptr[p + 1] - out : 0;
  const bool row = p < a.n;
  if (__ballot(row) == 0) return;  // uniform
  double xp[3] = {0, 0, 0};
  Window w{0, -1, 0, 0, 0, 0};
  int cy = 0, cz = 0;
  if (row) {
    load_point<D>(a.xb, a.n, p, xp);
    int c[3];
    decode_key(a.key[p], a.g, c);
    w = make_window<D>(a, c);
    cy = c[1];
    cz = c[2];
  }
  // nonstationary core: fields of the row's point
  double sp = 0.0, Sp = 0.0;
  if constexpr (CK == 2) {
    if (row) {
      sp = a.kt.core.sig[p];
      Sp = a.kt.core.Sig[p];
    }
  }
  int32_t cnt = 0;
  VT* val = static_cast<VT*>(a.val);
  // fill: hits are buffered kBuf at a time and written with vector stores
  int32_t bc[kBuf];
  VT bv[kBuf];
  int nb = 0;
  auto hit_at = [&](int32_t q, double u2, const double* xq) {
    if constexpr (FILL) {
      double cv = 1.0;
      if constexpr (CK == 1) cv = core_value<D, 1>(a.kt.core, xp, xq, 0.0, 0.0, 0.0, 0.0);
      if constexpr (CK == 2) cv = core_value<D, 2>(a.kt.core, xp, xq, sp, Sp, a.kt.core.sig[q], a.kt.core.Sig[q]);
      const double v = entry_value(a.kt, u2, 0, nullptr, nullptr, q == p, 1, 1, cv, p);
      const VT vs = static_cast<VT>(v);
      if (q == p) a.diag[p] = static_cast<double>(vs);
      // shift register (constant indices keep it in registers): newest last
#pragma unroll
      for (int j = 0; j + 1 < kBuf; ++j) {
        bc[j] = bc[j + 1];
        bv[j] = bv[j + 1];
      }
      bc[kBuf - 1] = q;
      bv[kBuf - 1] = vs;
      ++nb;
      if (nb % kBuf == 0 && cnt + 1 <= len) {  // never past the counted row
        __builtin_memcpy(a.col + out + cnt + 1 - kBuf, bc, sizeof(bc));
        __builtin_memcpy(val + out + cnt + 1 - kBuf, bv, sizeof(bv));
      }
    }
    ++cnt;
  };
  // a local candidate of this row: u0^2 < 1, and no group shared with a row that has one
  auto local = [&](int32_t q, double u2) { return u2 < 1.0 && (mp == 0 || (a.mask[q] & mp) == 0); };
  const int Ry = D >= 2 ? a.R[1] : 0, Rz = D >= 3 ? a.R[2] : 0;
  for (int dz = -Rz; dz <= Rz; ++dz)
    for (int dy = -Ry; dy <= Ry; ++dy) {
      // this lane's range in pencil (cy + dy, cz + dz)
      int32_t s = 0, e = 0;
      const int y = cy + dy, z = cz + dz;
      if (row && y >= w.y0 && y <= w.y1 && z >= w.z0 && z <= w.z1) {
        const int64_t base = (static_cast<int64_t>(z) * a.g[1] + y) * a.g[0];
        s = a.cell_start[base + w.x0];
        e = a.cell_start[base + w.x1 + 1];
      }
      int32_t lo = e > s ? s : INT32_MAX, hi = e > s ? e : INT32_MIN;
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off, kWave));
        hi = max(hi, __shfl_xor(hi, off, kWave));
      }
      if (hi <= lo) continue;  // uniform: no candidates for any lane
      if (hi - lo <= kStage) {
        wave_sync_lds();  // the previous pencil's reads are done
        for (int32_t j = lane; j < hi - lo; j += kWave) {
          double xq[3];
          load_point<D>(a.xb, a.n, lo + j, xq);
#pragma unroll
          for (int k = 0; k < D; ++k) st[k][j] = xq[k];
        }
        wave_sync_lds();
        // two candidates per step (independent chains); an odd last one alone
        int32_t q = s;
        for (; q + 1 < e; q += 2) {
          double xa[3], xb2[3];
#pragma unroll
          for (int k = 0; k < D; ++k) {
            xa[k] = st[k][q - lo];
            xb2[k] = st[k][q + 1 - lo];
          }
          const double ua = scaled_sq<D>(xp, xa, a.kt.inv0);
          const double ub = scaled_sq<D>(xp, xb2, a.kt.inv0);
          if (local(q, ua)) hit_at(q, ua, xa);
          if (local(q + 1, ub)) hit_at(q + 1, ub, xb2);
        }
        if (q < e) {
          double xq[3];
#pragma unroll
          for (int k = 0; k < D; ++k) xq[k] = st[k][q - lo];
          const double u2 = scaled_sq<D>(xp, xq, a.kt.inv0);
          if (local(q, u2)) hit_at(q, u2, xq);
        }
      } else {
        for (int32_t q0 = s; q0 < e; q0 += kCu) {
          double xq[kCu][3];
#pragma unroll
          for (int u = 0; u < kCu; ++u) load_point<D>(a.xb, a.n, min(q0 + u, e - 1), xq[u]);
#pragma unroll
          for (int u = 0; u < kCu; ++u) {
            const double u2 = scaled_sq<D>(xp, xq[u], a.kt.inv0);
            if (q0 + u < e && local(q0 + u, u2)) hit_at(q0 + u, u2, xq[u]);
          }
        }
      }
    }
  if (!row) return;
  if constexpr (!FILL) {
    a.counts[p] = cnt;
    if (mp == 0) a.gskip[p] = 0;
  } else {
    // the last nb % kBuf hits are still buffered, in bc[kBuf - rem ...]
    const int rem = nb % kBuf;
    if (cnt <= len)
#pragma unroll
      for (int j = 0; j < kBuf; ++j)
        if (j >= kBuf - rem) {
          a.col[out + cnt - kBuf + j] = bc[j];
          val[out + cnt - kBuf + j] = bv[j];
        }
    if (static_cast<int64_t>(cnt) != len) atomicOr(a.err, 1);
  }
}

// Rows with a group bit: |U_M| group entries come first in the row.
__global__ void __launch_bounds__(kThreads) k_group_counts(int64_t nm, const int32_t* __restrict__ mlist,
                                                           const int32_t* __restrict__ did,
                                                           const int64_t* __restrict__ uoff,
                                                           int32_t* __restrict__ counts, int32_t* __restrict__ gskip) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (k >= nm) return;
  const int32_t p = mlist[k];
  const int32_t nu = static_cast<int32_t>(uoff[did[k] + 1] - uoff[did[k]]);
  counts[p] += nu;
  gskip[p] = nu;
}

// Row layout of a row with group mask M: first the |U_M| group entries in U_M
// order (ascending column ids; every row with mask M shares this column list,
// which the group-block products exploit), then the local-only entries L'(p)
// in ascending order.
//
// The rows are written tile by tile: block (x, y) takes tile x of the group
// blocks (at most kTileRows rows, all with the mask M and so all with the
// column list U_M) and the chunk y of kUChunk entries of U_M.  Thread t takes
// the chunk's entries t, t + kThreads, ...: its point data (coordinates, mask
// and the f_i of its groups shared with M) are loaded once and serve every
// row of the tile, and each row's entries are written by consecutive threads
// to consecutive positions.  The rows' f_i are staged in LDS.  Every value
// is formed by the steps of entry_value with the row point first, as in the
// local rows, so K_pq and K_qp are bitwise equal.  The rows' local-only
// entries L'(p) after the group entries are written by k_local_rows.
constexpr int kUChunk = 1024;
constexpr int kFqRegs = 4;  // shared groups whose f_i(q) an entry keeps in registers

template <int D, typename VT, int CK>
__global__ void __launch_bounds__(kThreads) k_group_tile_fill(AsmArgs a, const int32_t* __restrict__ tiles,
                                                              const int32_t* __restrict__ grows) {
  __shared__ double sx[kTileRows][3];
  __shared__ double sF[kTileRows][kMaxGroups];
  __shared__ int32_t srow[kTileRows], sk[kTileRows];
  __shared__ int64_t sout[kTileRows];
  __shared__ double ssig[kTileRows], sSig[kTileRows];
  const int32_t* t = tiles + 4 * static_cast<int64_t>(blockIdx.x);
  const int32_t dm = t[0], i0 = t[1], rows = t[2];
  const int64_t u0 = a.uoff[dm];
  const int64_t nU = a.uoff[dm + 1] - u0;
  const int64_t c0 = static_cast<int64_t>(blockIdx.y) * kUChunk;
  if (c0 >= nU && blockIdx.y > 0) return;  // uniform: this tile has fewer chunks
  const int n1 = a.kt.n1;
  if (threadIdx.x < static_cast<unsigned>(rows)) {
    const int r = threadIdx.x;
    const int32_t p = grows[i0 + r];
    const int32_t k = a.midx[p];
    const int64_t out = a.row_ptr[p];
    const int64_t len = a.row_ptr[p + 1] - out;
    double xp[3] = {0, 0, 0};
    load_point<D>(a.xb, a.n, p, xp);
#pragma unroll
    for (int c = 0; c < 3; ++c) sx[r][c] = xp[c];
    srow[r] = p;
    sk[r] = k;
    // counts disagree: the row is left unwritten and the error reported
    const bool ok = a.gskip[p] == nU && len >= nU;
    sout[r] = ok ? out : -1;
    if (!ok && blockIdx.y == 0) atomicOr(a.err, 4);
    ssig[r] = CK == 2 ? a.kt.core.sig[p] : 0.0;
    sSig[r] = CK == 2 ? a.kt.core.Sig[p] : 0.0;
  }
  for (int e = threadIdx.x; e < rows * n1; e += kThreads) {
    const int r = e / n1, i = e % n1;
    sF[r][i] = a.F[static_cast<int64_t>(a.midx[grows[i0 + r]]) * n1 + i];
  }
  __syncthreads();
  const uint64_t M = a.mask[srow[0]];
  VT* val = static_cast<VT*>(a.val);
  const int64_t c1 = min(nU, c0 + kUChunk);
  for (int64_t kk = c0 + threadIdx.x; kk < c1; kk += kThreads) {
    const int32_t u = a.ulist[u0 + kk];
    double xq[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) xq[k] = a.ux[k * a.utotal + u0 + kk];
    const uint64_t shared = a.umask[u0 + kk] & M;
    // f_i(q) of the first kFqRegs shared groups, increasing i
    double fq[kFqRegs];
    int gi[kFqRegs];
    uint64_t rest = shared;
#pragma unroll
    for (int j = 0; j < kFqRegs; ++j) {
      gi[j] = rest ? __builtin_ctzll(rest) : 0;
      fq[j] = rest ? a.uF[gi[j] * a.utotal + u0 + kk] : 0.0;
      rest &= rest - 1;
    }
    const int ng = __popcll(shared);
    double sq = 0.0, Sq = 0.0;
    if constexpr (CK == 2) {
      sq = a.kt.core.sig[u];
      Sq = a.kt.core.Sig[u];
    }
    for (int r = 0; r < rows; ++r) {
      const int64_t out = sout[r];
      if (out < 0) continue;
      const int32_t p = srow[r];
      const double xp[3] = {sx[r][0], sx[r][1], sx[r][2]};
      const double u2 = scaled_sq<D>(xp, xq, a.kt.inv0);
      double cv = 1.0;
      if constexpr (CK == 1) cv = core_value<D, 1>(a.kt.core, xp, xq, 0.0, 0.0, 0.0, 0.0);
      if constexpr (CK == 2) cv = core_value<D, 2>(a.kt.core, xp, xq, ssig[r], sSig[r], sq, Sq);
      double acc = entry_local(a.kt, u2);
#pragma unroll
      for (int j = 0; j < kFqRegs; ++j)
        if (j < ng) acc = entry_add_group(acc, sF[r][gi[j]], fq[j]);
      if (ng > kFqRegs) {  // rare: the remaining groups from memory, increasing i
        uint64_t more = rest;
        while (more) {
          const int i = __builtin_ctzll(more);
          more &= more - 1;
          acc = entry_add_group(acc, sF[r][i], a.uF[i * a.utotal + u0 + kk]);
        }
      }
      const VT vs = static_cast<VT>(entry_finish(a.kt, acc, cv, u == p, p));
      a.col[out + kk] = u;
      val[out + kk] = vs;
      if (u == p) a.diag[p] = static_cast<double>(vs);
    }
  }
}

// long rows of the CSR part outside the group blocks (lengths without the
// leading group entries); also the longest full row
__global__ void __launch_bounds__(kThreads) k_long_flags(int64_t n, const int32_t* __restrict__ counts,
                                                         const int32_t* __restrict__ gskip,
                                                         int32_t* __restrict__ flag, int32_t* __restrict__ maxrow) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  int32_t c = 0;
  if (p < n) {
    c = counts[p];
    flag[p] = (c - gskip[p]) > kLongRow ? 1 : 0;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) c = max(c, __shfl_xor(c, off, kWave));
  __shared__ int32_t wmax[kThreads / kWave];
  if (lane_id() == 0) wmax[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t m = wmax[0];
    for (int i = 1; i < kThreads / kWave; ++i) m = max(m, wmax[i]);
    atomicMax(maxrow, m);
  }
}

__global__ void __launch_bounds__(kThreads) k_long_compact(int64_t n, const int32_t* __restrict__ flag,
                                                           const int32_t* __restrict__ pos,
                                                           int32_t* __restrict__ list) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (p < n && flag[p]) list[pos[p]] = static_cast<int32_t>(p);
}

// sigma(x_p), Sigma(x_p) of the nonstationary core for every binned point
template <int D>
__global__ void __launch_bounds__(kThreads) k_core_fields(CoreBasis cb, int64_t n, const double* __restrict__ xb,
                                                          double* __restrict__ sig, double* __restrict__ Sig) {
  const int64_t p = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x;
  if (p >= n) return;
  double x[3];
  load_point<D>(xb, n, p, x);
  double s, S;
  core_point_fields<D>(cb, x, &s, &S);
  sig[p] = s;
  Sig[p] = S;
}

template <typename F3>
void dispatch_core(int kind, F3&& f) {
  if (kind == GP_CORE_MATERN)
    f(std::integral_constant<int, 1>{});
  else if (kind == GP_CORE_PACIOREK)
    f(std::integral_constant<int, 2>{});
  else
    f(std::integral_constant<int, 0>{});
}

template <typename F3>
void dispatch_d(int d, F3&& f) {
  if (d == 1)
    f(std::integral_constant<int, 1>{});
  else if (d == 2)
    f(std::integral_constant<int, 2>{});
  else
    f(std::integral_constant<int, 3>{});
}

}  // namespace

// ------------------------------------------------------------------ host
void upload_theta(gp_ctx* c, const gp_theta* th, Bump** bumps_dev, KernelTheta* kt) {
  const int nb = th->n1 * th->n2;
  std::vector<Bump> hb(nb);
  for (int b = 0; b < nb; ++b) {
    for (int k = 0; k < 3; ++k) {
      hb[b].h[k] = k < th->d ? th->h[b * th->d + k] : 0.0;
      hb[b].inv[k] = k < th->d ? 1.0 / th->r[b * th->d + k] : 0.0;
    }
    hb[b].a = th->a[b];
    hb[b].b = th->b[b];
  }
  Bump* dst = static_cast<Bump*>(workspace(c, 0, sizeof(Bump) * std::max(nb, 1)));
  Bump* staging = static_cast<Bump*>(pinned_for_write(c, sizeof(Bump) * std::max(nb, 1)));
  std::memcpy(staging, hb.data(), sizeof(Bump) * nb);
  h2d_async(c, dst, staging, sizeof(Bump) * nb);
  *bumps_dev = dst;
  kt->d = th->d;
  kt->n1 = th->n1;
  kt->n2 = th->n2;
  kt->variant = th->wendland_variant;
  kt->s0 = th->s0;
  kt->nugget = th->nugget;
  for (int k = 0; k < 3; ++k) kt->inv0[k] = k < th->d ? 1.0 / th->r0[k] : 0.0;
  kt->bumps = dst;
  core_params(th, &kt->core, nullptr);
}

uint64_t theta_hash(const gp_theta* th) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t bytes) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < bytes; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  };
  auto arr = [&](const double* p, int64_t count) {
    if (p && count > 0) mix(p, sizeof(double) * static_cast<size_t>(count));
  };
  const int d = th->d, nb = th->n1 * th->n2;
  const int32_t ints[4] = {th->d, th->n1, th->n2, th->wendland_variant};
  mix(ints, sizeof(ints));
  mix(&th->s0, sizeof(double));
  arr(th->r0, d);
  arr(th->h, static_cast<int64_t>(nb) * d);
  arr(th->r, static_cast<int64_t>(nb) * d);
  arr(th->a, nb);
  arr(th->b, nb);
  mix(&th->nugget, sizeof(double));
  // tau2 is not hashed: it enters the matrix only, never C_y
  const gp_core* co = th->core;
  const int32_t kind = co ? co->kind : GP_CORE_NONE;
  mix(&kind, sizeof(kind));
  if (kind != GP_CORE_NONE) {
    mix(&co->nu2, sizeof(co->nu2));
    mix(&co->sigma0, sizeof(double));
    arr(co->ell, d);
    if (kind == GP_CORE_PACIOREK) {
      mix(&co->Sigma0, sizeof(double));
      mix(&co->n_basis, sizeof(co->n_basis));
      arr(co->width, d);
      arr(co->centers, static_cast<int64_t>(co->n_basis) * d);
      arr(co->phi_sigma, co->n_basis);
      arr(co->phi_Sigma, co->n_basis);
    }
  }
  return h;
}

void core_params(const gp_theta* th, KernelCore* kc, CoreBasis* cb) {
  *kc = KernelCore{};
  kc->kind = GP_CORE_NONE;
  if (cb) *cb = CoreBasis{};
  const gp_core* co = th->core;
  if (!co || co->kind == GP_CORE_NONE) return;
  const int d = th->d;
  kc->kind = co->kind;
  kc->nu2 = co->nu2;
  kc->s2 = co->sigma0 * co->sigma0;
  for (int k = 0; k < 3; ++k) kc->inv_ell[k] = k < d ? 1.0 / co->ell[k] : 0.0;
  if (cb && co->kind == GP_CORE_PACIOREK) {
    cb->nb = co->n_basis;
    cb->log_sigma0 = std::log(co->sigma0);
    cb->log_Sigma0 = std::log(co->Sigma0);
    for (int m = 0; m < co->n_basis; ++m) {
      for (int k = 0; k < d; ++k) cb->c[m][k] = co->centers[m * d + k];
      cb->phi_s[m] = co->phi_sigma[m];
      cb->phi_S[m] = co->phi_Sigma[m];
    }
    for (int k = 0; k < 3; ++k) cb->w[k] = k < d ? co->width[k] : 1.0;
  }
}

void core_fields(gp_ctx* c, const gp_dataset* ds, const CoreBasis& cb, double* sig, double* Sig) {
  const int64_t n = ds->n;
  dispatch_d(ds->d, [&](auto DD) {
    constexpr int D = decltype(DD)::value;
    ProfScope ps(c, "asm_core_fields");
    hipLaunchKernelGGL((k_core_fields<D>), dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, cb, n, ds->xb,
                       sig, Sig);
  });
  check_launch("core fields");
}

Grid make_grid(const gp_dataset* ds, const gp_theta* th) {
  Grid g{};
  for (int k = 0; k < 3; ++k) {
    g.lo[k] = ds->lo[k];
    g.cell[k] = ds->cell[k];
    g.inv_cell[k] = 1.0 / ds->cell[k];
    g.g[k] = ds->g[k];
    if (k < ds->d) {
      // rings needed so that |x_p - x_q| < r0 implies |cell_p - cell_q| <= R even
      // after rounding of the cell computation (margin 1e-9 relative)
      const double need = th->r0[k] * (1.0 + 1e-9) / ds->cell[k];
      double R = std::ceil(need);
      if (R < 1) R = 1;
      if (R > ds->g[k]) R = ds->g[k];
      g.R[k] = static_cast<int32_t>(R);
    } else {
      g.R[k] = 0;
    }
  }
  return g;
}

void compute_features(gp_ctx* c, const gp_dataset* ds, const KernelTheta& kt, Features* f, int ws_base) {
  const int64_t n = ds->n;
  f->mask = static_cast<uint64_t*>(workspace(c, ws_base + 0, sizeof(uint64_t) * n));
  f->midx = static_cast<int32_t*>(workspace(c, ws_base + 1, sizeof(int32_t) * n));
  int32_t* flag = static_cast<int32_t*>(workspace(c, ws_base + 2, sizeof(int32_t) * n));
  int32_t* pos = static_cast<int32_t*>(workspace(c, ws_base + 3, sizeof(int32_t) * (n + 1)));
  dispatch_d(ds->d, [&](auto DD) {
    constexpr int D = decltype(DD)::value;
    ProfScope ps(c, "asm_mask");
    hipLaunchKernelGGL((k_mask<D>), dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, kt, n, ds->xb,
                       f->mask, flag);
  });
  check_launch("mask");
  {
    ProfScope ps(c, "asm_scan");
    scan_i32_to_i32(c, flag, pos, n);
  }
  int32_t* h = static_cast<int32_t*>(pinned(c, sizeof(int32_t)));
  GPS_HIP(hipMemcpyAsync(h, pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  f->nm = *h;
  f->mlist = static_cast<int32_t*>(workspace(c, ws_base + 4, sizeof(int32_t) * std::max<int64_t>(f->nm, 1)));
  uint64_t* mmask = static_cast<uint64_t*>(workspace(c, ws_base + 5, sizeof(uint64_t) * std::max<int64_t>(f->nm, 1)));
  f->mmask = mmask;
  {
    ProfScope ps(c, "asm_compact");
    hipLaunchKernelGGL(k_compact_masked, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, n, flag, pos,
                       f->mask, f->midx, f->mlist, mmask);
  }
  check_launch("compact masked");
  f->F = static_cast<double*>(workspace(c, ws_base + 6, sizeof(double) * std::max<int64_t>(f->nm * kt.n1, 1)));
  if (f->nm > 0) {
    dispatch_d(ds->d, [&](auto DD) {
      constexpr int D = decltype(DD)::value;
      ProfScope ps(c, "asm_bump_values");
      hipLaunchKernelGGL((k_fvals<D>), dim3(grid_for(f->nm, kThreads)), dim3(kThreads), 0, c->stream, kt, n, f->nm,
                         ds->xb, f->mlist, f->F);
    });
    check_launch("bump values");
  }
}

// Workspace slots used by assembly (0: bumps; 1..7: features; 8..: below)
// Distinct masks of the masked points: dmask ascending, did[i] = index of hm[i]
// in dmask, mult[a] = number of points with mask dmask[a] (hash table, then
// the few distinct masks are sorted).
static void distinct_masks(const std::vector<uint64_t>& hm, std::vector<uint64_t>* dmask, std::vector<int32_t>* did,
                           std::vector<int64_t>* mult) {
  const int64_t nm = static_cast<int64_t>(hm.size());
  int bits = 10;
  std::vector<uint64_t> key(size_t(1) << bits, 0);   // 0 = empty (masks are nonzero)
  std::vector<int32_t> slot_id(size_t(1) << bits, -1);
  std::vector<uint64_t> first;                       // distinct masks in order of appearance
  std::vector<int32_t> tmp(nm);
  auto find = [&](uint64_t m) -> int32_t& {
    size_t h = static_cast<size_t>((m * 0x9E3779B97F4A7C15ull) >> (64 - bits));
    const size_t msk = (size_t(1) << bits) - 1;
    while (key[h] != 0 && key[h] != m) h = (h + 1) & msk;
    key[h] = m;
    return slot_id[h];
  };
  for (int64_t i = 0; i < nm; ++i) {
    int32_t& id = find(hm[i]);
    if (id < 0) {
      id = static_cast<int32_t>(first.size());
      first.push_back(hm[i]);
      if (2 * first.size() > key.size()) {  // keep the load below one half
        ++bits;
        key.assign(size_t(1) << bits, 0);
        slot_id.assign(size_t(1) << bits, -1);
        for (size_t d = 0; d < first.size(); ++d) find(first[d]) = static_cast<int32_t>(d);
      }
    }
    tmp[i] = find(hm[i]);
  }
  const size_t nD = first.size();
  std::vector<int32_t> order(nD), rank(nD);
  for (size_t d = 0; d < nD; ++d) order[d] = static_cast<int32_t>(d);
  std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return first[x] < first[y]; });
  dmask->resize(nD);
  mult->assign(nD, 0);
  for (size_t r = 0; r < nD; ++r) {
    rank[order[r]] = static_cast<int32_t>(r);
    (*dmask)[r] = first[order[r]];
  }
  did->resize(nm);
  for (int64_t i = 0; i < nm; ++i) {
    (*did)[i] = rank[tmp[i]];
    ++(*mult)[(*did)[i]];
  }
}

gp_matrix* assemble(gp_ctx* c, const gp_dataset* ds, const gp_theta* th, int prec) {
  const int64_t n = ds->n;
  Bump* bumps = nullptr;
  KernelTheta kt{};
  upload_theta(c, th, &bumps, &kt);
  if (th->tau2) {
    // per-point error variances to binned order, checked before any work
    double* t2 = static_cast<double*>(workspace(c, 121, sizeof(double) * n));
    permute_to_binned<double>(c, ds, 1, th->tau2, t2);
    GPS_HIP(hipMemsetAsync(c->err_flag, 0, sizeof(int), c->stream));
    hipLaunchKernelGGL(k_check_tau2, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, n, t2, c->err_flag);
    check_launch("tau2 check");
    int* herr = static_cast<int*>(pinned(c, sizeof(int)));
    GPS_HIP(hipMemcpyAsync(herr, c->err_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    GPS_REQUIRE(*herr == 0, GP_EINVAL, "gp_assemble: tau2 must be finite and >= 0");
    kt.tau2 = t2;
  }
  Features f;
  compute_features(c, ds, kt, &f, 1);
  const int64_t nm = f.nm;
  uint64_t* mmask = f.mmask;
  // masks of the masked points to the host; the local-row count pass (which
  // needs only the masks) runs while the host groups them
  std::vector<uint64_t> hm(nm);
  std::vector<int32_t> hmlist(nm);
  if (nm > 0) {
    GPS_HIP(hipMemcpyAsync(hm.data(), mmask, sizeof(uint64_t) * nm, hipMemcpyDeviceToHost, c->stream));
    GPS_HIP(hipMemcpyAsync(hmlist.data(), f.mlist, sizeof(int32_t) * nm, hipMemcpyDeviceToHost, c->stream));
    record_aux(c);
  }
  if (kt.core.kind == GP_CORE_PACIOREK) {
    KernelCore unused;
    CoreBasis cb;
    core_params(th, &unused, &cb);
    double* sig = static_cast<double*>(workspace(c, 90, sizeof(double) * n));
    double* Sig = static_cast<double*>(workspace(c, 91, sizeof(double) * n));
    core_fields(c, ds, cb, sig, Sig);
    kt.core.sig = sig;
    kt.core.Sig = Sig;
  }
  const Grid grid = make_grid(ds, th);
  AsmArgs a{};
  a.kt = kt;
  a.n = n;
  a.xb = ds->xb;
  a.key = ds->key;
  a.cell_start = ds->cell_start;
  for (int k = 0; k < 3; ++k) {
    a.g[k] = grid.g[k];
    a.R[k] = grid.R[k];
  }
  a.mask = f.mask;
  a.midx = f.midx;
  a.mlist = f.mlist;
  a.F = f.F;
  a.nm = nm;
  a.err = c->err_flag;
  const int d = ds->d;
  // gskip belongs to the matrix, allocated before the count pass writes it; a
  // failure below releases whatever the matrix holds by then
  auto release = [c](gp_matrix* x) { destroy_matrix(c, x); };
  std::unique_ptr<gp_matrix, decltype(release)> m(new gp_matrix(), release);
  m->ds = ds;
  m->n = n;
  m->prec = prec;
  m->gskip = dev_new<int32_t>(c, n);
  a.gskip = m->gskip;
  a.counts = static_cast<int32_t*>(workspace(c, 12, sizeof(int32_t) * n));
  dispatch_d(d, [&](auto DD) {
    constexpr int D = decltype(DD)::value;
    ProfScope ps(c, "asm_count_local");
    hipLaunchKernelGGL((k_local_rows<D, false, double>), dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream,
                       a);
  });
  check_launch("count local");
  std::vector<uint64_t> dmask;
  std::vector<int64_t> uoff(1, 0);
  std::vector<int32_t> did;
  std::vector<int64_t> mult;
  if (nm > 0) {
    wait_aux(c);
    distinct_masks(hm, &dmask, &did, &mult);
    const size_t nD = dmask.size();
    uoff.resize(nD + 1);
    uoff[0] = 0;
    for (size_t x = 0; x < nD; ++x) {
      int64_t sum = 0;
      for (size_t y = 0; y < nD; ++y)
        if (dmask[x] & dmask[y]) sum += mult[y];
      uoff[x + 1] = uoff[x] + sum;
    }
    GPS_REQUIRE(uoff[nD] < (int64_t(1) << 31), GP_ENOMEM, "gp_assemble: bump group lists too large");
  }
  const int64_t nD = static_cast<int64_t>(dmask.size());
  const int64_t utotal = uoff.back();
  int64_t max_nu = 1;
  for (int64_t x = 0; x < nD; ++x) max_nu = std::max(max_nu, uoff[x + 1] - uoff[x]);
  // rows grouped by their mask (stable, so ascending within a mask) and cut into
  // tiles of at most kTileRows rows for the group-block products
  std::vector<int32_t> goff(nD + 1, 0), grows(nm);
  for (int64_t i = 0; i < nm; ++i) ++goff[did[i] + 1];
  for (int64_t a = 0; a < nD; ++a) goff[a + 1] += goff[a];
  {
    std::vector<int32_t> cur(goff.begin(), goff.end() - 1);
    for (int64_t i = 0; i < nm; ++i) grows[cur[did[i]]++] = hmlist[i];
  }
  std::vector<int32_t> tiles, stiles, pieces;
  int64_t nnz_group = 0, gemv_stage = 0, gemm_stage = 0;
  for (int64_t a = 0; a < nD; ++a) {
    const int32_t nu = static_cast<int32_t>(uoff[a + 1] - uoff[a]);
    nnz_group += static_cast<int64_t>(goff[a + 1] - goff[a]) * nu;
    gemv_stage += static_cast<int64_t>((goff[a + 1] - goff[a] + kTileRows - 1) / kTileRows) * nu;
    gemm_stage += static_cast<int64_t>((goff[a + 1] - goff[a] + kSuperRows - 1) / kSuperRows) * nu;
    for (int32_t i = goff[a]; i < goff[a + 1]; i += kTileRows)
      tiles.insert(tiles.end(), {static_cast<int32_t>(a), i, std::min<int32_t>(kTileRows, goff[a + 1] - i), 0});
    for (int32_t i = goff[a]; i < goff[a + 1]; i += kSuperRows) {
      const int32_t rows = std::min<int32_t>(kSuperRows, goff[a + 1] - i);
      const int32_t np = (nu + kPiece - 1) / kPiece;
      stiles.insert(stiles.end(), {i, rows, static_cast<int32_t>(pieces.size() / 4), np});
      for (int32_t k0 = 0; k0 < nu; k0 += kPiece) pieces.insert(pieces.end(), {static_cast<int32_t>(a), i, rows, k0});
    }
  }
  // largest group blocks first, so that the short ones fill the tail of the launch
  {
    const size_t nt = tiles.size() / 4;
    std::vector<int32_t> idx(nt);
    for (size_t i = 0; i < nt; ++i) idx[i] = static_cast<int32_t>(i);
    auto work = [&](int32_t i) {
      const int32_t a = tiles[4 * i];
      return (uoff[a + 1] - uoff[a]) * static_cast<int64_t>(tiles[4 * i + 2]);
    };
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return work(x) > work(y); });
    std::vector<int32_t> sorted(tiles.size());
    for (size_t i = 0; i < nt; ++i)
      for (int f = 0; f < 4; ++f) sorted[4 * i + f] = tiles[4 * idx[i] + f];
    tiles.swap(sorted);
  }
  const int64_t ntiles = static_cast<int64_t>(tiles.size() / 4);
  const int64_t nstiles = static_cast<int64_t>(stiles.size() / 4);
  const int64_t npieces = static_cast<int64_t>(pieces.size() / 4);
  tiles.insert(tiles.end(), stiles.begin(), stiles.end());
  tiles.insert(tiles.end(), pieces.begin(), pieces.end());

  m->nugget = th->nugget;
  m->theta_hash = theta_hash(th);
  m->nnz_group = nnz_group;
  m->gemv_stage = gemv_stage;
  m->gemm_stage = gemm_stage;
  m->nD = nD;
  m->utotal = utotal;
  m->nm = nm;
  m->ntiles = ntiles;
  m->nstiles = nstiles;
  m->npieces = npieces;
  m->g_uoff = dev_new<int64_t>(c, nD + 1);
  m->g_ulist = dev_new<int32_t>(c, std::max<int64_t>(utotal, 1));
  m->g_rows = dev_new<int32_t>(c, std::max<int64_t>(nm, 1));
  m->g_tiles = dev_new<int32_t>(c, std::max<int64_t>(4 * (ntiles + nstiles + npieces), 4));
  m->bytes += sizeof(int32_t) * (n + utotal + nm + 4 * (ntiles + nstiles + npieces)) + sizeof(int64_t) * (nD + 1);
  int32_t* d_did = static_cast<int32_t*>(workspace(c, 8, sizeof(int32_t) * std::max<int64_t>(nm, 1)));
  uint64_t* d_dmask = static_cast<uint64_t*>(workspace(c, 9, sizeof(uint64_t) * std::max<int64_t>(nD, 1)));
  int64_t* d_uoff = m->g_uoff;
  int32_t* d_ulist = m->g_ulist;
  {
    const size_t b_did = sizeof(int32_t) * nm, b_dm = sizeof(uint64_t) * nD, b_uo = sizeof(int64_t) * (nD + 1);
    const size_t b_gr = sizeof(int32_t) * nm, b_ti = sizeof(int32_t) * tiles.size();
    char* st = static_cast<char*>(pinned_for_write(c, b_did + b_dm + b_uo + b_gr + b_ti + 64));
    char* o = st;
    auto put = [&](const void* src, size_t nb, void* dst) {
      if (!nb) return;
      std::memcpy(o, src, nb);
      h2d_async(c, dst, o, nb);
      o += nb;
    };
    put(did.data(), b_did, d_did);
    put(dmask.data(), b_dm, d_dmask);
    put(uoff.data(), b_uo, d_uoff);
    put(grows.data(), b_gr, m->g_rows);
    put(tiles.data(), b_ti, m->g_tiles);
    if (nD) {
      ProfScope ps(c, "asm_group_lists");
      hipLaunchKernelGGL(k_ulists, dim3(static_cast<unsigned>(nD)), dim3(kUlThreads), 0, c->stream, nm, mmask, f.mlist,
                         d_dmask, d_uoff, d_ulist);
      check_launch("group lists");
    }
  }

  a.did = d_did;
  a.uoff = d_uoff;
  a.ulist = d_ulist;
  a.utotal = utotal;
  GPS_HIP(hipMemsetAsync(c->err_flag, 0, sizeof(int), c->stream));
  // rows with a group bit: their |U_M| group entries come first
  if (nm > 0) {
    ProfScope ps(c, "asm_compact");
    hipLaunchKernelGGL(k_group_counts, dim3(grid_for(nm, kThreads)), dim3(kThreads), 0, c->stream, nm, f.mlist, d_did,
                       d_uoff, a.counts, m->gskip);
    check_launch("group counts");
  }

  m->row_ptr = dev_new<int64_t>(c, n + 1);
  m->bytes += sizeof(int64_t) * (n + 1);
  int32_t* lflag = static_cast<int32_t*>(workspace(c, 15, sizeof(int32_t) * n));
  int32_t* lpos = static_cast<int32_t*>(workspace(c, 16, sizeof(int32_t) * (n + 1)));
  int32_t* maxrow = static_cast<int32_t*>(workspace(c, 17, sizeof(int32_t) * 2));
  {
    ProfScope ps(c, "asm_scan");
    scan_i32_to_i64(c, a.counts, m->row_ptr, n);
    GPS_HIP(hipMemsetAsync(maxrow, 0, sizeof(int32_t), c->stream));
    hipLaunchKernelGGL(k_long_flags, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, n, a.counts,
                       m->gskip, lflag, maxrow);
    check_launch("long flags");
    scan_i32_to_i32(c, lflag, lpos, n);
  }
  // one synchronisation: nnz, number of long rows, longest row
  struct Sizes {
    int64_t nnz;
    int32_t nlong, maxrow;
  };
  Sizes* hs = static_cast<Sizes*>(pinned(c, sizeof(Sizes)));
  GPS_HIP(hipMemcpyAsync(&hs->nnz, m->row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  GPS_HIP(hipMemcpyAsync(&hs->nlong, lpos + n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  GPS_HIP(hipMemcpyAsync(&hs->maxrow, maxrow, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  const Sizes sz = *hs;
  m->nnz = sz.nnz;
  m->max_row = sz.maxrow;
  m->n_long = sz.nlong;
  GPS_REQUIRE(m->nnz < (int64_t(1) << 40), GP_ENOMEM, "gp_assemble: too many nonzeros");

  const size_t vbytes = prec == GP_MIXED ? sizeof(float) : sizeof(double);
  // 64 entries of padding: the products read column ids and values in groups
  // of four that can run past a row's end.  The padding is zeroed: a value read
  // there is multiplied by a zero weight, and 0 x (stale NaN or Inf) is NaN.
  m->col = dev_new<int32_t>(c, m->nnz + kCsrPad);
  m->val = dev_alloc(c, vbytes * (m->nnz + kCsrPad));
  GPS_HIP(hipMemsetAsync(m->col + m->nnz, 0, sizeof(int32_t) * kCsrPad, c->stream));
  GPS_HIP(hipMemsetAsync(static_cast<char*>(m->val) + vbytes * m->nnz, 0, vbytes * kCsrPad, c->stream));
  m->diag = dev_new<double>(c, n);
  m->long_rows = dev_new<int32_t>(c, std::max<int64_t>(m->n_long, 1));
  m->bytes += (sizeof(int32_t) + vbytes) * m->nnz + sizeof(double) * n + sizeof(int32_t) * m->n_long;
  {
    ProfScope ps(c, "asm_compact");
    hipLaunchKernelGGL(k_long_compact, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, c->stream, n, lflag, lpos,
                       m->long_rows);
  }
  check_launch("long rows");

  {
    const int64_t ut = std::max<int64_t>(utotal, 1);
    double* ux = static_cast<double*>(workspace(c, 19, sizeof(double) * 3 * ut));
    uint64_t* umask = static_cast<uint64_t*>(workspace(c, 10, sizeof(uint64_t) * ut));
    double* uF = static_cast<double*>(workspace(c, 11, sizeof(double) * std::max(kt.n1, 1) * ut));
    a.ux = ux;
    a.umask = umask;
    a.uF = uF;
    if (utotal > 0)
      dispatch_d(ds->d, [&](auto DD) {
        constexpr int D = decltype(DD)::value;
        ProfScope ps(c, "asm_group_lists");
        hipLaunchKernelGGL((k_ugather<D>), dim3(grid_for(utotal, kThreads)), dim3(kThreads), 0, c->stream, a, ux,
                           umask, uF);
      });
    check_launch("group member data");
  }
  a.row_ptr = m->row_ptr;
  a.col = m->col;
  a.val = m->val;
  a.diag = m->diag;
  dispatch_d(d, [&](auto DD) {
    constexpr int D = decltype(DD)::value;
    auto fill = [&](auto VTv) {
      using VT = decltype(VTv);
      dispatch_core(kt.core.kind, [&](auto CC) {
        constexpr int CK = decltype(CC)::value;
        {
          ProfScope ps(c, "asm_fill_local");
          hipLaunchKernelGGL((k_local_rows<D, true, VT, CK>), dim3(grid_for(n, kThreads)), dim3(kThreads), 0,
                             c->stream, a);
        }
        if (ntiles > 0) {
          ProfScope ps(c, "asm_fill_group");
          hipLaunchKernelGGL((k_group_tile_fill<D, VT, CK>),
                             dim3(static_cast<unsigned>(ntiles), static_cast<unsigned>((max_nu + kUChunk - 1) / kUChunk)),
                             dim3(kThreads), 0, c->stream, a, m->g_tiles, m->g_rows);
        }
      });
    };
    if (prec == GP_MIXED)
      fill(float{});
    else
      fill(double{});
  });
  check_launch("fill");
  int* herr = static_cast<int*>(pinned(c, sizeof(int)));
  GPS_HIP(hipMemcpyAsync(herr, c->err_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  sync(c);
  if (*herr != 0) {
    const int e = *herr;
    destroy_matrix(c, m.release());
    throw Error{GP_EDEVICE, "gp_assemble: count and fill passes disagree (code " + std::to_string(e) + ")"};
  }
  return m.release();
}

void destroy_matrix(gp_ctx* c, gp_matrix* m) {
  if (!m) return;
  const size_t vbytes = m->prec == GP_MIXED ? sizeof(float) : sizeof(double);
  if (m->row_ptr) dev_free(c, m->row_ptr, sizeof(int64_t) * (m->n + 1));
  if (m->col) dev_free(c, m->col, sizeof(int32_t) * (m->nnz + kCsrPad));
  if (m->val) dev_free(c, m->val, vbytes * (m->nnz + kCsrPad));
  if (m->diag) dev_free(c, m->diag, sizeof(double) * m->n);
  if (m->long_rows) dev_free(c, m->long_rows, sizeof(int32_t) * std::max<int64_t>(m->n_long, 1));
  free_block_jacobi(c, m);
  free_quads(c, m);
  free_col16(c, m);
  if (m->gskip) dev_free(c, m->gskip, sizeof(int32_t) * m->n);
  if (m->g_uoff) dev_free(c, m->g_uoff, sizeof(int64_t) * (m->nD + 1));
  if (m->g_ulist) dev_free(c, m->g_ulist, sizeof(int32_t) * std::max<int64_t>(m->utotal, 1));
  if (m->g_rows) dev_free(c, m->g_rows, sizeof(int32_t) * std::max<int64_t>(m->nm, 1));
  if (m->g_tiles)
    dev_free(c, m->g_tiles, sizeof(int32_t) * std::max<int64_t>(4 * (m->ntiles + m->nstiles + m->npieces), 4));
  delete m;
}

}  // namespace gps
