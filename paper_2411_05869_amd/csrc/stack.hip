// Block-diagonal stacking of assembled matrices, for the batched likelihood of
// several small problems (Sec. 3.3 and Appendix C: the sampler evaluates the
// likelihood of many hyper-parameter proposals, each a sparse solve and a
// log-determinant of a matrix with a few thousand to tens of thousands of
// rows).  A problem that small fills only a fraction of the chip per launch;
// stacked, the problems share every product and vector launch.
//
// The stacked matrix holds the arrays the products and the preconditioner
// read.  Problem r's rows, columns, group lists, tiles and row quads are
// shifted by its row (and list) offsets, so every stacked row holds the
// entries of the same row of its own matrix in the same order, and a product
// gives it bitwise the value the problem's own product gives.
#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "device.hpp"

namespace gps {
namespace {

constexpr int kThreads = 256;

// one piece of a stacked array: count entries of src, written from dst on,
// with add[] added as the mode says
struct Piece {
  const void* src;
  int64_t count;
  int64_t dst;
  int64_t add[4];
};

enum StackMode { kCopy = 0, kShift = 1, kShift4 = 2, kRowCode = 3 };

// piece blockIdx.y of the table; grid-stride over its entries
template <typename T, int MODE>
__global__ void __launch_bounds__(kThreads) k_stack(const Piece* __restrict__ pieces, T* __restrict__ out) {
  const Piece pc = pieces[blockIdx.y];
  const T* src = static_cast<const T*>(pc.src);
  T* dst = out + pc.dst;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < pc.count;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const T v = src[i];
    if constexpr (MODE == kCopy) {
      dst[i] = v;
    } else if constexpr (MODE == kShift) {
      dst[i] = static_cast<T>(v + pc.add[0]);
    } else if constexpr (MODE == kShift4) {
      dst[i] = static_cast<T>(v + pc.add[i & 3]);
    } else {
      // listed-row codes: -1 stays, a row r >= 0 and a group row -(r + 2) move by the row offset
      dst[i] = v == -1 ? v : (v >= 0 ? static_cast<T>(v + pc.add[0]) : static_cast<T>(v - pc.add[0]));
    }
  }
}

// the closing entry of an offset array (its total)
__global__ void k_put_i64(int64_t* __restrict__ p, int64_t v) { *p = v; }
__global__ void k_put_i32(int32_t* __restrict__ p, int32_t v) { *p = v; }

}  // namespace

gp_matrix* stack_matrices(gp_ctx* c, int R, const gp_matrix* const* ms, bool block_jacobi) {
  GPS_REQUIRE(R >= 1, GP_EINVAL, "stack: no matrices");
  const int prec = ms[0]->prec;
  for (int r = 0; r < R; ++r) {
    GPS_REQUIRE(ms[r]->prec == prec, GP_EINVAL, "stack: the matrices of a batch must share one precision");
    GPS_REQUIRE(ms[r]->qptr != nullptr, GP_EDEVICE, "stack: row quads not built");
    GPS_REQUIRE(ms[r]->ntrow % 4 == 0, GP_EDEVICE, "stack: listed rows not a multiple of four");
    GPS_REQUIRE(!block_jacobi || ms[r]->binv != nullptr, GP_EDEVICE, "stack: preconditioner not built");
  }
  const size_t vbytes = prec == GP_MIXED ? sizeof(float) : sizeof(double);
  // offsets of every problem in every stacked array
  struct Off {
    int64_t row, nnz, nlong, nD, utotal, nm, tiles, stiles, pieces, nblk, binv, trow, quads;
  };
  std::vector<Off> off(R + 1);
  off[0] = Off{};
  for (int r = 0; r < R; ++r) {
    const gp_matrix* m = ms[r];
    Off& a = off[r + 1];
    const Off& b = off[r];
    a.row = b.row + m->n;
    a.nnz = b.nnz + m->nnz;
    a.nlong = b.nlong + m->n_long;
    a.nD = b.nD + m->nD;
    a.utotal = b.utotal + m->utotal;
    a.nm = b.nm + m->nm;
    a.tiles = b.tiles + m->ntiles;
    a.stiles = b.stiles + m->nstiles;
    a.pieces = b.pieces + m->npieces;
    a.nblk = b.nblk + (block_jacobi ? m->nblk : 0);
    a.binv = b.binv + (block_jacobi ? m->binv_len : 0);
    a.trow = b.trow + m->ntrow;
    a.quads = b.quads + m->nquad;
  }
  const Off& tot = off[R];
  GPS_REQUIRE(tot.row + 2 < (int64_t(1) << 31) && tot.trow < (int64_t(1) << 31) && tot.nm < (int64_t(1) << 31) &&
                  tot.nD < (int64_t(1) << 31) && tot.pieces < (int64_t(1) << 31),
              GP_EINVAL, "stack: the batch is too large for 32-bit row ids");

  auto release = [c](gp_matrix* x) { destroy_matrix(c, x); };
  std::unique_ptr<gp_matrix, decltype(release)> s(new gp_matrix(), release);
  gp_matrix* m = s.get();
  m->ds = nullptr;  // a stacked matrix belongs to no single dataset
  m->prec = prec;
  m->n = tot.row;
  m->nnz = tot.nnz;
  m->n_long = tot.nlong;
  m->nD = tot.nD;
  m->utotal = tot.utotal;
  m->nm = tot.nm;
  m->ntiles = tot.tiles;
  m->nstiles = tot.stiles;
  m->npieces = tot.pieces;
  for (int r = 0; r < R; ++r) {
    m->max_row = std::max(m->max_row, ms[r]->max_row);
    m->nnz_group += ms[r]->nnz_group;
    m->gemv_stage += ms[r]->gemv_stage;
    m->gemm_stage += ms[r]->gemm_stage;
  }
  // allocations with the sizes destroy_matrix releases
  const int64_t n = m->n;
  m->row_ptr = dev_new<int64_t>(c, n + 1);
  m->col = dev_new<int32_t>(c, m->nnz + kCsrPad);
  m->val = dev_alloc(c, vbytes * (m->nnz + kCsrPad));
  m->diag = dev_new<double>(c, n);
  m->long_rows = dev_new<int32_t>(c, std::max<int64_t>(m->n_long, 1));
  m->gskip = dev_new<int32_t>(c, n);
  m->g_uoff = dev_new<int64_t>(c, m->nD + 1);
  m->g_ulist = dev_new<int32_t>(c, std::max<int64_t>(m->utotal, 1));
  m->g_rows = dev_new<int32_t>(c, std::max<int64_t>(m->nm, 1));
  m->g_tiles = dev_new<int32_t>(c, std::max<int64_t>(4 * (m->ntiles + m->nstiles + m->npieces), 4));
  m->bytes = sizeof(int64_t) * (n + 1) + (sizeof(int32_t) + vbytes) * (m->nnz + kCsrPad) + sizeof(double) * n +
             sizeof(int32_t) * (std::max<int64_t>(m->n_long, 1) + n + m->utotal + m->nm +
                                4 * (m->ntiles + m->nstiles + m->npieces)) +
             sizeof(int64_t) * (m->nD + 1);
  // quads: allocated before the table is filled (the sizes are known)
  m->ntrow = tot.trow;
  m->nquad = tot.quads;
  const int64_t ng = m->ntrow / 4;
  m->trow = dev_new<int32_t>(c, std::max<int64_t>(m->ntrow, 1));
  m->qptr = dev_new<int64_t>(c, ng + 1);
  m->qcol = dev_new<int32_t>(c, std::max<int64_t>(m->nquad, 1));
  m->qval = dev_alloc(c, vbytes * 4 * std::max<int64_t>(m->nquad, 1));
  m->bytes += sizeof(int32_t) * m->ntrow + sizeof(int64_t) * (ng + 1) + (sizeof(int32_t) + vbytes * 4) * m->nquad;
  if (block_jacobi) {
    m->nblk = tot.nblk;
    m->binv_len = tot.binv;
    m->bstart = dev_new<int32_t>(c, m->nblk + 1);
    m->rowblk = dev_new<int32_t>(c, n);
    m->boff = dev_new<int64_t>(c, m->nblk + 1);
    m->binv = dev_new<double>(c, std::max<int64_t>(m->binv_len, 1));
    m->bytes += sizeof(int32_t) * (m->nblk + 1 + n) + sizeof(int64_t) * (m->nblk + 1) + sizeof(double) * m->binv_len;
  }

  // the piece table: one run of R pieces per stacked array
  std::vector<Piece> tab;
  struct Run {
    size_t first;
    int64_t maxcount;
  };
  auto add_run = [&](auto piece_of) {
    Run run{tab.size(), 0};
    for (int r = 0; r < R; ++r) {
      Piece p = piece_of(r, ms[r], off[r]);
      run.maxcount = std::max(run.maxcount, p.count);
      tab.push_back(p);
    }
    return run;
  };
  auto P = [](const void* src, int64_t count, int64_t dst, int64_t a0 = 0, int64_t a1 = 0, int64_t a2 = 0,
              int64_t a3 = 0) { return Piece{src, count, dst, {a0, a1, a2, a3}}; };
  const Run r_rowptr = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->row_ptr, x->n, o.row, o.nnz); });
  const Run r_col = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->col, x->nnz, o.nnz, o.row); });
  const Run r_val = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->val, x->nnz, o.nnz); });
  const Run r_diag = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->diag, x->n, o.row); });
  const Run r_long =
      add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->long_rows, x->n_long, o.nlong, o.row); });
  const Run r_gskip = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->gskip, x->n, o.row); });
  const Run r_uoff = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->g_uoff, x->nD, o.nD, o.utotal); });
  const Run r_ulist =
      add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->g_ulist, x->utotal, o.utotal, o.row); });
  const Run r_grows = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->g_rows, x->nm, o.nm, o.row); });
  // tiles (mask, first group row, rows, 0); super-tiles (first group row,
  // rows, first piece, pieces); pieces (mask, first group row, rows, first U_M entry)
  const Run r_tiles = add_run([&](int, const gp_matrix* x, const Off& o) {
    return P(x->g_tiles, 4 * x->ntiles, 4 * o.tiles, o.nD, o.nm, 0, 0);
  });
  const Run r_stiles = add_run([&](int, const gp_matrix* x, const Off& o) {
    return P(x->g_tiles + 4 * x->ntiles, 4 * x->nstiles, 4 * (tot.tiles + o.stiles), o.nm, 0, o.pieces, 0);
  });
  const Run r_pieces = add_run([&](int, const gp_matrix* x, const Off& o) {
    return P(x->g_tiles + 4 * (x->ntiles + x->nstiles), 4 * x->npieces, 4 * (tot.tiles + tot.stiles + o.pieces), o.nD,
             o.nm, 0, 0);
  });
  const Run r_trow = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->trow, x->ntrow, o.trow, o.row); });
  const Run r_qptr =
      add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->qptr, x->ntrow / 4, o.trow / 4, o.quads); });
  const Run r_qcol = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->qcol, x->nquad, o.quads, o.row); });
  const Run r_qval = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->qval, 4 * x->nquad, 4 * o.quads); });
  Run r_bstart{}, r_rowblk{}, r_boff{}, r_binv{};
  if (block_jacobi) {
    r_bstart = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->bstart, x->nblk, o.nblk, o.row); });
    r_rowblk = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->rowblk, x->n, o.row, o.nblk); });
    r_boff = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->boff, x->nblk, o.nblk, o.binv); });
    r_binv = add_run([&](int, const gp_matrix* x, const Off& o) { return P(x->binv, x->binv_len, o.binv); });
  }
  TmpBuf dtab(c, sizeof(Piece) * tab.size());
  {
    Piece* h = static_cast<Piece*>(pinned_for_write(c, sizeof(Piece) * tab.size()));
    std::memcpy(h, tab.data(), sizeof(Piece) * tab.size());
    h2d_async(c, dtab.p, h, sizeof(Piece) * tab.size());
  }
  const Piece* dt = dtab.as<Piece>();
  auto launch = [&](auto kern, const Run& run, auto* out) {
    if (run.maxcount == 0) return;
    const unsigned gx = std::min<unsigned>(grid_for(run.maxcount, kThreads), 2048);
    hipLaunchKernelGGL(kern, dim3(gx, static_cast<unsigned>(R)), dim3(kThreads), 0, c->stream, dt + run.first, out);
  };
  launch(k_stack<int64_t, kShift>, r_rowptr, m->row_ptr);
  hipLaunchKernelGGL(k_put_i64, dim3(1), dim3(1), 0, c->stream, m->row_ptr + n, m->nnz);
  launch(k_stack<int32_t, kShift>, r_col, m->col);
  if (prec == GP_MIXED)
    launch(k_stack<float, kCopy>, r_val, static_cast<float*>(m->val));
  else
    launch(k_stack<double, kCopy>, r_val, static_cast<double*>(m->val));
  GPS_HIP(hipMemsetAsync(m->col + m->nnz, 0, sizeof(int32_t) * kCsrPad, c->stream));
  GPS_HIP(hipMemsetAsync(static_cast<char*>(m->val) + vbytes * m->nnz, 0, vbytes * kCsrPad, c->stream));
  launch(k_stack<double, kCopy>, r_diag, m->diag);
  launch(k_stack<int32_t, kShift>, r_long, m->long_rows);
  launch(k_stack<int32_t, kCopy>, r_gskip, m->gskip);
  launch(k_stack<int64_t, kShift>, r_uoff, m->g_uoff);
  hipLaunchKernelGGL(k_put_i64, dim3(1), dim3(1), 0, c->stream, m->g_uoff + m->nD, m->utotal);
  launch(k_stack<int32_t, kShift>, r_ulist, m->g_ulist);
  launch(k_stack<int32_t, kShift>, r_grows, m->g_rows);
  launch(k_stack<int32_t, kShift4>, r_tiles, m->g_tiles);
  launch(k_stack<int32_t, kShift4>, r_stiles, m->g_tiles);
  launch(k_stack<int32_t, kShift4>, r_pieces, m->g_tiles);
  launch(k_stack<int32_t, kRowCode>, r_trow, m->trow);
  launch(k_stack<int64_t, kShift>, r_qptr, m->qptr);
  hipLaunchKernelGGL(k_put_i64, dim3(1), dim3(1), 0, c->stream, m->qptr + ng, m->nquad);
  launch(k_stack<int32_t, kShift>, r_qcol, m->qcol);
  if (prec == GP_MIXED)
    launch(k_stack<float, kCopy>, r_qval, static_cast<float*>(m->qval));
  else
    launch(k_stack<double, kCopy>, r_qval, static_cast<double*>(m->qval));
  if (block_jacobi) {
    launch(k_stack<int32_t, kShift>, r_bstart, m->bstart);
    hipLaunchKernelGGL(k_put_i32, dim3(1), dim3(1), 0, c->stream, m->bstart + m->nblk, static_cast<int32_t>(n));
    launch(k_stack<int32_t, kShift>, r_rowblk, m->rowblk);
    launch(k_stack<int64_t, kShift>, r_boff, m->boff);
    hipLaunchKernelGGL(k_put_i64, dim3(1), dim3(1), 0, c->stream, m->boff + m->nblk, m->binv_len);
    launch(k_stack<double, kCopy>, r_binv, m->binv);
  }
  check_launch("stack matrices");
  sync(c);  // the piece table is released when this scope ends
  return s.release();
}

}  // namespace gps
