// Internal declarations of the gpsparse library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "../../include/gpsparse.h"

namespace gps {

constexpr int kWave = 64;
constexpr int kMaxGroups = 64;      // n1 <= 64: group membership is one uint64 per point
constexpr int kMaxBumps = 4096;     // n1 * n2
constexpr int kMaxBasis = 16;       // basis functions of the nonstationary core
constexpr int kLongRow = 128;       // rows longer than this get a wave of their own in SpMV
constexpr int64_t kCsrPad = 64;     // padding entries after the CSR column and value arrays
constexpr int kTileRows = 16;       // rows per tile of a group block
constexpr int kSuperRows = 64;      // rows per super-tile (multi-column products)
constexpr int kPiece = 256;         // U_M entries per block of a multi-column product

// ------------------------------------------------------------------ errors
struct Error {
  gp_status st;
  std::string msg;
};

#define GPS_HIP(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::gps::Error{GP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define GPS_REQUIRE(cond, code, text)                 \
  do {                                                \
    if (!(cond)) throw ::gps::Error{(code), (text)};  \
  } while (0)

inline void check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{GP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

inline unsigned grid_for(int64_t items, int per_block) {
  int64_t g = (items + per_block - 1) / per_block;
  return static_cast<unsigned>(g < 1 ? 1 : g);
}

// Work for the side stream handed over one unit at a time (see side_pump).
struct SideFeed {
  virtual ~SideFeed() = default;
  // enqueues the next unit on c->stream (the side stream while it runs);
  // false once the last unit has been enqueued
  virtual bool unit(gp_ctx* c) = 0;
};

}  // namespace gps

// ---------------------------------------------------------------- objects
struct gp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  gp_alloc_fn alloc = nullptr;
  gp_free_fn free_fn = nullptr;
  void* user = nullptr;
  std::string err;
  size_t in_use = 0, peak = 0;
  size_t budget = 0;  // 0: none
  // growable workspace slots, reused across calls on this context
  struct Slot {
    void* ptr = nullptr;
    size_t bytes = 0;
  };
  std::vector<Slot> slots;
  // pinned host staging for small device->host reads
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  int* err_flag = nullptr;  // device int, set by kernels on consistency failures
  bool h2d_pending = false;   // a host-to-device copy from the pinned buffer may not have run yet
  hipEvent_t ev_aux = nullptr;  // event for partial waits (created on first use)
  // optional per-kernel timing with events on the context's stream
  bool prof_on = false;
  struct ProfRec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof;
  std::vector<std::string> prof_only;  // names timed (empty: all)
  std::vector<hipEvent_t> evpool;
  size_t evnext = 0;
  // second stream for independent work of one call (the log det beside the
  // solve), created on first use; ordered against the main stream by events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool side_pending = false;  // work was forked to the side stream and not joined yet
  bool alloc_locked = false;  // set while work is enqueued on the side stream
  bool concurrent = true;     // the log det of a likelihood on the side stream
  // side-stream work not enqueued yet, and a ring of events marking the
  // completion of its latest units (side_pump)
  std::unique_ptr<gps::SideFeed> feed;
  std::vector<hipEvent_t> feed_ev;
  int64_t feed_issued = 0, feed_done = 0;
};

struct gp_dataset {
  int64_t n = 0;
  int d = 0;
  double lo[3] = {0, 0, 0};
  double cell[3] = {1, 1, 1};
  int32_t g[3] = {1, 1, 1};
  int64_t ncells = 1;
  double* xb = nullptr;         // d x n SoA, binned order
  int32_t* perm = nullptr;      // binned -> original
  int32_t* iperm = nullptr;     // original -> binned
  int32_t* key = nullptr;       // cell key of each binned point
  int32_t* cell_start = nullptr;// ncells + 1
  int32_t max_cell = 0;         // most points in one cell
  size_t bytes = 0;
};

struct gp_matrix {
  const gp_dataset* ds = nullptr;
  int64_t n = 0, nnz = 0, max_row = 0;
  int prec = GP_FP64;
  double nugget = 0;
  uint64_t theta_hash = 0;      // theta_hash() of the hyper-parameters assembled with
  int64_t* row_ptr = nullptr;   // n + 1
  int32_t* col = nullptr;       // nnz, binned column ids, ascending per row
  void* val = nullptr;          // nnz float or double
  double* diag = nullptr;       // n, diagonal of the stored matrix (float64)
  int32_t* long_rows = nullptr; // rows with more than kLongRow entries
  int64_t n_long = 0;
  // column offsets col - row as int16 for the CSR part (nnz + kCsrPad), built
  // on the first one-column product; null when an offset does not fit
  int16_t* col16 = nullptr;
  bool col16_tried = false;
  // row quads of the multi-column product, built on first use.  The rows
  // are listed along the grid axis with the most cells (a line: the cells
  // with every other cell coordinate fixed, one after another, binned order
  // within a cell) in segments of a few consecutive cells of a line, each
  // segment padded to a multiple of four rows (segments ordered by region of
  // lines, then position along the line, then line); quad q (listed rows
  // 4q .. 4q+3) holds the ascending union of its
  // rows' CSR-part columns (rows with more than kLongRow such entries left
  // out) with the four rows' values per column (0 where a row has none).
  int64_t ntrow = 0;             // listed rows (padded)
  // per listed row: -1 (padding, or a row with more than kLongRow entries
  // past its group part), the binned row (no group part) or -(row + 2)
  int32_t* trow = nullptr;
  int64_t nquad = 0;             // union entries over all quads
  int64_t* qptr = nullptr;       // ntrow / 4 + 1 offsets
  int32_t* qcol = nullptr;       // nquad column ids
  void* qval = nullptr;          // 4 * nquad float or double
  // rows with a bump-group mask start with the group entries of their mask
  // (|U_M| entries, shared column list U_M); the products treat these as dense
  // blocks (rows with mask M) x (columns U_M)
  int32_t* gskip = nullptr;     // n: number of leading group entries of each row
  int64_t nD = 0, utotal = 0, nm = 0, ntiles = 0, nstiles = 0, npieces = 0;
  int64_t nnz_group = 0;        // entries in the group blocks (sum of gskip)
  int64_t gemv_stage = 0;       // U_M entries staged by the one-column group product (sum over its tiles)
  int64_t gemm_stage = 0;       // U_M entries staged by the multi-column group product (sum over super-tiles)
  int64_t* g_uoff = nullptr;    // nD + 1 offsets into g_ulist
  int32_t* g_ulist = nullptr;   // concatenated U_M (binned column ids, ascending)
  int32_t* g_rows = nullptr;    // rows with a mask, grouped by mask
  // ntiles tiles of at most kTileRows rows, each (mask id, first index in
  // g_rows, rows, 0), largest (|U_M| x rows) first; then nstiles super-tiles of at most kSuperRows rows, each
  // (first index in g_rows, rows, first piece, pieces); then npieces pieces,
  // each (mask id, first index in g_rows, rows, first U_M entry): a piece is
  // a super-tile's rows times at most kPiece consecutive entries of U_M
  int32_t* g_tiles = nullptr;
  // block-Jacobi preconditioner, built on first use (blocks = binning cells)
  int64_t nblk = 0, binv_len = 0;
  int32_t* bstart = nullptr;    // nblk + 1 block starts (binned rows)
  int32_t* rowblk = nullptr;    // n, block of each row
  int64_t* boff = nullptr;      // nblk + 1 offsets into binv
  double* binv = nullptr;       // row-major inverses of the diagonal blocks
  size_t bytes = 0;
};

namespace gps {

// bump parameters as laid out for the kernels (64 bytes each)
struct Bump {
  double h[3];
  double inv[3];
  double a, b;
};

struct Grid {
  double lo[3];
  double inv_cell[3];   // unused by decisions on pattern membership
  double cell[3];
  int32_t g[3];
  int32_t R[3];         // neighbour rings per coordinate
};

// Per-theta point features (binned order).
struct Features {
  uint64_t* mask = nullptr;  // n
  int32_t* midx = nullptr;   // n, compact index of masked points or -1
  int32_t* mlist = nullptr;  // nm, binned ids of masked points (ascending)
  uint64_t* mmask = nullptr; // nm, their masks
  double* F = nullptr;       // nm x n1 values f_i
  int64_t nm = 0;
};

// Core kernel as the entry kernels use it: kind (GP_CORE_*), nu2, sigma0^2,
// 1 / ell; for the nonstationary core the per-point fields sigma(x_p) and
// Sigma(x_p) of the training points in binned order (device).
struct KernelCore {
  int kind, nu2;
  double s2;
  double inv_ell[3];
  const double* sig;
  const double* Sig;
};

// Parameters of the log-linear fields of the nonstationary core (Eq. PScov):
// log sigma = log sigma0 + sum_m s_m phi_s[m], log Sigma = log Sigma0 +
// sum_m s_m phi_S[m], s_m(x) = exp(-|(x - c[m]) / w|^2 / 2).
struct CoreBasis {
  int nb;
  double log_sigma0, log_Sigma0;
  double c[kMaxBasis][3];
  double w[3];
  double phi_s[kMaxBasis], phi_S[kMaxBasis];
};

struct KernelTheta {
  int d, n1, n2, variant;
  double s0, nugget;
  double inv0[3];
  const Bump* bumps;  // device, n1*n2
  KernelCore core;
  const double* tau2;  // device, per-point error variances in binned order, or null
};

// -------------------------------------------------------------- memory
void* dev_alloc(gp_ctx* c, size_t bytes);
void dev_free(gp_ctx* c, void* p, size_t bytes);
void* workspace(gp_ctx* c, int slot, size_t bytes);   // grows, never shrinks
// Pinned host staging.  pinned() is for device-to-host reads (the host reads
// after sync()); pinned_for_write() first waits for pending uploads from the
// buffer, and h2d_async() issues such an upload.
void* pinned(gp_ctx* c, size_t bytes);
void* pinned_for_write(gp_ctx* c, size_t bytes);
void h2d_async(gp_ctx* c, void* dst, const void* src, size_t bytes);
// record_aux() marks the current point of the context's stream; wait_aux()
// waits until the stream has reached it (work queued after the mark keeps
// running meanwhile)
void record_aux(gp_ctx* c);
void wait_aux(gp_ctx* c);
void sync(gp_ctx* c);
// Side stream: fork_side() orders the side stream after everything enqueued
// on the main stream so far; while a SideScope lives, the context's stream is
// the side stream and device allocations are refused (memory the side stream
// uses must be allocated before the fork, in the main stream's order);
// join_side() orders the main stream after the side stream's work.
void fork_side(gp_ctx* c);
void join_side(gp_ctx* c);
// A long side-stream sequence (the SLQ log det: several hundred launches) is
// not enqueued in one go: once the device queue is full the host blocks in
// the launch until the side stream has drained part of it, and the main
// stream's launches, issued after it, start late.  side_install() takes such
// work after fork_side() (its set-up already enqueued on the side stream);
// side_pump() keeps a few of its units in flight and is called from the main
// stream's host loops; join_side() enqueues the units still left before it
// joins.
void side_install(gp_ctx* c, std::unique_ptr<SideFeed> f);
void side_pump(gp_ctx* c);
struct SideScope {
  gp_ctx* c;
  hipStream_t main;
  explicit SideScope(gp_ctx* c_) : c(c_), main(c_->stream) {
    c->stream = c->side;
    c->alloc_locked = true;
  }
  ~SideScope() {
    c->stream = main;
    c->alloc_locked = false;
  }
  SideScope(const SideScope&) = delete;
  SideScope& operator=(const SideScope&) = delete;
};
// joins the side stream when it goes out of scope (also on an exception)
struct JoinGuard {
  gp_ctx* c;
  ~JoinGuard() {
    c->feed.reset();  // after an error: units not yet enqueued are dropped
    if (c->side_pending) {
      (void)hipEventRecord(c->ev_join, c->side);
      (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
      c->side_pending = false;
    }
  }
};

template <typename T>
T* dev_new(gp_ctx* c, size_t count) {
  return static_cast<T*>(dev_alloc(c, count * sizeof(T) > 0 ? count * sizeof(T) : 16));
}

// RAII holder for temporaries allocated from the context
struct TmpBuf {
  gp_ctx* c = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  TmpBuf() = default;
  TmpBuf(gp_ctx* c_, size_t b) : c(c_), p(dev_alloc(c_, b ? b : 16)), bytes(b ? b : 16) {}
  ~TmpBuf() {
    if (p) dev_free(c, p, bytes);
  }
  TmpBuf(const TmpBuf&) = delete;
  TmpBuf& operator=(const TmpBuf&) = delete;
  TmpBuf(TmpBuf&& o) noexcept : c(o.c), p(o.p), bytes(o.bytes) { o.p = nullptr; }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Brackets the launches issued in its scope with events when profiling is on.
hipEvent_t prof_event(gp_ctx* c);
struct ProfScope {
  gp_ctx* c;
  const char* name;
  hipEvent_t a = nullptr;
  ProfScope(gp_ctx* c_, const char* n) : c(c_), name(n) {
    if (c->prof_on && timed(n)) {
      a = prof_event(c);
      (void)hipEventRecord(a, c->stream);
    }
  }
  ~ProfScope() {
    if (c->prof_on && a) {
      hipEvent_t b = prof_event(c);
      (void)hipEventRecord(b, c->stream);
      c->prof.push_back({name, a, b});
    }
  }
  bool timed(const char* n) const {
    if (c->prof_only.empty()) return true;
    for (const std::string& o : c->prof_only)
      if (o == n) return true;
    return false;
  }
};

// -------------------------------------------------------------- scan
// out[i] = sum_{j<i} in[j] for i in [0, n]; out[n] = total.  Deterministic.
void scan_i32_to_i64(gp_ctx* c, const int32_t* in, int64_t* out, int64_t n);
void scan_i32_to_i32(gp_ctx* c, const int32_t* in, int32_t* out, int64_t n);
int64_t read_i64(gp_ctx* c, const int64_t* dev);   // synchronising read

// -------------------------------------------------------------- stages
void bin_dataset(gp_ctx* c, gp_dataset* ds, const double* x_dev, const double* cell);
void upload_theta(gp_ctx* c, const gp_theta* th, Bump** bumps_dev, KernelTheta* kt);
// Core parameters of theta (kind GP_CORE_NONE when theta has none); the field
// pointers of kc are left null.
void core_params(const gp_theta* th, KernelCore* kc, CoreBasis* cb);
// sigma(x_p), Sigma(x_p) of every binned point of ds (nonstationary core)
void core_fields(gp_ctx* c, const gp_dataset* ds, const CoreBasis& cb, double* sig, double* Sig);
void compute_features(gp_ctx* c, const gp_dataset* ds, const KernelTheta& kt, Features* f,
                      int ws_base);
Grid make_grid(const gp_dataset* ds, const gp_theta* th);
gp_matrix* assemble(gp_ctx* c, const gp_dataset* ds, const gp_theta* th, int prec);
void destroy_matrix(gp_ctx* c, gp_matrix* m);
void export_csr(gp_ctx* c, const gp_matrix* m, int64_t* row_ptr, int32_t* col, double* val);

// SpMV / SpMM in binned order.
// y = K x (float64 x and y; float32 or float64 values; float64 accumulation)
// skip (device int or null): when it holds a nonzero value at run time the
// product's kernels return at once (device-side control of the solvers)
void spmv_f64(gp_ctx* c, const gp_matrix* m, const double* x, double* y, const int* skip = nullptr);
// builds the caches the products read (int16 offsets, row quads) now, with
// host synchronisations, so that later products need none
void build_product_caches(gp_ctx* c, gp_matrix* m);
// allocates the work space of a 32-column product of m
void spmm_reserve(gp_ctx* c, const gp_matrix* m);
// Block-diagonal stack of R assembled matrices of one precision, whose product
// caches (and block-Jacobi blocks, when block_jacobi) are built: a new matrix
// with no dataset, row r of problem q at stacked row (rows of problems < q) + r.
gp_matrix* stack_matrices(gp_ctx* c, int R, const gp_matrix* const* ms, bool block_jacobi);
// the same product using only the caches already built (no allocation, no
// synchronisation, no profiling events)
void spmv_f64_enqueue(gp_ctx* c, const gp_matrix* m, const double* x, double* y);
// Y = S K S X D for k columns, X/Y n x ld row-major (S = diag(scale) or identity
// if null; D = diag(colscale), a device array of k values, or identity if null).
// share: the product runs beside another stream's kernels and holds fewer
// wave slots per CU, so that they find room (same results).
template <typename T>
void spmm(gp_ctx* c, const gp_matrix* m, int k, int ld, const T* X, T* Y, const T* scale,
          const double* colscale = nullptr, bool share = false);

// original <-> binned order for n x k row-major blocks
template <typename T>
void permute_to_binned(gp_ctx* c, const gp_dataset* ds, int k, const T* x, T* xb);
template <typename T>
void permute_to_orig(gp_ctx* c, const gp_dataset* ds, int k, const T* yb, T* y);

// ----------------------------------------------------------- Krylov drivers
struct SolveResult {
  int iters = 0;
  int refreshes = 0;
  double relres = 0;
  double quad = 0;
  gp_status st = GP_OK;
};
// alpha = K^-1 y (binned order); preconditioned CG with float64 vectors and
// products on the stored values (float32 for a GP_MIXED matrix).
SolveResult pcg_solve(gp_ctx* c, gp_matrix* m, const double* yb, double* xb, double rtol, int max_iter, int precond);
// alpha = K^-1 y by preconditioned MINRES (float64 products on the stored
// values); warm: start from the x passed in, else from 0.
// diag C_{y|z} at ntest test points (xs: ntest x d row-major, device; var:
// ntest doubles, device), 32 test points per batch
struct VarResult {
  int iters = 0;
  int max_batch_iters = 0;
  double relres = 0;
  gp_status st = GP_OK;
};
VarResult predict_variance(gp_ctx* c, const gp_matrix* m, const gp_theta* th, int64_t ntest, const double* xs,
                           double rtol, int max_iter, int precond, double* var);
// y = z - W beta (W: n x p column-major, device; beta: p values, host)
void mean_residual(gp_ctx* c, int64_t n, int p, const double* W, const double* beta_host, const double* z,
                   double* y);
// fingerprint of every hyper-parameter of theta (FNV-1a over their bits)
uint64_t theta_hash(const gp_theta* th);
SolveResult minres_solve(gp_ctx* c, gp_matrix* m, const double* yb, double* xb, bool warm, double rtol, int max_iter,
                         int precond);
void build_block_jacobi(gp_ctx* c, gp_matrix* m);
void free_quads(gp_ctx* c, gp_matrix* m);
void free_col16(gp_ctx* c, gp_matrix* m);
void free_block_jacobi(gp_ctx* c, gp_matrix* m);

struct LogdetResult {
  double logdet = 0, se = 0;
  int steps = 0;
  gp_status st = GP_OK;
};
// reorth: full re-orthogonalisation against every Lanczos block (work space
// n_steps x n x 32 float64)
LogdetResult slq_logdet(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, bool reorth);
LogdetResult exact_logdet(gp_ctx* c, const gp_matrix* m, uint64_t seed);

// allocation-free one-column product (fixed per-device scratch array)
void noalloc_init(int device);   // once per device, with the device current
size_t noalloc_scratch_bytes();
void matvec_noalloc(gp_ctx* c, const gp_matrix* m, const double* x, double* y);

// Device-driven forms (no host read before the end; used by gp_loglik_async).
// pcg_solve_device enqueues the conjugate gradients up to max_iter with
// every decision taken on the device; its results stay in device memory, at
// the addresses it returns.  The matrix's caches must be built already.
// Control state of a device-driven conjugate-gradient solve (one per problem
// of a batch), in device memory.
struct CgCtl {
  int skip_iter;    // nonzero: the iterations are over (converged or failed)
  int skip_true;    // nonzero: no true-residual pass after this block
  int skip_final;   // nonzero: no final true residual (converged, or y = 0)
  int iters, refreshes, status;
  double target;    // rtol |y|_2 (compared with |r|_2 as the host form does)
  double relres;
};
// the flags every problem of a batch shares (all problems' flags set)
struct CtlAll {
  int skip_iter, skip_true, skip_final;
};
// results of a device-driven solve of R problems: quad[r], ctl[r]
struct DeviceSolve {
  const double* quad;
  const CgCtl* ctl;
};
void pcg_solve_device(gp_ctx* c, gp_matrix* m, const double* yb, double* xb, double rtol, int max_iter, int precond,
                      DeviceSolve* out);
// R problems stacked along the rows of m (a block-diagonal matrix; off: R + 1
// device row offsets, nmax the longest problem), each solved as
// pcg_solve_device would solve it alone; the host checks after every block
// of iterations whether all have ended.
void pcg_solve_batch(gp_ctx* c, gp_matrix* m, const double* yb, double* xb, double rtol, int max_iter, int precond,
                     int R, const int64_t* off, int64_t nmax, DeviceSolve* out);
struct DeviceLogdet {
  double logdet, se;
  int steps, status;
};
// writes the SLQ estimate into out (device memory)
void slq_logdet_device(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, bool reorth,
                       DeviceLogdet* out);
// the same on the side stream beside the main stream's work: forks, enqueues
// the set-up and hands the Lanczos steps to side_install (one unit per step)
void slq_logdet_side(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, bool reorth,
                     DeviceLogdet* out);
// allocates (in the main stream's order) the work space slq_logdet_device and
// slq_logdet_batch (R problems of n stacked rows) will use, so that they can
// be enqueued on the side stream without allocating
void slq_reserve(gp_ctx* c, const gp_matrix* m, int n_probes, int n_steps, bool reorth, int R = 1);
// R problems stacked along the rows of m, each estimated as slq_logdet_device
// would estimate it alone (same probes, keyed by the problem's own original
// indices); out[r] per problem
struct SlqBatch {
  int R = 0;
  const int64_t* off = nullptr;   // R + 1 device row offsets
  const double* inv0 = nullptr;   // R device values 1 / sqrt(n_r)
  const int32_t* perm = nullptr;  // stacked rows -> the problem's original index
  int64_t nmax = 0;               // rows of the longest problem
};
void slq_logdet_batch(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, const SlqBatch& b,
                      DeviceLogdet* out);
// the batch estimate on the side stream (as slq_logdet_side; b is copied, the
// device arrays it points to must live until the join)
void slq_batch_side(gp_ctx* c, const gp_matrix* m, uint64_t seed, int n_probes, int n_steps, const SlqBatch& b,
                    DeviceLogdet* out);

// deterministic reductions
double dot_f64(gp_ctx* c, const double* a, const double* b, int64_t n);   // synchronising

}  // namespace gps
