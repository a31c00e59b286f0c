// C ABI entry points: validation, object lifetime, memory, and orchestration.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>

#include "internal.hpp"

namespace gps {
gp_predictor* make_predictor(gp_ctx* c, const gp_dataset* ds, const gp_theta* th, const double* alpha);
void destroy_predictor(gp_ctx* c, gp_predictor* p);
void predict(gp_ctx* c, const gp_predictor* p, int64_t m, const double* xs, int prec, double* out);
void predict_batch(gp_ctx* c, int32_t nreq, const gp_predictor* const* preds, const int64_t* roff_host,
                   const double* xs, int prec, double* out);

// ------------------------------------------------------------------ memory
void* dev_alloc(gp_ctx* c, size_t bytes) {
  if (c->alloc_locked) throw Error{GP_EDEVICE, "internal: device allocation while enqueueing on the side stream"};
  if (bytes == 0) bytes = 16;
  if (c->budget && bytes > c->budget - std::min(c->budget, c->in_use))
    throw Error{GP_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes exceeds the context's HBM budget (" +
                               std::to_string(c->in_use) + " of " + std::to_string(c->budget) + " bytes in use)"};
  void* p = nullptr;
  if (c->alloc) {
    p = c->alloc(bytes, c->user);
  } else {
    if (hipMallocAsync(&p, bytes, c->stream) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
  }
  if (!p) throw Error{GP_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
  c->in_use += bytes;
  c->peak = std::max(c->peak, c->in_use);
  return p;
}

void dev_free(gp_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  if (bytes == 0) bytes = 16;
  if (c->free_fn)
    c->free_fn(p, bytes, c->user);
  else
    (void)hipFreeAsync(p, c->stream);
  c->in_use -= std::min(c->in_use, bytes);
}

void* workspace(gp_ctx* c, int slot, size_t bytes) {
  if (static_cast<size_t>(slot) >= c->slots.size()) c->slots.resize(slot + 1);
  gp_ctx::Slot& s = c->slots[slot];
  if (s.bytes < bytes || !s.ptr) {
    if (s.ptr) dev_free(c, s.ptr, s.bytes);
    s.ptr = nullptr;
    const size_t want = std::max<size_t>(bytes + bytes / 4, 256);
    s.ptr = dev_alloc(c, want);
    s.bytes = want;
  }
  return s.ptr;
}

void* pinned(gp_ctx* c, size_t bytes) {
  if (bytes > c->pinned_bytes) {
    // earlier asynchronous copies may still use the old buffer
    sync(c);
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    const size_t want = std::max<size_t>(bytes, 1 << 20);
    GPS_HIP(hipHostMalloc(&c->pinned, want, hipHostMallocDefault));
    c->pinned_bytes = want;
  }
  return c->pinned;
}

void sync(gp_ctx* c) {
  GPS_HIP(hipStreamSynchronize(c->stream));
  c->h2d_pending = false;
}

void* pinned_for_write(gp_ctx* c, size_t bytes) {
  if (c->h2d_pending) sync(c);
  return pinned(c, bytes);
}

void record_aux(gp_ctx* c) {
  if (!c->ev_aux) GPS_HIP(hipEventCreateWithFlags(&c->ev_aux, hipEventDisableTiming));
  GPS_HIP(hipEventRecord(c->ev_aux, c->stream));
}

void wait_aux(gp_ctx* c) { GPS_HIP(hipEventSynchronize(c->ev_aux)); }

void fork_side(gp_ctx* c) {
  if (!c->side) {
    GPS_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    GPS_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    GPS_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  }
  GPS_HIP(hipEventRecord(c->ev_fork, c->stream));
  GPS_HIP(hipStreamWaitEvent(c->side, c->ev_fork, 0));
  c->side_pending = true;
}

// units of side-stream work in flight at most; a unit of the SLQ log det is
// one Lanczos step (about a millisecond at n = 10^6), so this covers the
// main stream's host waits between its pumps
constexpr int kSideAhead = 6;

void side_install(gp_ctx* c, std::unique_ptr<SideFeed> f) {
  GPS_REQUIRE(c->side_pending && !c->feed, GP_EDEVICE, "internal: side work installed twice");
  c->feed = std::move(f);
  c->feed_issued = c->feed_done = 0;
  side_pump(c);
}

void side_pump(gp_ctx* c) {
  if (!c->feed) return;
  if (c->feed_ev.empty()) {
    c->feed_ev.resize(kSideAhead + 1, nullptr);
    for (hipEvent_t& e : c->feed_ev) GPS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  const int64_t ring = static_cast<int64_t>(c->feed_ev.size());
  while (c->feed_done < c->feed_issued) {
    const hipError_t q = hipEventQuery(c->feed_ev[c->feed_done % ring]);
    if (q == hipErrorNotReady) break;
    GPS_HIP(q);
    ++c->feed_done;
  }
  // an event slot is recorded again only after its previous unit has completed
  while (c->feed && c->feed_issued - c->feed_done < kSideAhead) {
    bool more;
    {
      SideScope side(c);
      more = c->feed->unit(c);
      GPS_HIP(hipEventRecord(c->feed_ev[c->feed_issued % ring], c->stream));
    }
    ++c->feed_issued;
    if (!more) c->feed.reset();
  }
}

void join_side(gp_ctx* c) {
  if (!c->side_pending) return;
  while (c->feed) {  // the units not enqueued yet
    bool more;
    {
      SideScope side(c);
      more = c->feed->unit(c);
    }
    if (!more) c->feed.reset();
  }
  GPS_HIP(hipEventRecord(c->ev_join, c->side));
  GPS_HIP(hipStreamWaitEvent(c->stream, c->ev_join, 0));
  c->side_pending = false;
}

void h2d_async(gp_ctx* c, void* dst, const void* src, size_t bytes) {
  GPS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  c->h2d_pending = true;
}

hipEvent_t prof_event(gp_ctx* c) {
  if (c->evnext == c->evpool.size()) {
    hipEvent_t e;
    GPS_HIP(hipEventCreate(&e));
    c->evpool.push_back(e);
  }
  return c->evpool[c->evnext++];
}

}  // namespace gps

using gps::Error;

namespace {

template <typename F>
gp_status guarded(gp_ctx* c, F&& f) {
  try {
    if (c) {
      c->err.clear();
      GPS_HIP(hipSetDevice(c->device));
    }
    f();
    return GP_OK;
  } catch (const Error& e) {
    if (c) c->err = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    if (c) c->err = "host allocation failed";
    return GP_ENOMEM;
  } catch (...) {
    if (c) c->err = "unexpected internal error";
    return GP_EDEVICE;
  }
}

void validate_theta(const gp_theta* th, int d) {
  GPS_REQUIRE(th != nullptr, GP_EINVAL, "theta is NULL");
  GPS_REQUIRE(th->d == d, GP_EINVAL, "theta.d does not match the dataset");
  GPS_REQUIRE(th->n1 >= 0 && th->n1 <= gps::kMaxGroups, GP_EINVAL, "theta.n1 must be in 0..64");
  GPS_REQUIRE(th->n2 >= 0 && static_cast<int64_t>(th->n1) * th->n2 <= gps::kMaxBumps, GP_EINVAL,
              "theta.n1 * theta.n2 must be <= 4096");
  GPS_REQUIRE(th->wendland_variant == 0 || th->wendland_variant == 1, GP_EINVAL, "wendland_variant must be 0 or 1");
  GPS_REQUIRE(std::isfinite(th->s0) && th->s0 > 0, GP_EINVAL, "s0 must be finite and > 0");
  GPS_REQUIRE(std::isfinite(th->nugget) && th->nugget >= 0, GP_EINVAL, "nugget must be finite and >= 0");
  for (int k = 0; k < d; ++k)
    GPS_REQUIRE(std::isfinite(th->r0[k]) && th->r0[k] > 0, GP_EINVAL, "r0 must be finite and > 0");
  const int nb = th->n1 * th->n2;
  if (nb > 0) {
    GPS_REQUIRE(th->h && th->r && th->a && th->b, GP_EINVAL, "bump arrays must not be NULL");
    for (int i = 0; i < nb * d; ++i) {
      GPS_REQUIRE(std::isfinite(th->h[i]), GP_EINVAL, "bump centres must be finite");
      GPS_REQUIRE(th->r[i] > 0 && !std::isnan(th->r[i]), GP_EINVAL, "bump radii must be > 0 (+inf allowed)");
    }
    for (int i = 0; i < nb; ++i) {
      GPS_REQUIRE(std::isfinite(th->a[i]) && th->a[i] >= 0, GP_EINVAL, "bump amplitudes must be finite and >= 0");
      GPS_REQUIRE(std::isfinite(th->b[i]) && th->b[i] > 0, GP_EINVAL, "bump shapes must be finite and > 0");
    }
  }
  const gp_core* co = th->core;
  if (co && co->kind != GP_CORE_NONE) {
    auto pos = [](double v) { return std::isfinite(v) && v > 0; };
    GPS_REQUIRE(co->kind == GP_CORE_MATERN || co->kind == GP_CORE_PACIOREK, GP_EINVAL,
                "core.kind must be GP_CORE_NONE, GP_CORE_MATERN or GP_CORE_PACIOREK");
    GPS_REQUIRE(co->nu2 == 0 || co->nu2 == 1 || co->nu2 == 3 || co->nu2 == 5, GP_EINVAL, "core.nu2 must be 0, 1, 3 or 5");
    GPS_REQUIRE(pos(co->sigma0), GP_EINVAL, "core.sigma0 must be finite and > 0");
    for (int k = 0; k < d; ++k) GPS_REQUIRE(pos(co->ell[k]), GP_EINVAL, "core.ell must be finite and > 0");
    if (co->kind == GP_CORE_PACIOREK) {
      GPS_REQUIRE(pos(co->Sigma0), GP_EINVAL, "core.Sigma0 must be finite and > 0");
      GPS_REQUIRE(co->n_basis >= 0 && co->n_basis <= gps::kMaxBasis, GP_EINVAL, "core.n_basis must be in 0..16");
      for (int k = 0; k < d; ++k) GPS_REQUIRE(pos(co->width[k]), GP_EINVAL, "core.width must be finite and > 0");
      if (co->n_basis > 0) {
        GPS_REQUIRE(co->centers && co->phi_sigma && co->phi_Sigma, GP_EINVAL, "core basis arrays must not be NULL");
        for (int i = 0; i < co->n_basis * d; ++i)
          GPS_REQUIRE(std::isfinite(co->centers[i]), GP_EINVAL, "core.centers must be finite");
        for (int i = 0; i < co->n_basis; ++i)
          GPS_REQUIRE(std::isfinite(co->phi_sigma[i]) && std::isfinite(co->phi_Sigma[i]), GP_EINVAL,
                      "core basis coefficients must be finite");
      }
    }
  }
}

gp_solve_opts fill_opts(const gp_solve_opts* o) {
  gp_solve_opts d;
  gp_solve_opts_default(&d);
  if (!o) return d;
  gp_solve_opts r = *o;
  GPS_REQUIRE(std::isfinite(r.rtol) && r.rtol > 0 && r.rtol < 1, GP_EINVAL, "rtol must be in (0, 1)");
  GPS_REQUIRE(r.max_iter >= 1, GP_EINVAL, "max_iter must be >= 1");
  GPS_REQUIRE(r.n_probes >= 2 && r.n_probes <= 64, GP_EINVAL, "n_probes must be in 2..64");
  GPS_REQUIRE(r.n_lanczos >= 1 && r.n_lanczos <= 128, GP_EINVAL, "n_lanczos must be in 1..128");
  GPS_REQUIRE(r.logdet_mode >= 0 && r.logdet_mode <= 3, GP_EINVAL, "logdet_mode must be 0, 1, 2 or 3");
  GPS_REQUIRE(r.precond == GP_PRECOND_JACOBI || r.precond == GP_PRECOND_BLOCK_JACOBI, GP_EINVAL,
              "precond must be GP_PRECOND_JACOBI or GP_PRECOND_BLOCK_JACOBI");
  GPS_REQUIRE(r.solver >= GP_SOLVER_CG && r.solver <= GP_SOLVER_AUTO, GP_EINVAL,
              "solver must be GP_SOLVER_CG, GP_SOLVER_MINRES or GP_SOLVER_AUTO");
  return r;
}

}  // namespace

extern "C" {

void gp_solve_opts_default(gp_solve_opts* o) {
  if (!o) return;
  o->rtol = 1e-10;
  o->max_iter = 10000;
  o->n_probes = 30;
  o->n_lanczos = 50;
  o->logdet_mode = GP_LOGDET_SLQ;
  o->precond = GP_PRECOND_BLOCK_JACOBI;
  o->solver = GP_SOLVER_AUTO;
  o->seed = 0x5eed;
}

gp_status gp_ctx_create(int device, void* stream, gp_alloc_fn alloc, gp_free_fn free_fn, void* user, gp_ctx** out) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr)) return GP_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GP_EINVAL;
  std::unique_ptr<gp_ctx> c(new gp_ctx());
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  c->alloc = alloc;
  c->free_fn = free_fn;
  c->user = user;
  gp_status st = guarded(c.get(), [&] {
    if (!alloc) {
      hipMemPool_t pool;
      if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t thr = std::numeric_limits<uint64_t>::max();
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
      }
    }
    c->err_flag = static_cast<int*>(gps::dev_alloc(c.get(), sizeof(int) * 4));
    gps::pinned(c.get(), 1 << 20);
    gps::noalloc_init(device);
  });
  if (st != GP_OK) return st;
  *out = c.release();
  return GP_OK;
}

gp_status gp_ctx_destroy(gp_ctx* c) {
  if (!c) return GP_OK;
  gp_status st = guarded(c, [&] {
    for (auto& s : c->slots)
      if (s.ptr) gps::dev_free(c, s.ptr, s.bytes);
    c->slots.clear();
    if (c->err_flag) gps::dev_free(c, c->err_flag, sizeof(int) * 4);
    c->err_flag = nullptr;
    gps::sync(c);
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
    if (c->ev_aux) (void)hipEventDestroy(c->ev_aux);
    c->evpool.clear();
    c->feed.reset();
    if (c->side) {
      (void)hipStreamSynchronize(c->side);
      (void)hipStreamDestroy(c->side);
      (void)hipEventDestroy(c->ev_fork);
      (void)hipEventDestroy(c->ev_join);
    }
    for (hipEvent_t e : c->feed_ev) (void)hipEventDestroy(e);
    c->feed_ev.clear();
  });
  delete c;
  return st;
}

gp_status gp_ctx_set_stream(gp_ctx* c, void* stream) {
  if (!c) return GP_EINVAL;
  return guarded(c, [&] {
    gps::sync(c);
    c->stream = static_cast<hipStream_t>(stream);
  });
}

gp_status gp_profile_enable(gp_ctx* c, int32_t on) {
  if (!c) return GP_EINVAL;
  return guarded(c, [&] {
    gps::sync(c);
    c->prof.clear();
    c->evnext = 0;
    c->prof_on = on != 0;
  });
}

gp_status gp_profile_only(gp_ctx* c, const char* names) {
  if (!c) return GP_EINVAL;
  std::vector<std::string> v;
  if (names) {
    std::string cur;
    for (const char* q = names;; ++q) {
      if (*q == ',' || *q == '\0') {
        if (cur.size() > 31) return GP_EINVAL;
        if (!cur.empty()) v.push_back(cur);
        cur.clear();
        if (*q == '\0') break;
      } else {
        cur.push_back(*q);
      }
    }
  }
  c->prof_only = std::move(v);
  return GP_OK;
}

gp_status gp_profile_read(gp_ctx* c, int32_t max_entries, gp_profile_entry* out, int32_t* n_out) {
  if (!c || !n_out || (max_entries > 0 && !out)) return GP_EINVAL;
  return guarded(c, [&] {
    gps::sync(c);
    std::vector<gp_profile_entry> agg;
    for (const auto& r : c->prof) {
      float ms = 0;
      GPS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      auto it = std::find_if(agg.begin(), agg.end(),
                             [&](const gp_profile_entry& e) { return std::strncmp(e.name, r.name, 31) == 0; });
      if (it == agg.end()) {
        gp_profile_entry e{};
        std::strncpy(e.name, r.name, 31);
        agg.push_back(e);
        it = agg.end() - 1;
      }
      it->count += 1;
      it->total_ms += ms;
    }
    *n_out = static_cast<int32_t>(agg.size());
    for (int32_t i = 0; i < std::min<int32_t>(max_entries, static_cast<int32_t>(agg.size())); ++i) out[i] = agg[i];
  });
}

const char* gp_last_error(const gp_ctx* c) { return c ? c->err.c_str() : "context is NULL"; }

gp_status gp_ctx_set_concurrency(gp_ctx* c, int32_t on) {
  if (!c || (on != 0 && on != 1)) return GP_EINVAL;
  c->concurrent = on == 1;
  return GP_OK;
}

gp_status gp_ctx_set_hbm_budget(gp_ctx* c, size_t bytes) {
  if (!c) return GP_EINVAL;
  c->budget = bytes;
  return GP_OK;
}

gp_status gp_ctx_memory(const gp_ctx* c, size_t* in_use, size_t* peak) {
  if (!c) return GP_EINVAL;
  if (in_use) *in_use = c->in_use;
  if (peak) *peak = c->peak;
  return GP_OK;
}

gp_status gp_dataset_create(gp_ctx* c, int64_t n, int32_t d, const double* x_dev, const double* cell,
                            gp_dataset** out) {
  if (!c || !out) return GP_EINVAL;
  *out = nullptr;
  return guarded(c, [&] {
    GPS_REQUIRE(n >= 1 && n < (int64_t(1) << 31) - 1, GP_EINVAL, "gp_dataset_create: n must be in 1..2^31-2");
    GPS_REQUIRE(d >= 1 && d <= 3, GP_EINVAL, "gp_dataset_create: d must be 1, 2 or 3");
    GPS_REQUIRE(x_dev != nullptr, GP_EINVAL, "gp_dataset_create: x is NULL");
    std::unique_ptr<gp_dataset> ds(new gp_dataset());
    ds->n = n;
    ds->d = d;
    try {
      gps::bin_dataset(c, ds.get(), x_dev, cell);
    } catch (...) {
      gps::dev_free(c, ds->xb, sizeof(double) * d * n);
      gps::dev_free(c, ds->perm, sizeof(int32_t) * n);
      gps::dev_free(c, ds->iperm, sizeof(int32_t) * n);
      gps::dev_free(c, ds->key, sizeof(int32_t) * n);
      gps::dev_free(c, ds->cell_start, sizeof(int32_t) * (ds->ncells + 1));
      throw;
    }
    *out = ds.release();
  });
}

gp_status gp_dataset_destroy(gp_ctx* c, gp_dataset* ds) {
  if (!c) return GP_EINVAL;
  if (!ds) return GP_OK;
  gp_status st = guarded(c, [&] {
    const int64_t n = ds->n;
    gps::dev_free(c, ds->xb, sizeof(double) * ds->d * n);
    gps::dev_free(c, ds->perm, sizeof(int32_t) * n);
    gps::dev_free(c, ds->iperm, sizeof(int32_t) * n);
    gps::dev_free(c, ds->key, sizeof(int32_t) * n);
    gps::dev_free(c, ds->cell_start, sizeof(int32_t) * (ds->ncells + 1));
  });
  delete ds;
  return st;
}

gp_status gp_dataset_info(const gp_dataset* ds, int64_t* n, int32_t* d, int64_t* n_cells, double* cell_out) {
  if (!ds) return GP_EINVAL;
  if (n) *n = ds->n;
  if (d) *d = ds->d;
  if (n_cells) *n_cells = ds->ncells;
  if (cell_out)
    for (int k = 0; k < ds->d; ++k) cell_out[k] = ds->cell[k];
  return GP_OK;
}

gp_status gp_dataset_permutation(gp_ctx* c, const gp_dataset* ds, int32_t* perm_dev) {
  if (!c || !ds || !perm_dev) return GP_EINVAL;
  return guarded(c, [&] {
    GPS_HIP(hipMemcpyAsync(perm_dev, ds->perm, sizeof(int32_t) * ds->n, hipMemcpyDeviceToDevice, c->stream));
    gps::sync(c);
  });
}

gp_status gp_assemble(gp_ctx* c, const gp_dataset* ds, const gp_theta* th, gp_precision prec, gp_matrix** out) {
  if (!c || !out) return GP_EINVAL;
  *out = nullptr;
  return guarded(c, [&] {
    GPS_REQUIRE(ds != nullptr, GP_EINVAL, "gp_assemble: dataset is NULL");
    GPS_REQUIRE(prec == GP_FP64 || prec == GP_MIXED, GP_EINVAL, "gp_assemble: unknown precision");
    validate_theta(th, ds->d);
    *out = gps::assemble(c, ds, th, prec);
  });
}

gp_status gp_matrix_destroy(gp_ctx* c, gp_matrix* m) {
  if (!c) return GP_EINVAL;
  if (!m) return GP_OK;
  return guarded(c, [&] { gps::destroy_matrix(c, m); });
}

gp_status gp_matrix_info(const gp_matrix* m, int64_t* n, int64_t* nnz, size_t* bytes, int32_t* prec,
                         int64_t* max_row) {
  if (!m) return GP_EINVAL;
  if (n) *n = m->n;
  if (nnz) *nnz = m->nnz;
  if (bytes) *bytes = m->bytes;
  if (prec) *prec = m->prec;
  if (max_row) *max_row = m->max_row;
  return GP_OK;
}

gp_status gp_matrix_layout(const gp_matrix* m, gp_matrix_layout_info* out) {
  if (!m || !out) return GP_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->nnz_group = m->nnz_group;
  out->nnz_csr = m->nnz - m->nnz_group;
  out->group_rows = m->nm;
  out->group_masks = m->nD;
  out->group_list_entries = m->utotal;
  out->gemv_stage_entries = m->gemv_stage;
  out->gemm_stage_entries = m->gemm_stage;
  out->long_rows = m->n_long;
  out->col16 = m->col16 ? 1 : 0;
  out->listed_rows = m->ntrow;
  out->quad_entries = m->nquad;
  return GP_OK;
}

gp_status gp_matrix_export_csr(gp_ctx* c, const gp_matrix* m, int64_t* row_ptr, int32_t* col, double* val) {
  if (!c || !m || !row_ptr || !col || !val) return GP_EINVAL;
  return guarded(c, [&] { gps::export_csr(c, m, row_ptr, col, val); });
}

gp_status gp_matvec(gp_ctx* c, const gp_matrix* m, int32_t nrhs, const double* x, double* y) {
  if (!c || !m || !x || !y) return GP_EINVAL;
  return guarded(c, [&] {
    GPS_REQUIRE(nrhs >= 1 && nrhs <= 32, GP_EINVAL, "gp_matvec: nrhs must be in 1..32");
    const int64_t n = m->n;
    double* xb = static_cast<double*>(gps::workspace(c, 42, sizeof(double) * n * nrhs));
    double* yb = static_cast<double*>(gps::workspace(c, 43, sizeof(double) * n * nrhs));
    gps::permute_to_binned<double>(c, m->ds, nrhs, x, xb);
    if (nrhs == 1)
      gps::spmv_f64(c, m, xb, yb);
    else
      gps::spmm<double>(c, m, nrhs, nrhs, xb, yb, nullptr);
    gps::permute_to_orig<double>(c, m->ds, nrhs, yb, y);
    gps::sync(c);
  });
}

gp_status gp_matvec_noalloc(gp_ctx* c, const gp_matrix* m, const double* x, double* y) {
  if (!c || !m || !x || !y) return GP_EINVAL;
  return guarded(c, [&] { gps::matvec_noalloc(c, m, x, y); });
}

static gp_status loglik_common(gp_ctx* c, const gp_matrix* m, const double* y, const gp_solve_opts* opts,
                               double* alpha, gp_loglik_result* out, bool with_logdet) {
  if (!c || !m || !y || !out) return GP_EINVAL;
  std::memset(out, 0, sizeof(*out));
  gp_status solve_status = GP_OK;
  gp_status st = guarded(c, [&] {
    const gp_solve_opts o = fill_opts(opts);
    const int64_t n = m->n;
    double* yb = static_cast<double*>(gps::workspace(c, 44, sizeof(double) * n));
    double* xb = static_cast<double*>(gps::workspace(c, 45, sizeof(double) * n));
    gps::permute_to_binned<double>(c, m->ds, 1, y, yb);
    // the preconditioner is cached in the matrix object on first use
    gp_matrix* mm = const_cast<gp_matrix*>(m);
    // The SLQ log det does not depend on the solve: it is enqueued first on
    // the side stream (its device-driven form, nothing read back until the
    // end) and runs beside the solver's launches; the solve's host checks
    // wait on the main stream only.
    const bool slq = with_logdet && (o.logdet_mode == GP_LOGDET_SLQ || o.logdet_mode == GP_LOGDET_SLQ_REORTH);
    const bool reorth = o.logdet_mode == GP_LOGDET_SLQ_REORTH;
    gps::JoinGuard join{c};
    gps::DeviceLogdet* dld = nullptr;
    if (slq) {
      gps::build_product_caches(c, mm);
      gps::slq_reserve(c, m, o.n_probes, o.n_lanczos, reorth);
      dld = static_cast<gps::DeviceLogdet*>(gps::workspace(c, 126, sizeof(gps::DeviceLogdet)));
      if (c->concurrent) gps::slq_logdet_side(c, m, o.seed, o.n_probes, o.n_lanczos, reorth, dld);
    }
    gps::SolveResult sr;
    if (o.solver != GP_SOLVER_MINRES) {
      sr = gps::pcg_solve(c, mm, yb, xb, o.rtol, o.max_iter, o.precond);
      out->cg_iters = sr.iters;
      out->refreshes = sr.refreshes;
    }
    if (o.solver == GP_SOLVER_MINRES || (o.solver == GP_SOLVER_AUTO && sr.st != GP_OK)) {
      // after GP_ENOTCONV from the conjugate gradients' last iterate; after
      // non-positive curvature (their iterate is then no useful start) from zero
      const bool warm = o.solver == GP_SOLVER_AUTO && sr.st == GP_ENOTCONV;
      sr = gps::minres_solve(c, mm, yb, xb, warm, o.rtol, o.max_iter, o.precond);
      out->minres_iters = sr.iters;
    }
    out->quad = sr.quad;
    out->relres = sr.relres;
    GPS_REQUIRE(std::isfinite(sr.quad), GP_EINVAL, "y holds non-finite values");
    solve_status = sr.st;
    if (alpha) gps::permute_to_orig<double>(c, m->ds, 1, xb, alpha);
    if (slq) {
      if (c->concurrent)
        gps::join_side(c);
      else
        gps::slq_logdet_device(c, m, o.seed, o.n_probes, o.n_lanczos, reorth, dld);
      gps::DeviceLogdet* h = static_cast<gps::DeviceLogdet*>(gps::pinned(c, sizeof(gps::DeviceLogdet)));
      GPS_HIP(hipMemcpyAsync(h, dld, sizeof(gps::DeviceLogdet), hipMemcpyDeviceToHost, c->stream));
      gps::sync(c);
      out->logdet = h->logdet;
      out->logdet_se = h->se;
      out->lanczos_steps = h->steps;
      if (solve_status == GP_OK) solve_status = static_cast<gp_status>(h->status);
    } else if (with_logdet && o.logdet_mode == GP_LOGDET_EXACT) {
      const gps::LogdetResult lr = gps::exact_logdet(c, m, o.seed);
      out->logdet = lr.logdet;
      out->logdet_se = lr.se;
      out->lanczos_steps = lr.steps;
      if (solve_status == GP_OK) solve_status = lr.st;
    }
    out->loglik = -0.5 * out->logdet - 0.5 * out->quad - 0.5 * static_cast<double>(n) * std::log(2.0 * M_PI);
    gps::sync(c);
  });
  if (st != GP_OK) {
    out->status = st;
    return st;
  }
  out->status = solve_status;
  if (solve_status != GP_OK) {
    c->err = solve_status == GP_ENOTCONV ? "the solver did not reach rtol within max_iter"
                                         : "non-positive curvature: matrix not positive definite";
  }
  return solve_status;
}

namespace {

// The results of the device-driven likelihood of R problems, written by the
// device into the caller's (pinned or device) memory:
// -1/2 logdet - 1/2 quad - (n/2) log 2 pi, with (n/2) log 2 pi formed on the
// host as gp_loglik forms it (half_n_log2pi[r], or half1 for one problem).
__global__ void k_loglik_result(gps::DeviceSolve sv, const gps::DeviceLogdet* __restrict__ ld, int with_logdet,
                                const double* __restrict__ half_n_log2pi, double half1, int R,
                                gp_loglik_result* __restrict__ out) {
#pragma clang fp contract(off)
  for (int q = threadIdx.x; q < R; q += blockDim.x) {
    const gps::CgCtl& ctl = sv.ctl[q];
    gp_loglik_result r{};
    r.quad = sv.quad[q];
    r.relres = ctl.relres;
    r.cg_iters = ctl.iters;
    r.refreshes = ctl.refreshes;
    int st = ctl.status;
    if (with_logdet) {
      r.logdet = ld[q].logdet;
      r.logdet_se = ld[q].se;
      r.lanczos_steps = ld[q].steps;
      if (st == GP_OK) st = ld[q].status;
    }
    r.loglik = -0.5 * r.logdet - 0.5 * r.quad - (half_n_log2pi ? half_n_log2pi[q] : half1);
    r.status = st;
    out[q] = r;
  }
}

}  // namespace

gp_status gp_loglik_async(gp_ctx* c, const gp_matrix* m, const double* y, const gp_solve_opts* opts, double* alpha,
                          gp_loglik_result* out, void* event) {
  if (!c || !m || !y || !out) return GP_EINVAL;
  return guarded(c, [&] {
    const gp_solve_opts o = fill_opts(opts);
    GPS_REQUIRE(o.solver == GP_SOLVER_CG || o.solver == GP_SOLVER_AUTO, GP_EINVAL,
                "gp_loglik_async: the solver must be GP_SOLVER_CG (or AUTO, run as CG)");
    GPS_REQUIRE(o.logdet_mode != GP_LOGDET_EXACT, GP_EINVAL, "gp_loglik_async: GP_LOGDET_EXACT is not available");
    // the result is written by a kernel: it must be memory the device can reach
    hipPointerAttribute_t attr{};
    const hipError_t pe = hipPointerGetAttributes(&attr, out);
    (void)hipGetLastError();
    GPS_REQUIRE(pe == hipSuccess && (attr.type == hipMemoryTypeHost || attr.type == hipMemoryTypeDevice ||
                                     attr.type == hipMemoryTypeManaged),
                GP_EINVAL, "gp_loglik_async: out must be pinned host memory (or device memory)");
    const int64_t n = m->n;
    gp_matrix* mm = const_cast<gp_matrix*>(m);
    // caches of the products and the preconditioner (built with host
    // synchronisations the first time a matrix is used, not again)
    gps::build_product_caches(c, mm);
    if (o.precond == GP_PRECOND_BLOCK_JACOBI) gps::build_block_jacobi(c, mm);
    double* yb = static_cast<double*>(gps::workspace(c, 44, sizeof(double) * n));
    double* xb = static_cast<double*>(gps::workspace(c, 45, sizeof(double) * n));
    gps::permute_to_binned<double>(c, m->ds, 1, y, yb);
    // the log det on the side stream beside the solve (joined before the result)
    const bool with_logdet = o.logdet_mode != GP_LOGDET_NONE;
    const bool reorth = o.logdet_mode == GP_LOGDET_SLQ_REORTH;
    gps::DeviceLogdet* ld = static_cast<gps::DeviceLogdet*>(gps::workspace(c, 124, sizeof(gps::DeviceLogdet)));
    gps::JoinGuard join{c};
    if (with_logdet && c->concurrent) {
      gps::slq_reserve(c, m, o.n_probes, o.n_lanczos, reorth);
      gps::slq_logdet_side(c, m, o.seed, o.n_probes, o.n_lanczos, reorth, ld);
    }
    gps::DeviceSolve sv{};
    gps::pcg_solve_device(c, mm, yb, xb, o.rtol, o.max_iter, o.precond, &sv);
    if (alpha) gps::permute_to_orig<double>(c, m->ds, 1, xb, alpha);
    if (with_logdet && !c->concurrent)
      gps::slq_logdet_device(c, m, o.seed, o.n_probes, o.n_lanczos, reorth, ld);
    gps::join_side(c);
    // (n/2) log(2 pi) formed on the host as gp_loglik forms it
    const double half_n_log2pi = 0.5 * static_cast<double>(n) * std::log(2.0 * M_PI);
    hipLaunchKernelGGL(k_loglik_result, dim3(1), dim3(64), 0, c->stream, sv, ld, with_logdet ? 1 : 0, nullptr,
                       half_n_log2pi, 1, out);
    gps::check_launch("loglik result");
    if (event) GPS_HIP(hipEventRecord(static_cast<hipEvent_t>(event), c->stream));
  });
}

gp_status gp_loglik_batch(gp_ctx* c, int32_t nreq, const gp_matrix* const* K, const double* const* y,
                          const gp_solve_opts* opts, double* const* alpha, gp_loglik_result* out) {
  if (!c || !K || !y || !out || nreq < 1) return GP_EINVAL;
  for (int r = 0; r < nreq; ++r)
    if (!K[r] || !y[r]) return GP_EINVAL;
  std::memset(out, 0, sizeof(gp_loglik_result) * nreq);
  const gp_solve_opts o = fill_opts(opts);
  gp_status st = guarded(c, [&] {
    GPS_REQUIRE(o.solver == GP_SOLVER_CG || o.solver == GP_SOLVER_AUTO, GP_EINVAL,
                "gp_loglik_batch: the solver must be GP_SOLVER_CG or GP_SOLVER_AUTO");
    GPS_REQUIRE(o.logdet_mode == GP_LOGDET_SLQ || o.logdet_mode == GP_LOGDET_NONE, GP_EINVAL,
                "gp_loglik_batch: the log det mode must be GP_LOGDET_SLQ or GP_LOGDET_NONE");
    const int R = nreq;
    const bool bj = o.precond == GP_PRECOND_BLOCK_JACOBI;
    for (int r = 0; r < R; ++r) {
      gp_matrix* mm = const_cast<gp_matrix*>(K[r]);
      GPS_REQUIRE(mm->ds != nullptr, GP_EINVAL, "gp_loglik_batch: a matrix has no dataset");
      gps::build_product_caches(c, mm);
      if (bj) gps::build_block_jacobi(c, mm);
    }
    auto release = [c](gp_matrix* x) { gps::destroy_matrix(c, x); };
    std::unique_ptr<gp_matrix, decltype(release)> S(gps::stack_matrices(c, R, K, bj), release);
    const int64_t n = S->n;
    // per problem: row offsets, 1 / sqrt(n_r) (the first Lanczos scale), (n_r / 2) log 2 pi
    std::vector<int64_t> off(R + 1, 0);
    int64_t nmax = 0;
    for (int r = 0; r < R; ++r) {
      off[r + 1] = off[r] + K[r]->n;
      nmax = std::max(nmax, K[r]->n);
    }
    const size_t tb = sizeof(int64_t) * (R + 1) + 2 * sizeof(double) * R;
    char* h = static_cast<char*>(gps::pinned_for_write(c, tb));
    std::memcpy(h, off.data(), sizeof(int64_t) * (R + 1));
    double* hinv = reinterpret_cast<double*>(h + sizeof(int64_t) * (R + 1));
    double* hhalf = hinv + R;
    for (int r = 0; r < R; ++r) {
      hinv[r] = 1.0 / std::sqrt(static_cast<double>(K[r]->n));
      hhalf[r] = 0.5 * static_cast<double>(K[r]->n) * std::log(2.0 * M_PI);
    }
    char* dtab = static_cast<char*>(gps::workspace(c, 131, tb));
    gps::h2d_async(c, dtab, h, tb);
    const int64_t* doff = reinterpret_cast<const int64_t*>(dtab);
    const double* dinv = reinterpret_cast<const double*>(dtab + sizeof(int64_t) * (R + 1));
    const double* dhalf = dinv + R;
    // stacked right-hand sides and probe keys (each problem's own original indices)
    double* yb = static_cast<double*>(gps::workspace(c, 44, sizeof(double) * n));
    double* xb = static_cast<double*>(gps::workspace(c, 45, sizeof(double) * n));
    int32_t* perm = static_cast<int32_t*>(gps::workspace(c, 132, sizeof(int32_t) * n));
    for (int r = 0; r < R; ++r) {
      gps::permute_to_binned<double>(c, K[r]->ds, 1, y[r], yb + off[r]);
      GPS_HIP(hipMemcpyAsync(perm + off[r], K[r]->ds->perm, sizeof(int32_t) * K[r]->n, hipMemcpyDeviceToDevice,
                             c->stream));
    }
    // the log dets on the side stream beside the solves
    const bool with_logdet = o.logdet_mode == GP_LOGDET_SLQ;
    gps::DeviceLogdet* ld = static_cast<gps::DeviceLogdet*>(gps::workspace(c, 133, sizeof(gps::DeviceLogdet) * R));
    gps::JoinGuard join{c};
    gps::SlqBatch b;
    b.R = R;
    b.off = doff;
    b.inv0 = dinv;
    b.perm = perm;
    b.nmax = nmax;
    if (with_logdet && c->concurrent) {
      gps::slq_reserve(c, S.get(), o.n_probes, o.n_lanczos, false, R);
      gps::slq_batch_side(c, S.get(), o.seed, o.n_probes, o.n_lanczos, b, ld);
    }
    gps::DeviceSolve sv{};
    gps::pcg_solve_batch(c, S.get(), yb, xb, o.rtol, o.max_iter, o.precond, R, doff, nmax, &sv);
    if (alpha)
      for (int r = 0; r < R; ++r)
        if (alpha[r]) gps::permute_to_orig<double>(c, K[r]->ds, 1, xb + off[r], alpha[r]);
    if (with_logdet && !c->concurrent) gps::slq_logdet_batch(c, S.get(), o.seed, o.n_probes, o.n_lanczos, b, ld);
    gps::join_side(c);
    gp_loglik_result* dres = static_cast<gp_loglik_result*>(gps::workspace(c, 134, sizeof(gp_loglik_result) * R));
    hipLaunchKernelGGL(k_loglik_result, dim3(1), dim3(64), 0, c->stream, sv, ld, with_logdet ? 1 : 0, dhalf, 0.0, R,
                       dres);
    gps::check_launch("loglik batch result");
    gp_loglik_result* hres = static_cast<gp_loglik_result*>(gps::pinned(c, sizeof(gp_loglik_result) * R));
    GPS_HIP(hipMemcpyAsync(hres, dres, sizeof(gp_loglik_result) * R, hipMemcpyDeviceToHost, c->stream));
    gps::sync(c);
    std::memcpy(out, hres, sizeof(gp_loglik_result) * R);
  });
  if (st != GP_OK) {
    for (int r = 0; r < nreq; ++r) out[r].status = st;
    return st;
  }
  // GP_SOLVER_AUTO: a problem whose conjugate gradients did not succeed is
  // evaluated again alone, where MINRES takes over as in gp_loglik
  gp_status first = GP_OK;
  for (int r = 0; r < nreq; ++r) {
    if (o.solver == GP_SOLVER_AUTO && (out[r].status == GP_ENOTCONV || out[r].status == GP_ENOTPD))
      (void)loglik_common(c, K[r], y[r], &o, alpha ? alpha[r] : nullptr, &out[r], true);
    if (first == GP_OK && out[r].status != GP_OK) first = static_cast<gp_status>(out[r].status);
  }
  if (first != GP_OK) c->err = "at least one problem of the batch did not succeed (see its status)";
  return first;
}

gp_status gp_loglik(gp_ctx* c, const gp_matrix* m, const double* y, const gp_solve_opts* opts, double* alpha,
                    gp_loglik_result* out) {
  return loglik_common(c, m, y, opts, alpha, out, true);
}

gp_status gp_solve(gp_ctx* c, const gp_matrix* m, const double* y, const gp_solve_opts* opts, double* alpha,
                   gp_loglik_result* out) {
  return loglik_common(c, m, y, opts, alpha, out, false);
}

gp_status gp_predictor_create(gp_ctx* c, const gp_dataset* train, const gp_theta* th, const double* alpha,
                              gp_predictor** out) {
  if (!c || !out) return GP_EINVAL;
  *out = nullptr;
  return guarded(c, [&] {
    GPS_REQUIRE(train && alpha, GP_EINVAL, "gp_predictor_create: NULL argument");
    validate_theta(th, train->d);
    *out = gps::make_predictor(c, train, th, alpha);
  });
}

gp_status gp_predictor_destroy(gp_ctx* c, gp_predictor* p) {
  if (!c) return GP_EINVAL;
  if (!p) return GP_OK;
  return guarded(c, [&] { gps::destroy_predictor(c, p); });
}

gp_status gp_predict(gp_ctx* c, const gp_predictor* p, int64_t m, const double* xs, gp_precision prec,
                     double* mean) {
  if (!c || !p) return GP_EINVAL;
  return guarded(c, [&] {
    GPS_REQUIRE(m >= 0, GP_EINVAL, "gp_predict: m must be >= 0");
    GPS_REQUIRE(m == 0 || (xs && mean), GP_EINVAL, "gp_predict: NULL buffer");
    GPS_REQUIRE(prec == GP_FP64 || prec == GP_MIXED, GP_EINVAL, "gp_predict: unknown precision");
    gps::predict(c, p, m, xs, prec, mean);
    gps::sync(c);
  });
}

gp_status gp_predict_batch(gp_ctx* c, int32_t nreq, const gp_predictor* const* preds, const int64_t* row_offsets,
                           const double* xs, gp_precision prec, double* mean) {
  if (!c) return GP_EINVAL;
  return guarded(c, [&] {
    GPS_REQUIRE(nreq >= 0, GP_EINVAL, "gp_predict_batch: nreq must be >= 0");
    if (nreq == 0) return;
    GPS_REQUIRE(preds && row_offsets, GP_EINVAL, "gp_predict_batch: NULL argument");
    GPS_REQUIRE(prec == GP_FP64 || prec == GP_MIXED, GP_EINVAL, "gp_predict_batch: unknown precision");
    GPS_REQUIRE(row_offsets[0] == 0, GP_EINVAL, "gp_predict_batch: row_offsets[0] must be 0");
    for (int32_t r = 0; r < nreq; ++r) {
      GPS_REQUIRE(preds[r] != nullptr, GP_EINVAL, "gp_predict_batch: NULL predictor");
      GPS_REQUIRE(row_offsets[r + 1] >= row_offsets[r], GP_EINVAL,
                  "gp_predict_batch: row_offsets must be non-decreasing");
    }
    const int64_t m = row_offsets[nreq];
    GPS_REQUIRE(m == 0 || (xs && mean), GP_EINVAL, "gp_predict_batch: NULL buffer");
    gps::predict_batch(c, nreq, preds, row_offsets, xs, prec, mean);
    gps::sync(c);
  });
}

gp_status gp_mean_residual(gp_ctx* c, int64_t n, int32_t p, const double* W, const double* beta, const double* z,
                           double* y) {
  if (!c) return GP_EINVAL;
  return guarded(c, [&] {
    GPS_REQUIRE(n >= 1 && p >= 0, GP_EINVAL, "gp_mean_residual: n must be >= 1 and p >= 0");
    GPS_REQUIRE(z && y && (p == 0 || (W && beta)), GP_EINVAL, "gp_mean_residual: NULL buffer");
    for (int k = 0; k < p; ++k)
      GPS_REQUIRE(std::isfinite(beta[k]), GP_EINVAL, "gp_mean_residual: beta must be finite");
    gps::mean_residual(c, n, p, W, beta, z, y);
    gps::sync(c);
  });
}

gp_status gp_predict_var(gp_ctx* c, const gp_matrix* K, const gp_theta* th, int64_t m, const double* xs,
                         const gp_solve_opts* opts, double* var, gp_var_result* out) {
  if (!c || !K) return GP_EINVAL;
  if (out) std::memset(out, 0, sizeof(*out));
  gp_status solve_status = GP_OK;
  gp_status st = guarded(c, [&] {
    validate_theta(th, K->ds->d);
    GPS_REQUIRE(gps::theta_hash(th) == K->theta_hash, GP_EINVAL,
                "gp_predict_var: theta differs from the hyper-parameters K was assembled with");
    GPS_REQUIRE(m >= 0, GP_EINVAL, "gp_predict_var: m must be >= 0");
    GPS_REQUIRE(m == 0 || (xs && var), GP_EINVAL, "gp_predict_var: NULL buffer");
    const gp_solve_opts o = fill_opts(opts);
    const gps::VarResult r = gps::predict_variance(c, K, th, m, xs, o.rtol, o.max_iter, o.precond, var);
    gps::sync(c);
    if (out) {
      out->iters = r.iters;
      out->max_batch_iters = r.max_batch_iters;
      out->relres = r.relres;
    }
    solve_status = r.st;
  });
  if (st != GP_OK) {
    if (out) out->status = st;
    return st;
  }
  if (out) out->status = solve_status;
  if (solve_status != GP_OK)
    c->err = solve_status == GP_ENOTCONV ? "gp_predict_var: a column did not reach rtol within max_iter"
                                         : "gp_predict_var: non-positive curvature";
  return solve_status;
}

}  // extern "C"
