// C-ABI of the krs library: argument checking and dispatch to the drivers.
#include <climits>
#include <cmath>
#include <new>
#include <string>

#include "internal.hpp"

using krs::set_err;

namespace {

size_t dsize(krs_dtype dt) { return dt == KRS_F64 ? sizeof(double) : sizeof(float); }

bool valid_dtype(int dt) { return dt == KRS_F64 || dt == KRS_F32; }

int check_opts(krs_ctx* ctx, const krs_opts* o, bool needs_m) {
  if (!o) return set_err(ctx, KRS_ERR_ARG, "opts is NULL");
  if (needs_m && (o->m < 1 || o->m > krs::kMaxM))
    return set_err(ctx, KRS_ERR_ARG, "opts.m must be in 1..64");
  if (!(o->tol >= 0)) return set_err(ctx, KRS_ERR_ARG, "opts.tol must be >= 0");
  if (o->history_cap < 0 || (o->history_cap > 0 && !o->history))
    return set_err(ctx, KRS_ERR_ARG, "history buffer inconsistent");
  if (o->recycle_rule != KRS_RECYCLE_HARMONIC && o->recycle_rule != KRS_RECYCLE_GCROT)
    return set_err(ctx, KRS_ERR_ARG, "unknown opts.recycle_rule");
  if (o->recycle_rule == KRS_RECYCLE_GCROT) {
    if (o->gcrot_p < 0 || o->gcrot_p > 4)
      return set_err(ctx, KRS_ERR_ARG, "opts.gcrot_p must be in 0..4");
    if (o->gcrot_s > o->m) return set_err(ctx, KRS_ERR_ARG, "opts.gcrot_s must not exceed opts.m");
    if (o->gcrot_kt > 0 && o->gcrot_kt >= o->k)
      return set_err(ctx, KRS_ERR_ARG, "opts.gcrot_kt must be below opts.k");
  }
  return KRS_OK;
}

int check_rec(krs_ctx* ctx, const krs_matrix* A, const krs_recycle* rec, const krs_opts* o,
              bool updating) {
  if (!rec) return KRS_OK;
  if (rec->n != A->n) return set_err(ctx, KRS_ERR_STATE, "recycle space size differs from matrix");
  if (rec->dt != A->dt) return set_err(ctx, KRS_ERR_STATE, "recycle space dtype differs from matrix");
  if (o && updating) {
    if (o->k < 1 || o->k > rec->kmax)
      return set_err(ctx, KRS_ERR_ARG, "opts.k must be in 1..kmax of the recycle space");
    if (o->k + o->m + 1 > 64)
      return set_err(ctx, KRS_ERR_ARG, "opts.k + opts.m + 1 must not exceed 64");
  }
  if (o && rec->dim + o->m + 1 > 64)
    return set_err(ctx, KRS_ERR_ARG, "recycle dimension + opts.m + 1 must not exceed 64");
  return KRS_OK;
}

int check_precond(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M) {
  if (M && M->A != A) {
    const krs_matrix* B = M->A;
    if (B->n != A->n || B->dt != A->dt)
      return set_err(ctx, KRS_ERR_STATE, "preconditioner built for another matrix");
  }
  return KRS_OK;
}

}  // namespace

extern "C" {

const char* krs_version(void) { return "krs 0.1 (gfx950)"; }

int krs_create(krs_ctx** out, void* hip_stream) {
  if (!out) return KRS_ERR_ARG;
  *out = nullptr;
  krs_ctx* c = new (std::nothrow) krs_ctx();
  if (!c) return KRS_ERR_ARG;
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return KRS_ERR_HIP;
  }
  if (hipHostMalloc((void**)&c->pin, sizeof(double) * krs::kPinDoubles, hipHostMallocDefault) !=
      hipSuccess) {
    delete c;
    return KRS_ERR_HIP;
  }
  // device address of this GPU's static workspace (krs_rbicgstab_solve_noalloc)
  if (krs::noalloc_init(c) != KRS_OK) {
    (void)hipHostFree(c->pin);
    delete c;
    return KRS_ERR_HIP;
  }
  *out = c;
  return KRS_OK;
}

void krs_destroy(krs_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  krs::timing_release(ctx);
  for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
  if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  delete ctx;
}

const char* krs_last_error(const krs_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int krs_set_stream(krs_ctx* ctx, void* hip_stream) {
  if (!ctx) return KRS_ERR_ARG;
  ctx->stream = (hipStream_t)hip_stream;
  return KRS_OK;
}

int krs_matrix_create(krs_ctx* ctx, const krs_grid* g, krs_dtype dt, const void* bands,
                      krs_matrix** out) {
  return krs::matrix_create(ctx, g, dt, bands, 7, out);
}

int krs_matrix_create_19pt(krs_ctx* ctx, const krs_grid* g, krs_dtype dt, const void* bands,
                           krs_matrix** out) {
  return krs::matrix_create(ctx, g, dt, bands, 19, out);
}
}  // extern "C"

namespace krs {
int matrix_create(krs_ctx* ctx, const krs_grid* g, krs_dtype dt, const void* bands, int pts,
                  krs_matrix** out) {
  if (!ctx || !g || !out) return KRS_ERR_ARG;
  *out = nullptr;
  if (!valid_dtype(dt)) return set_err(ctx, KRS_ERR_ARG, "unknown dtype");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return set_err(ctx, KRS_ERR_ARG, "grid sizes must be >= 1");
  const int64_t n = g->nx * g->ny * g->nz;
  if (g->nx > INT_MAX || g->ny > INT_MAX || g->nz > INT_MAX || n > (int64_t)INT_MAX)
    return set_err(ctx, KRS_ERR_ARG, "grid too large (N must fit in 31 bits)");
  const int64_t dims[3] = {g->nx, g->ny, g->nz};
  for (int a = 0; a < 3; ++a)
    if (g->periodic[a] && dims[a] < 3)
      return set_err(ctx, KRS_ERR_ARG, "a periodic axis needs at least 3 cells");
  if (!bands) return set_err(ctx, KRS_ERR_ARG, "bands is NULL");
  krs_matrix* A = new (std::nothrow) krs_matrix();
  if (!A) return KRS_ERR_ARG;
  A->ctx = ctx;
  A->g = *g;
  A->dt = dt;
  A->bands = bands;
  A->n = n;
  A->pts = pts;
  *out = A;
  return KRS_OK;
}
}  // namespace krs

extern "C" {

void krs_matrix_destroy(krs_matrix* A) { delete A; }

size_t krs_precond_workspace_size(const krs_matrix* A, const krs_precond_desc* d) {
  if (!A || !d) return 0;
  if (d->type != KRS_PC_SCHWARZ_JACOBI) return 0;
  size_t v = krs::align_up((size_t)krs::vec_ld(A->n) * dsize(A->dt));
  return v + krs::align_up(krs::precond_pack_bytes(A, d));
}

int krs_precond_refresh(krs_ctx* ctx, krs_precond* M) {
  if (!ctx || !M) return KRS_ERR_ARG;
  return krs::precond_pack(ctx, M);
}

int krs_precond_create(krs_ctx* ctx, const krs_matrix* A, const krs_precond_desc* d, void* ws,
                       size_t ws_bytes, krs_precond** out) {
  if (!ctx || !A || !d || !out) return KRS_ERR_ARG;
  *out = nullptr;
  if (d->type != KRS_PC_NONE && d->type != KRS_PC_JACOBI && d->type != KRS_PC_SCHWARZ_JACOBI)
    return set_err(ctx, KRS_ERR_ARG, "unknown preconditioner type");
  if (d->type == KRS_PC_SCHWARZ_JACOBI) {
    if (d->tile != 4 && d->tile != 8) return set_err(ctx, KRS_ERR_ARG, "tile must be 4 or 8");
    if (d->overlap != 1) return set_err(ctx, KRS_ERR_ARG, "overlap must be 1");
    if (d->local_sweeps < 0 || d->global_sweeps < 0)
      return set_err(ctx, KRS_ERR_ARG, "sweep counts must be >= 0");
    if (d->local_solver != KRS_LOCAL_JACOBI && d->local_solver != KRS_LOCAL_SSOR)
      return set_err(ctx, KRS_ERR_ARG, "unknown local solver");
    if (d->local_solver == KRS_LOCAL_SSOR && A->pts != 7)
      return set_err(ctx, KRS_ERR_ARG,
                     "SSOR local solves need 7-point bands (two colours decouple only those)");
    const int64_t dims[3] = {A->g.nx, A->g.ny, A->g.nz};
    for (int a = 0; a < 3; ++a) {
      if (dims[a] % d->tile)
        return set_err(ctx, KRS_ERR_ARG, "grid sizes must be multiples of the tile size");
      if (A->g.periodic[a] && dims[a] <= d->tile + 2 * d->overlap)
        return set_err(ctx, KRS_ERR_ARG, "a periodic axis must be longer than an extended tile");
    }
    if (!ws || ws_bytes < krs_precond_workspace_size(A, d))
      return set_err(ctx, KRS_ERR_WORKSPACE, "preconditioner workspace too small");
  }
  krs_precond* M = new (std::nothrow) krs_precond();
  if (!M) return KRS_ERR_ARG;
  M->ctx = ctx;
  M->A = A;
  M->d = *d;
  if (d->type == KRS_PC_SCHWARZ_JACOBI) {
    M->tmp = ws;
    M->pack = krs::precond_pack_bytes(A, d) > 0
                  ? (char*)ws + krs::align_up((size_t)krs::vec_ld(A->n) * dsize(A->dt))
                  : nullptr;
    const int rc = krs::precond_pack(ctx, M);
    if (rc) {
      delete M;
      return rc;
    }
  }
  *out = M;
  return KRS_OK;
}

void krs_precond_destroy(krs_precond* M) { delete M; }

int krs_recycle_create(krs_ctx* ctx, int64_t N, int kmax, krs_dtype dt, void* U, void* C,
                       int64_t ld, krs_recycle** out) {
  if (!ctx || !out) return KRS_ERR_ARG;
  *out = nullptr;
  if (!valid_dtype(dt)) return set_err(ctx, KRS_ERR_ARG, "unknown dtype");
  if (N < 1 || kmax < 1 || kmax > krs::kMaxK)
    return set_err(ctx, KRS_ERR_ARG, "recycle space: need N >= 1 and 1 <= kmax <= 62");
  if (ld < N || !U || !C) return set_err(ctx, KRS_ERR_ARG, "recycle space: bad U, C or ld");
  krs_recycle* r = new (std::nothrow) krs_recycle();
  if (!r) return KRS_ERR_ARG;
  r->ctx = ctx;
  r->n = N;
  r->kmax = kmax;
  r->dt = dt;
  r->U = U;
  r->C = C;
  r->ld = ld;
  r->dim = 0;
  *out = r;
  return KRS_OK;
}

void krs_recycle_destroy(krs_recycle* rec) { delete rec; }

int krs_recycle_dim(const krs_recycle* rec) { return rec ? rec->dim : KRS_ERR_ARG; }

int krs_recycle_set_dim(krs_recycle* rec, int k) {
  if (!rec || k < 0 || k > rec->kmax) return KRS_ERR_ARG;
  rec->dim = k;
  return KRS_OK;
}

int krs_recycle_mark_stale(krs_recycle* rec) {
  if (!rec) return KRS_ERR_ARG;
  rec->stale = true;
  return KRS_OK;
}

int krs_workspace_size(krs_solver solver, int64_t N, int m, int k, krs_dtype dt, size_t* bytes) {
  if (!bytes || N < 1 || m < 0 || m > krs::kMaxM || !valid_dtype(dt)) return KRS_ERR_ARG;
  return krs::workspace_bytes(solver, N, m, k, dt, bytes);
}

int krs_stencil_apply(krs_ctx* ctx, const krs_matrix* A, const void* x, void* y, double alpha,
                      double beta, const void* b) {
  if (!ctx || !A || !x || !y) return KRS_ERR_ARG;
  if (x == y) return set_err(ctx, KRS_ERR_ARG, "y must not alias x");
  const krs::Grid3 g = krs::grid3(A);
  const int mode = b ? 1 : (beta != 0.0 ? 2 : 0);
  hipError_t e;
  if (A->dt == KRS_F64)
    e = krs::stencil<double>(ctx->stream, g, (const double*)A->bands, (const double*)x, (double*)y,
                             alpha, beta, (const double*)b, mode);
  else
    e = krs::stencil<float>(ctx->stream, g, (const float*)A->bands, (const float*)x, (float*)y,
                            alpha, beta, (const float*)b, mode);
  if (e != hipSuccess) return set_err(ctx, KRS_ERR_HIP, hipGetErrorString(e));
  return KRS_OK;
}

int krs_precond_apply(krs_ctx* ctx, const krs_precond* M, const void* r, void* z) {
  if (!ctx || !M || !r || !z) return KRS_ERR_ARG;
  if (r == z) return set_err(ctx, KRS_ERR_ARG, "z must not alias r");
  return krs::precond_apply(ctx, M, r, z, M->tmp);
}

int krs_operator_apply(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, const void* v,
                       void* w, void* tmp) {
  if (!ctx || !A || !v || !w || !tmp) return KRS_ERR_ARG;
  if (v == w || v == tmp || w == tmp)
    return set_err(ctx, KRS_ERR_ARG, "v, w and tmp must be distinct buffers");
  int rc = check_precond(ctx, A, M);
  if (rc) return rc;
  return krs::operator_apply(ctx, A, M, v, w, tmp);
}

int krs_gmres(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, const void* b, void* x,
              const krs_opts* opts, void* ws, size_t ws_bytes, krs_stats* stats) {
  if (!ctx || !A || !b || !x) return KRS_ERR_ARG;
  int rc = check_opts(ctx, opts, true);
  if (rc) return rc;
  if ((rc = check_precond(ctx, A, M))) return rc;
  return krs::gmres_rgcrot(ctx, A, M, nullptr, false, b, x, opts, ws, ws_bytes, stats);
}

int krs_rgcrot_solve(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                     const void* b, void* x, const krs_opts* opts, void* ws, size_t ws_bytes,
                     krs_stats* stats) {
  if (!ctx || !A || !b || !x) return KRS_ERR_ARG;
  int rc = check_opts(ctx, opts, true);
  if (rc) return rc;
  if ((rc = check_precond(ctx, A, M))) return rc;
  const bool upd = rec && opts->update_recycle;
  if ((rc = check_rec(ctx, A, rec, opts, upd))) return rc;
  return krs::gmres_rgcrot(ctx, A, M, rec, upd, b, x, opts, ws, ws_bytes, stats);
}

int krs_rbicgstab_solve(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M,
                        const krs_recycle* rec, const void* b, void* x, const krs_opts* opts,
                        void* ws, size_t ws_bytes, krs_stats* stats) {
  if (!ctx || !A || !b || !x) return KRS_ERR_ARG;
  int rc = check_opts(ctx, opts, false);
  if (rc) return rc;
  if (opts->flags & KRS_FLAG_LEFT_PRECOND)
    return set_err(ctx, KRS_ERR_ARG, "rBiCGStab is right-preconditioned");
  if ((rc = check_precond(ctx, A, M))) return rc;
  if (rec) {
    if (rec->n != A->n || rec->dt != A->dt)
      return set_err(ctx, KRS_ERR_STATE, "recycle space does not match the matrix");
  }
  return krs::rbicgstab(ctx, A, M, rec, b, x, opts, ws, ws_bytes, stats);
}

int krs_recycle_update(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                       void* ws, size_t ws_bytes) {
  if (!ctx || !A || !rec) return KRS_ERR_ARG;
  int rc = check_precond(ctx, A, M);
  if (rc) return rc;
  if ((rc = check_rec(ctx, A, rec, nullptr, false))) return rc;
  return krs::recycle_setup(ctx, A, M, rec, ws, ws_bytes);
}

int krs_hybrid_solve(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                     int step, int n_switch, const void* b, void* x, const krs_opts* opts,
                     void* ws, size_t ws_bytes, krs_stats* stats) {
  if (!ctx || !A || !b || !x || !rec) return KRS_ERR_ARG;
  int rc = check_opts(ctx, opts, true);
  if (rc) return rc;
  if (opts->flags & KRS_FLAG_LEFT_PRECOND)
    return set_err(ctx, KRS_ERR_ARG, "the hybrid is right-preconditioned");
  if (opts->recycle_rule != KRS_RECYCLE_HARMONIC)
    return set_err(ctx, KRS_ERR_ARG, "the hybrid updates (U, C) by the harmonic-Ritz rule");
  if ((rc = check_precond(ctx, A, M))) return rc;
  if ((rc = check_rec(ctx, A, rec, opts, true))) return rc;
  if (opts->switch_back < 0 || !std::isfinite(opts->switch_back))
    return set_err(ctx, KRS_ERR_ARG, "switch_back must be >= 0");
  bool refreshed = false;
  if (rec->stale) {
    // the operator changed: C = qr(A~ U).Q and U <- U R^-1 again
    if (rec->dim > 0) {
      rc = krs::recycle_setup(ctx, A, M, rec, ws, ws_bytes);
      if (rc) return rc;
      refreshed = true;
    }
    rec->stale = false;
  }
  auto finish = [&](int code, int64_t solver) {
    if (stats) {
      stats->solver = solver;
      stats->refreshed = refreshed ? 1 : 0;
    }
    return code;
  };
  if (step < n_switch || rec->force_rgcrot) {
    rec->force_rgcrot = false;
    rec->ref_mv = 0;
    rc = krs::gmres_rgcrot(ctx, A, M, rec, true, b, x, opts, ws, ws_bytes, stats);
    return finish(rc, KRS_SOLVER_RGCROT);
  }
  krs_stats first;
  rc = krs::rbicgstab(ctx, A, M, rec, b, x, opts, ws, ws_bytes, &first);
  if (rc <= 0) {
    if (stats) *stats = first;
    if (rc == KRS_OK && opts->switch_back > 0) {
      if (rec->ref_mv == 0) rec->ref_mv = first.matvecs;
      else if ((double)first.matvecs > opts->switch_back * (double)rec->ref_mv)
        rec->force_rgcrot = true;
    }
    return finish(rc, KRS_SOLVER_RBICGSTAB);
  }
  // rBiCGStab failed: solve this system again with rGCROT (switch back)
  rec->ref_mv = 0;
  rc = krs::gmres_rgcrot(ctx, A, M, rec, true, b, x, opts, ws, ws_bytes, stats);
  if (stats) {
    stats->matvecs += first.matvecs;
    stats->time_ms += first.time_ms;
    stats->bytes_model += first.bytes_model;
  }
  return finish(rc, KRS_SOLVER_RGCROT);
}

int krs_ir_solve(krs_ctx* ctx, const krs_matrix* A64, const krs_matrix* A32,
                 const krs_precond* M32, krs_recycle* rec32, const void* b, void* x,
                 const krs_opts* opts, void* ws, size_t ws_bytes, krs_stats* stats) {
  if (!ctx || !A64 || !A32 || !b || !x) return KRS_ERR_ARG;
  int rc = check_opts(ctx, opts, true);
  if (rc) return rc;
  if (opts->flags & KRS_FLAG_LEFT_PRECOND)
    return set_err(ctx, KRS_ERR_ARG, "refinement runs right-preconditioned inner solves");
  if (opts->recycle_rule != KRS_RECYCLE_HARMONIC)
    return set_err(ctx, KRS_ERR_ARG, "refinement updates (U, C) by the harmonic-Ritz rule");
  if (A64->dt != KRS_F64 || A32->dt != KRS_F32)
    return set_err(ctx, KRS_ERR_STATE, "IR needs an FP64 and an FP32 matrix");
  if (A64->n != A32->n) return set_err(ctx, KRS_ERR_STATE, "IR matrices differ in size");
  if (A64->pts != A32->pts) return set_err(ctx, KRS_ERR_STATE, "IR matrices differ in stencil");
  if ((rc = check_precond(ctx, A32, M32))) return rc;
  if (opts->inner_solver != KRS_SOLVER_RGCROT && opts->inner_solver != KRS_SOLVER_RBICGSTAB)
    return set_err(ctx, KRS_ERR_ARG, "inner solver must be RGCROT or RBICGSTAB");
  const bool upd = rec32 && (opts->update_recycle || opts->inner_solver == KRS_SOLVER_RBICGSTAB);
  if ((rc = check_rec(ctx, A32, rec32, opts, upd))) return rc;
  return krs::ir_solve(ctx, A64, A32, M32, rec32, b, x, opts, ws, ws_bytes, stats);
}


int krs_ir_solve_batched(krs_ctx* ctx, int nsys, const krs_ir_system* sys, const krs_opts* opts,
                         void* ws, size_t ws_bytes) {
  if (!ctx || nsys < 0 || (nsys > 0 && !sys)) return KRS_ERR_ARG;
  int rc = check_opts(ctx, opts, true);
  if (rc) return rc;
  if (opts->flags & KRS_FLAG_LEFT_PRECOND)
    return set_err(ctx, KRS_ERR_ARG, "refinement runs right-preconditioned inner solves");
  if (opts->inner_solver != KRS_SOLVER_RBICGSTAB)
    return set_err(ctx, KRS_ERR_ARG, "batched refinement runs rBiCGStab inner solves");
  if (!ws || ws_bytes < KRS_BATCH_WORKSPACE_BYTES)
    return set_err(ctx, KRS_ERR_WORKSPACE, "batch workspace missing or too small");
  for (int i = 0; i < nsys; ++i) {
    const krs_ir_system& q = sys[i];
    if (!q.A64 || !q.A32 || !q.b || !q.x || !q.ws)
      return set_err(ctx, KRS_ERR_ARG, "system " + std::to_string(i) + ": missing argument");
    if (q.A64->dt != KRS_F64 || q.A32->dt != KRS_F32)
      return set_err(ctx, KRS_ERR_STATE, "IR needs an FP64 and an FP32 matrix");
    if (q.A64->n != q.A32->n || q.A64->pts != q.A32->pts)
      return set_err(ctx, KRS_ERR_STATE, "IR matrices differ");
    if ((rc = check_precond(ctx, q.A32, q.M32))) return rc;
    if ((rc = check_rec(ctx, q.A32, q.rec32, opts, q.rec32 != nullptr))) return rc;
    size_t need = 0;
    krs::workspace_bytes(KRS_SOLVER_IR, q.A64->n, opts->m, opts->k, KRS_F32, &need);
    if (q.ws_bytes < need)
      return set_err(ctx, KRS_ERR_WORKSPACE, "system " + std::to_string(i) + ": workspace too small");
    for (int j = 0; j < i; ++j)
      if (sys[j].x == q.x || sys[j].ws == q.ws || (q.rec32 && sys[j].rec32 == q.rec32))
        return set_err(ctx, KRS_ERR_ARG, "systems share x, a workspace or a recycle space");
  }
  return krs::ir_solve_batched(ctx, nsys, sys, opts, ws, ws_bytes);
}

}  // extern "C"
