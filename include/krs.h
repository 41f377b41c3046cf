/*
 * krs -- recycling Krylov solvers for sequences of structured-grid pressure
 * Poisson systems A x_t = b_t on AMD Instinct MI355X (gfx950).
 *
 * Method: Amritkar, de Sturler, Swirydowicz, Tafti, Ahuja, "Recycling Krylov
 * subspaces for CFD applications and a new hybrid recycling solver".
 *   GMRES(m) ............................ Alg. 1 (Sec. 2.2)
 *   BiCGStab ............................ Alg. 2 (Sec. 2.2)
 *   rGCROT(m,k)/GCRODR(m,k) ............. Alg. 3 (Sec. 2.3)
 *   rBiCGStab with one recycle space .... Alg. 4 (Sec. 2.3)
 *   hybrid rGCROT -> rBiCGStab .......... Sec. 2.4
 *   banded 7-point storage .............. Sec. 2.1, "Data Layout"
 *   Schwarz-Jacobi preconditioner ....... Sec. 2.1, "Preconditioners"
 *
 * Conventions (all entry points)
 * ------------------------------
 * Grid (nx, ny, nz); unknown i = x + nx*(y + ny*z), x fastest; N = nx*ny*nz.
 * Bands: one device array of 7*N values, band-major ([7][N]) in the order
 *   C, W (x-1), E (x+1), S (y-1), N (y+1), B (z-1), T (z+1):
 *   (A u)_i = C_i u_i + W_i u_{i-1} + E_i u_{i+1} + S_i u_{i-nx} + ...
 * A periodic axis wraps; across a non-periodic boundary the neighbour term is
 * dropped (the band there must be 0 or folded into C).
 * Vectors: device arrays of N values of the handle's dtype (FP64 or FP32),
 *   except where an argument says otherwise.
 * Multi-vectors (U, C): column-major, column c at base + c*ld, ld >= N.
 * An ld that is not a multiple of a large power of two streams faster (the
 * library's own multi-vectors use N rounded up to 64, plus 1088).
 * Solvers are right-preconditioned: they iterate on A~ = A M^-1 and return
 *   x = M^-1 y; the initial guess is always x = 0 (Sec. 2.2), the stopping
 *   test is ||b - A x|| <= tol ||b|| (the loop test of Alg. 1-4).
 * Recycle space: (U, C) with A~ U = C and C^T C = I (the R factor of
 *   the recycle-space setup of Alg. 3 is absorbed into U).
 *
 * Ownership: every device pointer belongs to the caller and must stay valid
 *   while a handle that borrowed it is alive.  The library never allocates
 *   device memory: solver scratch is a caller-provided workspace of the size
 *   returned by krs_workspace_size.  A context owns a small pinned host
 *   buffer and its HIP events.
 * Streams: every call enqueues on the context's stream.  krs_stencil_apply
 *   and krs_precond_apply are asynchronous; solver calls synchronise the
 *   stream (for convergence tests) and return when done; statistics are
 *   valid on return.
 * Threads: a context and the handles created from it are used by one host
 *   thread at a time; distinct contexts are independent.
 * Errors: functions return an int status; no exception crosses the ABI.
 *   0 = KRS_OK; > 0 = solver outcome (x holds the final iterate, stats are
 *   filled); < 0 = error (outputs unspecified); krs_last_error() describes
 *   the most recent error of a context.
 */
#ifndef KRS_H
#define KRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define KRS_OK 0
#define KRS_NOT_CONVERGED 1   /* max_matvecs reached before tol */
#define KRS_BREAKDOWN 2       /* rho = 0, r~^T v = 0 or t^T t = 0 (Alg. 2/4) */
#define KRS_DIVERGED 3        /* non-finite residual or growth above div_factor */
#define KRS_ERR_ARG (-1)      /* invalid argument or unsupported shape */
#define KRS_ERR_HIP (-2)      /* HIP runtime error */
#define KRS_ERR_WORKSPACE (-3)/* workspace missing or too small */
#define KRS_ERR_STATE (-4)    /* handles do not match (size, dtype) */
#define KRS_ERR_EIG (-5)      /* host eigen-solver of the recycle update failed */

typedef enum krs_dtype { KRS_F64 = 0, KRS_F32 = 1 } krs_dtype;

typedef enum krs_solver {
  KRS_SOLVER_GMRES = 0,     /* Alg. 1 */
  KRS_SOLVER_RGCROT = 1,    /* Alg. 3 */
  KRS_SOLVER_RBICGSTAB = 2, /* Alg. 4 (Alg. 2 with an empty recycle space) */
  KRS_SOLVER_IR = 3,        /* FP32 inner solver inside FP64 refinement: extra FP64/FP32 vectors */
  KRS_SOLVER_RGCROT_T = 4   /* workspace size only: rGCROT with the GCROT rule
                               (opts.recycle_rule = KRS_RECYCLE_GCROT), m vectors more */
} krs_solver;

/* How rGCROT updates (U, C) at a cycle end (the cycle-end step of Alg. 3; the paper
 * leaves the details to its references, Sec. 2.3).
 * KRS_RECYCLE_HARMONIC: the GCRODR rule - the k harmonic Ritz vectors of the
 *   search space range(U) + range(V_j) with the smallest |theta|.
 * KRS_RECYCLE_GCROT: a reading of the GCROT rule, which measures angles
 *   between successive search spaces.  The outer space gains the cycle's
 *   own correction and gcrot_p directions of this cycle's selection space
 *   (the images of its last gcrot_s inner vectors) that make the smallest
 *   angles with the previous cycle's selection space (within one solve);
 *   when it would exceed k it is first cut to gcrot_kt columns, those making
 *   the smallest angles with the cycle's search space; two Cholesky-QR
 *   passes then restore C^T C = I.  Sec. 3 uses kt = k - 10, s = m / 2 and
 *   p = 1 or 2 (its fourth parameter, latest inner vectors kept, is 0 and
 *   not modelled).  Needs the KRS_SOLVER_RGCROT_T workspace; rGCROT only
 *   (the hybrid and refinement drivers reject it). */
typedef enum krs_recycle_rule { KRS_RECYCLE_HARMONIC = 0, KRS_RECYCLE_GCROT = 1 } krs_recycle_rule;

typedef enum krs_pc_type {
  KRS_PC_NONE = 0,
  KRS_PC_JACOBI = 1,          /* point Jacobi, M = diag(A) */
  KRS_PC_SCHWARZ_JACOBI = 2   /* overlapping tiles, damped Jacobi sweeps, global Jacobi sweep */
} krs_pc_type;

typedef struct krs_ctx krs_ctx;
typedef struct krs_matrix krs_matrix;
typedef struct krs_precond krs_precond;
typedef struct krs_recycle krs_recycle;

typedef struct krs_grid {
  int64_t nx, ny, nz;
  int32_t periodic[3];   /* nonzero: axis x / y / z wraps */
} krs_grid;

/* Local smoother of the Schwarz preconditioner (Sec. 2.1: Jacobi or SSOR). */
typedef enum krs_local_solver {
  KRS_LOCAL_JACOBI = 0,  /* damped Jacobi sweeps (factor omega_local) */
  KRS_LOCAL_SSOR = 1     /* SSOR iterations (relaxation omega_local): a forward SOR sweep
                            over the even-parity cells of the extended tile, then the odd
                            ones, and a backward sweep odd then even */
} krs_local_solver;

/* Preconditioner (Sec. 2.1, "Preconditioners in GenIDLEST"): cubic tiles of
 * `tile` owned cells per axis (4 or 8; grid sizes must be multiples; a
 * periodic axis must be longer than tile + 2*overlap), extended by `overlap`
 * (= 1) cells; `local_sweeps` iterations of the local smoother from zero on
 * each extended tile with zero values outside it; every cell keeps the value
 * of the tile owning it; then `global_sweeps` damped point-Jacobi sweeps
 * (factor omega_global) on the whole grid. */
typedef struct krs_precond_desc {
  int32_t type;            /* krs_pc_type */
  int32_t tile;
  int32_t overlap;
  int32_t local_sweeps;
  int32_t global_sweeps;
  int32_t local_solver;    /* krs_local_solver */
  double omega_local;
  double omega_global;
} krs_precond_desc;

/* GMRES-type solvers stop as soon as the least-squares residual estimate
 * meets tol, without confirming it with the true residual (used for the
 * inner solves of iterative refinement, whose outer FP64 residual decides). */
#define KRS_FLAG_TRUST_ESTIMATE 1
/* Test convergence on the host after every step: rBiCGStab after every half
 * step (two host round trips per iteration), GMRES / rGCROT after every
 * Arnoldi step (the host then applies the Givens rotations of Alg. 1 / 3 and
 * tests the residual estimate).  By default these tests run on the device
 * (the scalar steps of Alg. 4; the Givens rotations, estimate and stopping
 * tests of an Arnoldi step, in FP64 with the host's operation order) and the
 * host enqueues several iterations or steps between reads; work enqueued
 * after the stop changes nothing that the result reads, so both modes give
 * bitwise the same result, history, recycle space and counts. */
#define KRS_FLAG_HOST_LOOP 2
/* rBiCGStab, device-driven loop: replay a captured HIP graph of one
 * iteration instead of enqueuing its kernels one by one (grids of at most
 * 2^20 cells, kernel timing off).  The context keeps up to 8 graphs, keyed by
 * every pointer and size they contain (matrix, preconditioner, recycle space,
 * workspace), and releases them in krs_destroy.  Results are bitwise the same
 * either way.  Off by default: on gfx950 the replay saves no time per
 * iteration (the kernels' own dispatch latency dominates, not host launch
 * cost) and the first replay of a key pays for capture and instantiation. */
#define KRS_FLAG_GRAPH 4
/* GMRES / rGCROT only: precondition from the left, as the paper does for
 * these solvers (Sec. 2.1): iterate on M^-1 A x = M^-1 b and stop when
 * ||M^-1 (b - A x)|| <= tol ||M^-1 b||; stats->rel_res_est reports that ratio
 * and stats->rel_res_true the unpreconditioned ||b - A x|| / ||b||.  A
 * recycle space built this way belongs to M^-1 A and serves only
 * left-preconditioned solves.  The hybrid and refinement drivers reject it
 * (rBiCGStab is right-preconditioned, Sec. 2.1). */
#define KRS_FLAG_LEFT_PRECOND 8

typedef struct krs_opts {
  int32_t m;               /* Arnoldi steps per cycle (GMRES, rGCROT), 1..64 */
  int32_t k;               /* maximum recycle dimension (rGCROT update), <= recycle kmax;
                              rGCROT needs k + m + 1 <= 64 (one block pass over [C, V]) */
  int32_t update_recycle;  /* rGCROT: update (U, C) at every cycle end (Alg. 3) */
  int32_t inner_solver;    /* IR only: KRS_SOLVER_RGCROT or KRS_SOLVER_RBICGSTAB */
  double tol;              /* relative tolerance on ||b - A x|| / ||b|| */
  int64_t max_matvecs;     /* cap on applications of A~ in the iteration */
  double div_factor;       /* rBiCGStab: ||r|| > div_factor ||b|| => KRS_DIVERGED (<= 0: off) */
  double inner_tol;        /* IR only: relative tolerance of each inner solve */
  int32_t max_outer;       /* IR only: cap on refinement steps */
  int32_t flags;           /* KRS_FLAG_* */
  double* history;         /* optional host buffer: residual history (relative) */
  int64_t history_cap;
  double switch_back;      /* hybrid only: > 0 => after an rBiCGStab system needing more than
                              switch_back times the matvecs of the first rBiCGStab system
                              since the last rGCROT one, the next system runs rGCROT
                              (recycle space refreshed); 0 = off */
  int32_t recycle_rule;    /* krs_recycle_rule (rGCROT only) */
  int32_t gcrot_kt;        /* GCROT rule: outer vectors kept at a cut, 1..k-1 (<= 0: max(1, k-10)) */
  int32_t gcrot_s;         /* GCROT rule: inner vectors to select from, 1..m (<= 0: max(1, m/2)) */
  int32_t gcrot_p;         /* GCROT rule: inner vectors selected per cycle, 0..4 */
} krs_opts;

typedef struct krs_stats {
  int32_t status;
  int32_t eig_ties;        /* recycle updates whose k-th/(k+1)-th |theta| nearly tie */
  int64_t matvecs;         /* applications of A~ (iteration + residual checks) */
  int64_t iterations;      /* Arnoldi steps / BiCGStab while-loop passes */
  int64_t cycles;          /* GMRES-type cycles */
  int64_t outer;           /* IR refinement steps */
  int64_t history_len;
  double rel_res_true;     /* ||b - A x|| / ||b|| at exit, FP64 where applicable */
  double rel_res_est;      /* last recurrence/least-squares estimate */
  double time_ms;          /* wall time of the call */
  double host_eig_ms;      /* time in the host eigen step of the recycle update */
  double bytes_model;      /* algorithmic HBM bytes of the call (byte model) */
  int64_t second_passes;   /* Arnoldi steps that needed a second Gram-Schmidt pass */
  int64_t solver;          /* krs_hybrid_solve: solver that produced x (KRS_SOLVER_*) */
  int64_t refreshed;       /* krs_hybrid_solve: 1 if C was re-formed first (space marked stale) */
  int64_t breakdown_site;  /* (r)BiCGStab: 0 none, 1 r~^T v = 0 (alpha), 2 t^T t = 0
                              (omega), 3 rho = 0 */
} krs_stats;

/* ---------------- context ---------------- */

/* Creates a context enqueuing on `hip_stream` (a hipStream_t; NULL = the
 * default stream) of the current device. */
int krs_create(krs_ctx** out, void* hip_stream);
void krs_destroy(krs_ctx* ctx);
const char* krs_last_error(const krs_ctx* ctx);
int krs_set_stream(krs_ctx* ctx, void* hip_stream);

/* ---------------- handles ---------------- */

/* Matrix: borrows `bands` (7*N device values of `dt`). */
int krs_matrix_create(krs_ctx* ctx, const krs_grid* g, krs_dtype dt, const void* bands,
                      krs_matrix** out);
/* Matrix of a 19-point stencil (non-orthogonal grids, Sec. 2.1 "Data
 * Layout"): borrows `bands`, 19*N device values of `dt`, band-major.  Band 0
 * couples a cell to itself, bands 1-6 to its face neighbours in the order
 * of the 7-point layout (x-1, x+1, y-1, y+1, z-1, z+1), bands 7-18 to its
 * edge neighbours (dx, dy, dz): (-1,-1,0) (1,-1,0) (-1,1,0) (1,1,0),
 * (-1,0,-1) (1,0,-1) (-1,0,1) (1,0,1), (0,-1,-1) (0,1,-1) (0,-1,1) (0,1,1).
 * Periodic axes wrap; a neighbour beyond a non-periodic face contributes
 * nothing.  Every solver takes it; the Schwarz preconditioner then reads the
 * bands in its local solves (no coefficient pack) and runs the global sweep
 * and the matvec as separate passes; SSOR local solves are refused (the two
 * colours do not decouple edge neighbours). */
int krs_matrix_create_19pt(krs_ctx* ctx, const krs_grid* g, krs_dtype dt, const void* bands,
                           krs_matrix** out);
void krs_matrix_destroy(krs_matrix* A);

/* Preconditioner for A; `ws` is a device buffer of at least
 * krs_precond_workspace_size(A, d) bytes, owned by the caller (NULL allowed
 * when the size is 0).  For SCHWARZ_JACOBI it holds one temporary vector and a
 * copy of the local-solve coefficients (omega_local / a_C and
 * omega_local * a_k / a_C) for every cell of the extended tiles, grouped in
 * bricks of 2x2x2 tiles when every tile count is even (each cell stored once
 * per brick: 7 (2 tile+2)^3 / (2 tile)^3 values per cell, 9.97 for tile 8),
 * else per tile (7 (tile+2)^3 / tile^3, 13.7 for tile 8); built here on the
 * context stream from A's current bands.  If the caller changes A's bands
 * afterwards it must call krs_precond_refresh. */
int krs_precond_create(krs_ctx* ctx, const krs_matrix* A, const krs_precond_desc* d,
                       void* ws, size_t ws_bytes, krs_precond** out);
size_t krs_precond_workspace_size(const krs_matrix* A, const krs_precond_desc* d);
/* Rebuilds the stored coefficients from A's current bands. Asynchronous. */
int krs_precond_refresh(krs_ctx* ctx, krs_precond* M);
void krs_precond_destroy(krs_precond* M);

/* Recycle space: borrows U and C (each kmax columns of ld >= N values of
 * `dt`, 1 <= kmax <= 62); starts with dimension 0 (no recycling). */
int krs_recycle_create(krs_ctx* ctx, int64_t N, int kmax, krs_dtype dt, void* U, void* C,
                       int64_t ld, krs_recycle** out);
void krs_recycle_destroy(krs_recycle* rec);
int krs_recycle_dim(const krs_recycle* rec);
/* Sets the dimension (0..kmax), e.g. after U was filled by the caller; call
 * krs_recycle_update before solving if C does not hold A~ U. */
int krs_recycle_set_dim(krs_recycle* rec, int k);
/* Marks (U, C) stale: A or M changed since C = A~ U was formed.  The next
 * krs_hybrid_solve first re-forms C from U (the recycle-space setup of Alg. 3, which applies
 * whenever the matrix changes), keeping range(U).  Sec. 2.4 leaves the policy for changing
 * matrices open (intermittent rGCROT); this is the cheapest consistent one. */
int krs_recycle_mark_stale(krs_recycle* rec);

/* Workspace (bytes) for `solver` on N unknowns with parameters m, k. */
int krs_workspace_size(krs_solver solver, int64_t N, int m, int k, krs_dtype dt, size_t* bytes);

/* ---------------- operations ---------------- */

/* y = alpha * A x + beta * (b if b != NULL else y); y may not alias x.
 * The stencil of Sec. 2.1 in banded storage. Asynchronous. */
int krs_stencil_apply(krs_ctx* ctx, const krs_matrix* A, const void* x, void* y, double alpha,
                      double beta, const void* b);

/* z = M^-1 r (Sec. 2.1, "Preconditioners"); z may not alias r. Asynchronous. */
int krs_precond_apply(krs_ctx* ctx, const krs_precond* M, const void* r, void* z);

/* w = A M^-1 v, the right-preconditioned operator every solver iterates on
 * (Sec. 2.2: A and b stand for the preconditioned matrix and right-hand
 * side).  `tmp` is a caller device buffer of N values of A's dtype that
 * receives intermediate values; v, w and tmp must not alias one another.
 * With Schwarz-Jacobi and one global sweep on grids of at least 2^22 cells,
 * the sweep and the matvec run as one fused pass and tmp holds the
 * local-solve result, not M^-1 v (elsewhere tmp holds M^-1 v); both forms
 * give bitwise the same w.  M may be NULL (w = A v).  Asynchronous. */
int krs_operator_apply(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, const void* v,
                       void* w, void* tmp);

/* GMRES(m), Alg. 1, right-preconditioned (M may be NULL: no preconditioner).
 * b, x: N values of A's dtype. Uses opts.m, tol, max_matvecs. */
int krs_gmres(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, const void* b, void* x,
              const krs_opts* opts, void* ws, size_t ws_bytes, krs_stats* stats);

/* rGCROT(m,k)/GCRODR(m,k), Alg. 3.  Projects b against C, runs augmented
 * Arnoldi cycles (each new vector orthogonalised against C, then V), updates
 * x with V y - U B y at each cycle end (the sign minimising the residual over
 * range(U)+range(V)), and, when opts.update_recycle, replaces (U, C) at every
 * cycle end by the k harmonic Ritz vectors of smallest |theta| of
 * range(U)+range(V_j) (GCRODR rule; eigenproblem in FP64 on the host).  With an empty recycle
 * space and no update this is GMRES(m). */
int krs_rgcrot_solve(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                     const void* b, void* x, const krs_opts* opts, void* ws, size_t ws_bytes,
                     krs_stats* stats);

/* rBiCGStab with one recycle space, Alg. 4 (rec may be NULL or of dimension
 * 0: BiCGStab, Alg. 2).  r~ = r_0 after projection; U-updates postponed to
 * the end of the solve; rec is read only. */
int krs_rbicgstab_solve(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M,
                        const krs_recycle* rec, const void* b, void* x, const krs_opts* opts,
                        void* ws, size_t ws_bytes, krs_stats* stats);

/* Size (bytes) of the static device workspace of krs_rbicgstab_solve_noalloc,
 * one per GPU the library runs on, held until the process ends. */
#define KRS_NOALLOC_SCRATCH_BYTES ((size_t)48 << 20)

/* krs_rbicgstab_solve without allocations, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): the same solve with its workspace in a static device
 * array of KRS_NOALLOC_SCRATCH_BYTES (whose device address is looked up when
 * a context is created on that GPU) instead of a caller buffer.  Arguments as
 * for krs_rbicgstab_solve; the caller still provides b, x, the matrix,
 * preconditioner and recycle space.  Returns KRS_ERR_WORKSPACE when
 * krs_workspace_size(KRS_SOLVER_RBICGSTAB, N, ...) exceeds the static size
 * (FP64 up to about 5.2e5 unknowns, FP32 up to about 1.3e6), KRS_ERR_ARG
 * with KRS_FLAG_GRAPH and KRS_ERR_STATE while kernel timing is on (both
 * create runtime objects).  Calls no allocating routine.  All calls on one
 * GPU share the array: calls that overlap in time on one GPU (concurrent
 * streams or threads) race and must be serialised by the caller. */
int krs_rbicgstab_solve_noalloc(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M,
                                const krs_recycle* rec, const void* b, void* x,
                                const krs_opts* opts, krs_stats* stats);

/* Recycle-space setup of Alg. 3 and 4: C~ = A~ U, thin QR C~ = C R (Cholesky QR,
 * twice), U <- U R^-1.  Call when A changed or U was set by the caller. */
int krs_recycle_update(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                       void* ws, size_t ws_bytes);

/* Hybrid solver step (Sec. 2.4): systems with step < n_switch are solved by
 * rGCROT(m,k) with recycle updates, later ones by rBiCGStab with (U, C)
 * fixed; when rBiCGStab diverges, breaks down or does not converge, the
 * system is solved again by rGCROT (switch back).  With opts.switch_back > 0
 * a system whose rBiCGStab solve needed more than switch_back times the
 * matvecs of the first rBiCGStab system since the last rGCROT one makes the
 * next system run rGCROT (Sec. 2.4: switch back when convergence becomes
 * poor).  A space marked stale is re-formed from U first.  stats->solver
 * and stats->refreshed tell what ran.  The policy state lives in rec.
 * ws: krs_workspace_size(KRS_SOLVER_RGCROT). */
int krs_hybrid_solve(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                     int step, int n_switch, const void* b, void* x, const krs_opts* opts,
                     void* ws, size_t ws_bytes, krs_stats* stats);

/* Mixed precision: FP64 iterative refinement around an FP32 inner solver.
 * A64/b/x are FP64 (true residual b - A64 x, update x += d in FP64);
 * A32, M32, rec32 are the FP32 operator, preconditioner and recycle space
 * used by the inner solver opts.inner_solver (RGCROT: with recycle updates
 * when opts.update_recycle; RBICGSTAB: rec32 read only).  Each inner solve
 * runs to the relative tolerance max(opts.inner_tol, tol ||b|| / (2 ||r||))
 * on its scaled right-hand side r / ||r|| (no tighter than the refinement
 * still needs) and stops on its own residual estimate.  Stops when
 * ||b - A64 x|| <= tol ||b||, or when a refinement step reduces ||r|| by
 * less than 10%.
 * ws: krs_workspace_size(KRS_SOLVER_IR, N, m, k, KRS_F32). */
int krs_ir_solve(krs_ctx* ctx, const krs_matrix* A64, const krs_matrix* A32,
                 const krs_precond* M32, krs_recycle* rec32, const void* b, void* x,
                 const krs_opts* opts, void* ws, size_t ws_bytes, krs_stats* stats);

/* One system of krs_ir_solve_batched: the arguments of krs_ir_solve for
 * it (ws: krs_workspace_size(KRS_SOLVER_IR, N, opts.m, k, KRS_F32) bytes of
 * its own) and where its statistics go (may be NULL). */
typedef struct krs_ir_system {
  const krs_matrix* A64;
  const krs_matrix* A32;
  const krs_precond* M32;
  krs_recycle* rec32;
  const void* b;
  void* x;
  void* ws;
  size_t ws_bytes;
  krs_stats* stats;
} krs_ir_system;

/* Bytes of the shared workspace of krs_ir_solve_batched (the table of the
 * grouped launches). */
#define KRS_BATCH_WORKSPACE_BYTES ((size_t)64 << 10)

/* FP64 iterative refinement of nsys independent systems at once, each with
 * rBiCGStab inner solves (opts.inner_solver must be KRS_SOLVER_RBICGSTAB;
 * Sec. 2.4: the later systems of a sequence, once a recycle space exists),
 * for many small systems whose solves alone would be bound by kernel launch
 * latency.  Each inner rBiCGStab pass runs as one launch per step for all
 * systems (a block range of the grid per system), with a fixed per-system
 * reduction tree: every system's result, statistics and iteration counts
 * are bitwise those of krs_ir_solve on it alone.  Grouped: FP32 7-point
 * systems with the Schwarz-Jacobi preconditioner (8^3 tiles in bricks of
 * 2^3, Jacobi local sweeps, one global sweep) whose recycle spaces have the
 * same dimension as the first such system, up to 32 of them; every other
 * system is solved alone after them.  Systems converge and leave the group
 * independently.  Returns KRS_OK when every system converged, else the
 * largest per-system status (each in its stats->status), or a negative
 * error.  ws: KRS_BATCH_WORKSPACE_BYTES of device memory.  Synchronous. */
int krs_ir_solve_batched(krs_ctx* ctx, int nsys, const krs_ir_system* sys,
                         const krs_opts* opts, void* ws, size_t ws_bytes);

/* ---------------- measurement ---------------- */

/* Kernel classes timed by the per-class HIP-event timers. */
typedef enum krs_kernel_class {
  KRS_K_STENCIL = 0,        /* y = alpha A x + beta (b | y) */
  KRS_K_RESIDUAL = 1,       /* r = b - A x with the partial sums of |r|^2 */
  KRS_K_SCHWARZ_LOCAL = 2,  /* local sweeps on the extended tiles */
  KRS_K_JACOBI_SWEEP = 3,   /* global damped Jacobi sweep / point Jacobi */
  KRS_K_BLOCK_DOT = 4,      /* [C V]^T w and other block dot products */
  KRS_K_BLOCK_DOT2 = 5,     /* second Gram-Schmidt pass: [C V]^T (w - [C V] h) */
  KRS_K_BLOCK_UPDATE = 6,   /* w - [C V] h, solution and projection updates */
  KRS_K_BICG_P = 7,         /* full-step tests and p = r + beta (p - omega v); the separate
                               half-step exit of the host-tested loop */
  KRS_K_BICG_SV = 8,        /* v -= C eta1, s = r - alpha v, |s|^2 */
  KRS_K_BICG_YR = 9,        /* y += alpha p + omega s, r = s - omega (t - C eta2), dots; or the
                               half-step exit update */
  KRS_K_GRAM = 10,          /* Gram blocks of the recycle update */
  KRS_K_ROW_TRANSFORM = 11, /* in-place (U, C) row-block updates */
  KRS_K_OTHER = 12,         /* finishing reductions, copies, casts, coefficient packing */
  KRS_K_SWEEP_STENCIL = 13, /* global Jacobi sweep fused with the matvec of A M^-1 */
  KRS_K_COUNT = 14
} krs_kernel_class;

/* While enabled, every kernel launch of the context is bracketed by two HIP
 * events on the context's stream and its duration and algorithmic bytes
 * (byte model: every array read once and written once) are accumulated per
 * class.  Adds two event records per launch. */
int krs_timing_enable(krs_ctx* ctx, int on);
/* Restricts the timing to the classes whose bit is set in `mask` (bit c for
 * class c; every class by default): launches of other classes get no events
 * and add nothing to the totals but their bytes.  Takes effect from the next
 * launch.  KRS_ERR_ARG for a null context. */
int krs_timing_classes(krs_ctx* ctx, unsigned int mask);
int krs_timing_reset(krs_ctx* ctx);
/* Totals of one class since the last reset: launches, milliseconds, bytes. */
int krs_timing_read(krs_ctx* ctx, int kernel_class, int64_t* launches, double* ms,
                    double* bytes);

/* Library version string. */
const char* krs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* KRS_H */
