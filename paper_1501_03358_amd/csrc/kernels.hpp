// Device kernel launchers for the recycling Krylov solvers (gfx950).
//
// All launchers enqueue on the given stream and return hipGetLastError().
// Reductions are deterministic: a fixed number of blocks (a function of the
// row count only) writes per-block partial sums, and a finishing kernel adds
// them in a fixed order.  Per-thread and per-block sums use the working
// precision T; the cross-block sum and every scalar recurrence use FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace krs {

constexpr int kThreads = 256;      // threads per block (4 wave64)
constexpr int kMaxRedBlocks = 1024;

struct Grid3 {
  int nx, ny, nz;
  int px, py, pz;
  int64_t n;
  int pts = 7;   // stencil points: 7 (orthogonal grids) or 19 (non-orthogonal)
};

// A column set [P1 (n1 columns, ld1) | P2 (n2 columns, ld2)].
template <class T>
struct Cols {
  const T* p1 = nullptr;
  int64_t ld1 = 0;
  int n1 = 0;
  const T* p2 = nullptr;
  int64_t ld2 = 0;
  int n2 = 0;
  int count() const { return n1 + n2; }
};

inline int red_blocks(int64_t n) {
  int64_t b = (n + kThreads * 4 - 1) / (kThreads * 4);
  if (b < 1) b = 1;
  if (b > kMaxRedBlocks) b = kMaxRedBlocks;
  return (int)b;
}

// y = alpha*A x (+ beta*b | + beta*y): mode 0 / 1 / 2.
template <class T>
hipError_t stencil(hipStream_t s, const Grid3& g, const T* bands, const T* x, T* y, double alpha,
                   double beta, const T* b, int mode);
// y = b - A x and per-block partial sums of y^2 (reduction grid red_blocks(n)).
template <class T>
hipError_t residual_norm(hipStream_t s, const Grid3& g, const T* bands, const T* x, const T* b,
                         T* y, T* partials);
// z_out = z_in + omega * (r - A z_in) / diag(A)
template <class T>
hipError_t jacobi_sweep(hipStream_t s, const Grid3& g, const T* bands, const T* r, const T* zin,
                        T* zout, double omega);
// w = A (zl + omega (r - A zl) / diag(A)): one global damped Jacobi sweep
// fused with the following matvec (the swept vector is not stored)
template <class T>
hipError_t sweep_stencil(hipStream_t s, const Grid3& g, const T* bands, const T* r, const T* zl,
                         T* w, double omega);
// z = r / diag(A)
template <class T>
hipError_t point_jacobi(hipStream_t s, const Grid3& g, const T* bands, const T* r, T* z);
// Local Schwarz-Jacobi on every (tile+2)^3 extended tile; writes owned cells.
template <class T>
hipError_t schwarz_local(hipStream_t s, const Grid3& g, int tile, const T* bands, const T* r, T* z,
                         double omega, int sweeps);

// Tiles per brick edge of the coefficient pack: 2 when every tile count is
// even (a brick of 2^3 tiles stores each cell of its extended tiles once),
// else 1 (one extended tile per brick).
inline int schwarz_brick(const Grid3& g, int tile) {
  const int ntx = g.nx / tile, nty = g.ny / tile, ntz = g.nz / tile;
  return (ntx % 2 == 0 && nty % 2 == 0 && ntz % 2 == 0) ? 2 : 1;
}
// Values in the pack: 7 * (brick*tile + 2)^3 per brick.
inline int64_t schwarz_pack_values(const Grid3& g, int tile) {
  const int br = schwarz_brick(g, tile);
  const int64_t nb = (int64_t)(g.nx / tile / br) * (g.ny / tile / br) * (g.nz / tile / br);
  const int64_t eb = (int64_t)br * tile + 2;
  return nb * 7 * eb * eb * eb;
}
// Brick-major coefficients of the local solves: s = omega / a_C and s * a_k
// for every cell of a brick's extended tiles; rebuilt whenever A changes.
template <class T>
hipError_t schwarz_pack(hipStream_t s, const Grid3& g, int tile, const T* bands, T* pk,
                        double omega);
// Local Schwarz-Jacobi from the packed coefficients (omega must match the pack).
template <class T>
hipError_t schwarz_local_packed(hipStream_t s, const Grid3& g, int tile, const T* pk, const T* r,
                                T* z, double omega, int sweeps, bool ssor = false);

// partials[c*nblk + blk] = sum_rows Q_c * w  (c < ncols), then w.w if self_dot
template <class T>
hipError_t block_dot(hipStream_t s, const Cols<T>& Q, const T* w, int64_t n, int self_dot,
                     T* partials, int nblk);
// w_out = (w_in + sgn * Q coef) * (scale ? *scale : 1); w_in may be null (0).
// dots: 0 none; 1 partial |w_out|^2; 2 partial Q^T w_out and |w_out|^2.
// run_if: when not NULL, the launch does nothing unless *run_if != 0 (device flag).
template <class T>
hipError_t block_update(hipStream_t s, const Cols<T>& Q, const double* coef, double sgn,
                        const T* w_in, T* w_out, int64_t n, const double* scale, int dots,
                        T* partials, int nblk, const int* run_if = nullptr);
// partials of Q^T (w - Q coef) and |w - Q coef|^2 without writing anything;
// returns at once when skip != NULL and *skip != 0 (device flag).
template <class T>
hipError_t block_dot_after_update(hipStream_t s, const Cols<T>& Q, const double* coef,
                                  const T* w, int64_t n, T* partials, int nblk,
                                  const int* skip = nullptr);
// Gram: partials[(a*nb + b)*nblk + blk] = sum_rows X_a * Y_b
template <class T>
hipError_t gram(hipStream_t s, const Cols<T>& X, const Cols<T>& Y, int64_t n, T* partials,
                int nblk);
// out[:, o] = sum_c In_c * M[c + nin*o]   (o < nout; in place over In1 allowed)
template <class T>
hipError_t row_transform(hipStream_t s, const Cols<T>& In, const double* M, int nout, T* out,
                         int64_t ldo, int64_t n);

// out[c] = sum_blk partials[c*nblk + blk]   (fixed order, FP64)
template <class T>
hipError_t finish_sum(hipStream_t s, const T* partials, int nblk, int ncols, double* out,
                      const int* run_if = nullptr);
// CGS2 end: h2 = sum(partials[0..ncols)), nrm2 = sum(partials[ncols]);
// hcol[c] = h1[c] + h2[c]; hcol[ncols] = sqrt(nrm2 - |h2|^2) (flag = 1 when the
// Pythagorean form is unreliable and an explicit norm is needed); inv = 1/hcol[ncols].
template <class T>
hipError_t finish_cgs2(hipStream_t s, const T* partials, int nblk, int ncols, const double* h1,
                       double* h2, double* hcol, double* inv, int* flag,
                       const int* skip = nullptr);
// After the first pass with |w|^2 in h1[ncols]: if |w - Q h1|^2 = |w|^2 - |h1|^2
// >= |w|^2 / 2, one pass suffices: hcol = h1 with the norm appended, inv = 1/norm,
// flag = 0, *skip = 1 (the second pass and finish_cgs2 then return at once);
// else *skip = 0.
hipError_t cgs_decide(hipStream_t s, int ncols, const double* h1, double* hcol, double* inv,
                      int* flag, int* skip);

// ---- BiCGStab fused passes (all scalars in the FP64 array `sc`) ----
// scalar slots
// kRho is the rho of the current iteration; the full step stores the next
// one in kRhoNew and the next alpha step takes it over into kRho (so that no
// block of the full-step launch reads a slot that its block 0 writes).
// Breakdown flags: kFlag from the alpha step (1), kFlagT from the omega step
// (2), whose launch may also run the half-step tests that read kFlag.
enum BicgSlot {
  kRho = 0, kRhoNew, kAlpha, kOmega, kBeta, kRtv, kSnorm2, kRnorm2, kTs, kTt, kFlag, kFlagT,
  // device-driven iteration: state (kDone), iterations started, history
  // entries written, absolute stopping and divergence thresholds, and whether
  // the stop came at the half step
  kDone, kIts, kHlen, kTolAbs, kDivAbs, kEndHalf,
  kSlots
};
// kDone values: 0 running, 1 converged at the half step (the exit is applied
// by the launch that sets it, except in the host-tested loop, where the next
// yr pass marks it applied), 2 converged at the full step, 3 breakdown, 4
// diverged or non-finite, 5 early exit applied (set by the pass after the
// one that stored 1).  Every BiCGStab pass returns at once when kDone is
// neither 0 nor, inside the launch that stored it, 1, so iterations enqueued
// after the stop change nothing that the result reads.
enum BicgDone { kRunning = 0, kConvHalf = 1, kConvFull = 2, kBreak = 3, kDiverge = 4, kExited = 5 };
// history ring of the device-driven loop (absolute norms, 2 per iteration)
constexpr int kHistOff = 512, kHistRing = 128;
// BiCGStab pieces; `sums` are finished FP64 dot products.
// The sv pass (v -= C eta1 ; s = r - alpha v ; partial |s|^2) and the yr pass
// (y += alpha p + omega s ; r = s - omega (t - C eta2) ; partials r~.r,
// |r|^2), each with its scalar step in front (alpha, resp. omega and xi):
// every block sums the dot pass's partials `dot` itself and block 0 stores
// the scalars; their own partials go to `partials`, which must not overlap
// `dot`.
template <class T>
hipError_t bicg_sv_fused(hipStream_t s, const Cols<T>& C, const T* r, T* v, T* sv, double* sc,
                         int off_eta1, int off_ctrt, double* sums, int64_t n, const T* dot,
                         T* partials, int nblk);
// With `spart` (the sv pass's |s|^2 partials) the yr pass first takes the
// half-step tests and, on convergence there, applies the exit instead of its
// update; without it (null) the tests ran in bicg_half_exit.
template <class T>
hipError_t bicg_yr_fused(hipStream_t s, const Cols<T>& C, const T* t, const T* sv, const T* p,
                         T* y, T* r, const T* rt, double* sc, int off_eta1, int off_eta2,
                         int off_xi, double* sums, int64_t n, const T* dot, const T* spart,
                         T* partials, int nblk);
// The half-step tests fused with the vector part of the early exit, in a
// launch of their own (the host-tested loop reads the state after it).
template <class T>
hipError_t bicg_half_exit(hipStream_t s, const T* p, T* y, const T* sv, T* r, double* sc,
                          int off_eta1, int off_xi, int kc, const T* partials, int nblk,
                          int64_t n);
// The full step: every block finishes rho = r~.r and |r|^2 from the yr
// pass's partials, forms beta and takes the full-step tests; block 0 stores
// the state; unless the iteration stops there, the blocks then update
// p = r + beta (p - omega v) for the next iteration.
template <class T>
hipError_t bicg_finish_p(hipStream_t s, const T* partials, int nblk, double* sums, double* sc,
                         const T* r, T* p, const T* v, int64_t n);
// hcol_last = sqrt(*nrm2), inv = 1/hcol_last
hipError_t set_norm_from_sum(hipStream_t s, const double* nrm2, double* hcol_last, double* inv,
                             const int* run_if = nullptr);

// ---- device-side Arnoldi cycle state (GMRES / rGCROT), offsets in doubles ----
// stop flag, steps done in the cycle, Arnoldi steps of the solve, last
// estimate, absolute tolerance, step limit, second Gram-Schmidt passes and
// their column count; then g, the rotations, the history ring, Hbar and its
// rotated form R (leading dimension m + 1) and B (leading dimension k_c).
constexpr int kMaxArnM = 64;
enum ArnSlot {
  kArnStop = 0, kArnJ, kArnIts, kArnEst, kArnTolAbs, kArnMaxIts, kArnTwo, kArnTwoCols,
  kArnG = 16, kArnCs = kArnG + kMaxArnM + 16, kArnSn = kArnCs + kMaxArnM,
  kArnHist = kArnSn + kMaxArnM, kArnHistRing = 64,
  kArnH = kArnHist + kArnHistRing, kArnR = kArnH + (kMaxArnM + 1) * kMaxArnM,
  kArnB = kArnR + (kMaxArnM + 1) * kMaxArnM, kArnSize = kArnB + 1024
};
// End of Arnoldi step j (k_c recycle columns, cycle length m) from hcol:
// store the column, Givens rotations, estimate, history and stop state.
// hcol holds k_c + j + 2 values; skip: the step took one Gram-Schmidt pass;
// flag (may be NULL): when set, the step's norm needs an explicit pass, and
// the kernel only records stop state 2 at step j for the host to redo it.
hipError_t arnoldi_givens(hipStream_t s, double* arn, const double* hcol, const int* skip,
                          const int* flag, int j, int kc, int m);

// offsets (doubles) of the rBiCGStab scalar area beyond the BicgSlot slots:
// finished sums, C^T v / C^T t (eta1, eta2), the postponed U-coefficients
// xi, C^T r~, ||b||^2
enum BicgOff {
  kBSums = 32, kBEta1 = 128, kBEta2 = 192, kBXi = 256, kBCtrt = 320, kBNrm = 384, kBNb2 = 385
};
// Starting state of an rBiCGStab solve from its setup sums: xi = -eta1, the
// slots (rho = rho_new = |r_0|^2, omega = 1, beta = 0, the absolute tolerance and
// divergence thresholds from ||b|| = sqrt(sc[kBNb2])); |r_0|^2 is sc[kBNrm]
// after the projection (kc > 0) or ||b||^2 (kc = 0).  The same values the
// host forms and uploads in the single-system driver.
hipError_t bicg_setup(hipStream_t s, double* sc, int kc, double tol, double div_factor);

// ---- grouped rBiCGStab passes over several independent FP32 systems ----
// Every launch covers all systems of a batch: system s owns the block range
// [off[s], off[s+1]) of the grid (each range starts at a multiple of 8 blocks,
// so the XCD mapping within a system is that of a launch of its own), and
// its blocks compute exactly what the same launch of that system alone
// computes (same rows per block, same partial-sum slots, same finishing
// order): each result is bitwise that of the system solved alone.
constexpr int kMaxBatch = 32;
struct BatchSys {
  Grid3 g;
  const float* bands;     // 7 bands
  const float* pk;        // Schwarz local-solve coefficients, bricks of 2^3 tiles of 8^3
  int nbx, nby;           // bricks along x, y
  float omega_l, omega_g;
  int sweeps;             // local Jacobi sweeps
  Cols<float> C;          // recycle space C (C.n1 = k_c columns)
  const float* rt;        // shadow residual r~
  float *r, *p, *v, *sv, *t, *z, *y;
  float* part;            // per-block partial sums of the dot passes
  float* part2;           // |s|^2 partials of the sv pass (after part's)
  float* part3;           // partials of the yr pass (after part2's)
  double* sc;             // scalar area (BicgSlot, BicgOff)
  int nblk;               // blocks of the streaming passes
  int64_t n;
  int64_t ld;             // leading dimension of the vectors
};
struct BatchTable {
  int nsys;
  int pack[kMaxBatch + 1];   // block ranges: four rows per thread (stencil packs)
  int tile[kMaxBatch + 1];   //   two Schwarz tiles (an x-pair) per block
  int pass[kMaxBatch + 1];   //   streaming passes (nblk blocks)
  BatchSys sys[kMaxBatch];
};
// Fills the block ranges of `tb` from its systems (host side).
void batch_layout(BatchTable& tb);
// One rBiCGStab pass sequence for all systems of the table (device copy
// d_tb, host copy tb): the first half (A~ p, C-projection, alpha, s) and
// the second half (A~ s, the half-step tests and exit, omega, y and r
// updates, full-step tests, next p).  The operator is Schwarz-Jacobi (packed Jacobi
// local sweeps, one global sweep) followed by the matvec.  Systems whose stop
// state is set skip every launch.  `nc` is the recycle dimension shared by
// all systems of the table.
hipError_t batch_bicg_first_half(hipStream_t s, const BatchTable* d_tb, const BatchTable& tb,
                                 int nc);
hipError_t batch_bicg_second_half(hipStream_t s, const BatchTable* d_tb, const BatchTable& tb,
                                  int nc);

// misc
template <class T>
hipError_t fill(hipStream_t s, T* x, int64_t n, double v);
template <class T>
hipError_t copy(hipStream_t s, const T* x, T* y, int64_t n);
// x32 = (float)(x64 * (*scale))
hipError_t cast_scale_f64_f32(hipStream_t s, const double* x, float* y, int64_t n,
                              const double* scale);
// x64 += (*scale) * (double)d32
hipError_t axpy_f32_into_f64(hipStream_t s, const float* d, double* x, int64_t n,
                             const double* scale);

}  // namespace krs
