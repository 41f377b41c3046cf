// Host drivers of the Krylov solvers: GMRES(m) (Alg. 1), rGCROT(m,k)/GCRODR
// (Alg. 3) with the harmonic-Ritz recycle update, the thin-QR recycle setup
// (Alg. 3), rBiCGStab with one recycle space (Alg. 4) and FP64
// iterative refinement around an FP32 inner solver.
//
// All vector work runs in the device kernels of kernels.hip; the host keeps
// the small FP64 matrices (Hessenberg columns, Givens rotations, B = C^T A~ V,
// the harmonic-Ritz eigenproblem) and reads a few scalars per step to drive
// convergence tests.  Every solver is right-preconditioned and works on the
// iterate y of A~ y = b with A~ = A M^-1, x = M^-1 y.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dense.hpp"
#include "internal.hpp"

namespace krs {
namespace {

template <class T>
struct Ws {
  // scalar area layout (doubles)
  static constexpr int kH1 = 0, kH2 = 128, kHcol = 256, kInv = 384, kFlagOff = 392;
  // Gram results: up to 64 x 62 and 62 x 62; kM: the recycle update's two
  // coefficient blocks, up to (63 + 64) x 62
  static constexpr int kCoef = 512, kXi = 768, kNrm = 832, kAux = 840;
  static constexpr int kGram1 = 4096, kGram2 = 8192, kM = 12288;
  // device-side Arnoldi cycle state (ArnSlot offsets from here)
  static constexpr int kArn = 20480;
  static_assert(kArn + kArnSize <= kScalarDoubles, "scalar area");
};

// y-space operator A~ = A M^-1 and its pieces
template <class T>
struct Op {
  krs_ctx* ctx;
  const krs_matrix* A;
  const krs_precond* M;
  Grid3 g;
  T* z;     // M^-1 v
  T* tmp;   // preconditioner temporary
  const T* bands() const { return (const T*)A->bands; }

  int minv(const T* r, T* out) { return minv_s(r, out, tmp); }
  // z = M^-1 r using `scratch` (distinct from r and out) as the temporary
  int minv_s(const T* r, T* out, T* scratch) {
    hipStream_t s = ctx->stream;
    T* tmp = scratch;
    const double NW = (double)g.n * sizeof(T);
    if (!M || M->d.type == KRS_PC_NONE) {
      KRS_LAUNCH(ctx, KRS_K_OTHER, 2 * NW, copy<T>(s, r, out, g.n));
      return 0;
    }
    if (M->d.type == KRS_PC_JACOBI) {
      KRS_LAUNCH(ctx, KRS_K_JACOBI_SWEEP, 3 * NW, point_jacobi<T>(s, g, bands(), r, out));
      return 0;
    }
    const int gs = M->d.global_sweeps;
    T* first = (gs % 2 == 0) ? out : tmp;
    const double PW = (double)(g.pts + 2) * NW;   // bands, input and output
    if (M->d.local_sweeps > 0 && M->pack) {
      KRS_LAUNCH(ctx, KRS_K_SCHWARZ_LOCAL, PW,
                 schwarz_local_packed<T>(s, g, M->d.tile, (const T*)M->pack, r, first,
                                         M->d.omega_local, M->d.local_sweeps,
                                         M->d.local_solver == KRS_LOCAL_SSOR));
    } else if (M->d.local_sweeps > 0) {
      KRS_LAUNCH(ctx, KRS_K_SCHWARZ_LOCAL, PW,
                 schwarz_local<T>(s, g, M->d.tile, bands(), r, first, M->d.omega_local,
                                  M->d.local_sweeps));
    } else {
      KRS_LAUNCH(ctx, KRS_K_OTHER, NW, fill<T>(s, first, g.n, 0.0));
    }
    T* cur = first;
    for (int i = 0; i < gs; ++i) {
      T* nxt = (cur == out) ? tmp : out;
      KRS_LAUNCH(ctx, KRS_K_JACOBI_SWEEP, PW + NW,
                 jacobi_sweep<T>(s, g, bands(), r, cur, nxt, M->d.omega_global));
      cur = nxt;
    }
    return 0;
  }
  // w = A M^-1 v
  // (w, not yet written, is the preconditioner's temporary)
  int apply(const T* v, T* w) {
    if (M && M->d.type == KRS_PC_SCHWARZ_JACOBI && M->d.global_sweeps == 1 &&
        g.n >= kFuseMinN && g.pts == 7) {
      // local solves into z, then the global sweep and the matvec in one pass
      // (on smaller grids the two streaming kernels are as fast: the fused
      // pass recomputes two halo planes per column chunk)
      hipStream_t s = ctx->stream;
      const double NW = (double)g.n * sizeof(T);
      if (M->d.local_sweeps > 0 && M->pack) {
        KRS_LAUNCH(ctx, KRS_K_SCHWARZ_LOCAL, 9 * NW,
                   schwarz_local_packed<T>(s, g, M->d.tile, (const T*)M->pack, v, z,
                                           M->d.omega_local, M->d.local_sweeps,
                                           M->d.local_solver == KRS_LOCAL_SSOR));
      } else if (M->d.local_sweeps > 0) {
        KRS_LAUNCH(ctx, KRS_K_SCHWARZ_LOCAL, 9 * NW,
                   schwarz_local<T>(s, g, M->d.tile, bands(), v, z, M->d.omega_local,
                                    M->d.local_sweeps));
      } else {
        KRS_LAUNCH(ctx, KRS_K_OTHER, NW, fill<T>(s, z, g.n, 0.0));
      }
      KRS_LAUNCH(ctx, KRS_K_SWEEP_STENCIL, 10 * NW,
                 sweep_stencil<T>(s, g, bands(), v, z, w, M->d.omega_global));
      return 0;
    }
    int rc = minv_s(v, z, w);
    if (rc) return rc;
    KRS_LAUNCH(ctx, KRS_K_STENCIL, (g.pts + 2.0) * g.n * sizeof(T),
               stencil<T>(ctx->stream, g, bands(), z, w, 1.0, 0.0, nullptr, 0));
    return 0;
  }
};

int read_dev(krs_ctx* ctx, const double* src, int count) {
  KRS_CHECK_HIP(ctx, hipMemcpyAsync(ctx->pin, src, sizeof(double) * count, hipMemcpyDeviceToHost,
                                    ctx->stream));
  KRS_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  timing_flush(ctx);
  return 0;
}

int upload(krs_ctx* ctx, double* dst, const double* src, int count) {
  double* stage = ctx->pin + kPinDoubles / 2;
  KRS_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::memcpy(stage, src, sizeof(double) * count);
  KRS_CHECK_HIP(ctx, hipMemcpyAsync(dst, stage, sizeof(double) * count, hipMemcpyHostToDevice,
                                    ctx->stream));
  KRS_CHECK_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return 0;
}

template <class T>
Cols<T> cols(const T* p1, int64_t ld1, int n1, const T* p2 = nullptr, int64_t ld2 = 0, int n2 = 0) {
  Cols<T> c;
  c.p1 = p1;
  c.ld1 = ld1;
  c.n1 = n1;
  c.p2 = p2;
  c.ld2 = ld2;
  c.n2 = n2;
  return c;
}

// ||w||^2 -> host
template <class T>
int norm2(krs_ctx* ctx, const T* w, int64_t n, T* part, double* d_out, double& out) {
  const int nblk = red_blocks(n);
  KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, (double)n * sizeof(T),
             block_dot<T>(ctx->stream, Cols<T>{}, w, n, 1, part, nblk));
  KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(ctx->stream, part, nblk, 1, d_out));
  int rc = read_dev(ctx, d_out, 1);
  if (rc) return rc;
  out = ctx->pin[0];
  return 0;
}

void init_stats(krs_stats* st) {
  if (!st) return;
  std::memset(st, 0, sizeof(*st));
  st->rel_res_true = NAN;
  st->rel_res_est = NAN;
}

template <class T>
size_t ws_gmres(int64_t n, int m) {
  Carver c(nullptr, 0);
  const int64_t ld = vec_ld(n);
  c.vec<T>(ld * (m + 1));
  c.vec<T>(ld);
  c.vec<T>(ld);
  c.take(partials_bytes(sizeof(T)));
  c.vec<double>(kScalarDoubles);
  c.vec<T>(ld);   // left preconditioning: M^-1 b
  c.vec<T>(ld);   // left preconditioning: preconditioner temporary
  return c.off;
}

template <class T>
size_t ws_bicg(int64_t n) {
  Carver c(nullptr, 0);
  const int64_t ld = vec_ld(n);
  for (int i = 0; i < 8; ++i) c.vec<T>(ld);
  c.take(partials_bytes(sizeof(T)));
  c.vec<double>(kScalarDoubles);
  return c.off;
}

size_t ws_ir(int64_t n, int m) {
  Carver c(nullptr, 0);
  const int64_t ld = vec_ld(n);
  c.take(std::max(ws_gmres<float>(n, m), ws_bicg<float>(n)));
  c.vec<double>(ld);
  c.vec<float>(ld);
  c.vec<float>(ld);
  c.take(partials_bytes(sizeof(double)));
  c.vec<double>(kScalarDoubles);
  return c.off;
}

// ---------------------------------------------------------------------------
// recycle-space update at a cycle end of Alg. 3 (harmonic Ritz, GCRODR rule)
// ---------------------------------------------------------------------------
template <class T>
int harmonic_update(krs_ctx* ctx, krs_recycle* rec, const T* V, int64_t ld, int jj,
                    const std::vector<double>& Hbar, int ldh, const std::vector<double>& Bm,
                    int ldb, int k, T* part, double* sc, krs_stats* st) {
  hipStream_t s = ctx->stream;
  const int64_t n = rec->n;
  const int kc = rec->dim;
  const int ng = kc + jj, mg = ng + 1;
  if (jj == 0) return 0;
  T* U = (T*)rec->U;
  T* C = (T*)rec->C;
  const int64_t ldr = rec->ld;
  std::vector<double> dvec(kc), CtU((size_t)kc * kc), VtU((size_t)(jj + 1) * kc);
  if (kc > 0) {
    const int na = kc + jj + 1;
    const double NW = (double)n * sizeof(T);
    const int gb1 = gram_blocks(na, kc, n), gb2 = gram_blocks(kc, kc, n);
    KRS_LAUNCH(ctx, KRS_K_GRAM, NW * (2 * kc + jj + 1),
               gram<T>(s, cols<T>(C, ldr, kc, V, ld, jj + 1), cols<T>(U, ldr, kc), n, part, gb1));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, gb1, na * kc, sc + Ws<T>::kGram1));
    KRS_LAUNCH(ctx, KRS_K_GRAM, NW * kc,
               gram<T>(s, cols<T>(U, ldr, kc), cols<T>(U, ldr, kc), n, part, gb2));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, gb2, kc * kc, sc + Ws<T>::kGram2));
    int rc = read_dev(ctx, sc + Ws<T>::kGram1, na * kc);
    if (rc) return rc;
    for (int a = 0; a < kc; ++a)
      for (int b = 0; b < kc; ++b) CtU[a + (size_t)kc * b] = ctx->pin[a * kc + b];
    for (int r = 0; r <= jj; ++r)
      for (int b = 0; b < kc; ++b) VtU[r + (size_t)(jj + 1) * b] = ctx->pin[(kc + r) * kc + b];
    rc = read_dev(ctx, sc + Ws<T>::kGram2, kc * kc);
    if (rc) return rc;
    for (int i = 0; i < kc; ++i) dvec[i] = 1.0 / std::sqrt(ctx->pin[i * kc + i]);
  }
  Timer te;
  // G = [[D, B], [0, Hbar]]
  std::vector<double> G((size_t)mg * ng, 0.0);
  auto gref = [&](int i, int j) -> double& { return G[i + (size_t)mg * j]; };
  for (int i = 0; i < kc; ++i) gref(i, i) = dvec[i];
  for (int j = 0; j < jj; ++j)
    for (int i = 0; i < kc; ++i) gref(i, kc + j) = Bm[i + (size_t)ldb * j];
  for (int j = 0; j < jj; ++j)
    for (int i = 0; i <= jj; ++i) gref(kc + i, kc + j) = Hbar[i + (size_t)ldh * j];
  std::vector<double> P;
  int kk = 0, ties = 0;
  if (ng <= k) {
    kk = ng;
    P.assign((size_t)ng * ng, 0.0);
    for (int i = 0; i < ng; ++i) P[i + (size_t)ng * i] = 1.0;
  } else {
    // F = W^T V^ = [[C^T U D, 0], [V_{j+1}^T U D, I~]]
    std::vector<double> F((size_t)mg * ng, 0.0);
    for (int b = 0; b < kc; ++b) {
      for (int a = 0; a < kc; ++a) F[a + (size_t)mg * b] = CtU[a + (size_t)kc * b] * dvec[b];
      for (int r = 0; r <= jj; ++r)
        F[kc + r + (size_t)mg * b] = VtU[r + (size_t)(jj + 1) * b] * dvec[b];
    }
    for (int c = 0; c < jj; ++c) F[kc + c + (size_t)mg * (kc + c)] = 1.0;
    if (!dense::harmonic_ritz_select(mg, ng, G.data(), F.data(), k, P, kk, ties)) {
      if (st) st->host_eig_ms += te.ms();
      return set_err(ctx, KRS_ERR_EIG, "harmonic Ritz eigen-solver failed");
    }
  }
  // [Q, R] = qr(G P);  U <- V^ P R^-1 (D folded in), C <- W^ Q
  std::vector<double> GP((size_t)mg * kk, 0.0);
  for (int c = 0; c < kk; ++c)
    for (int j = 0; j < ng; ++j) {
      const double pj = P[j + (size_t)ng * c];
      if (pj == 0) continue;
      for (int i = 0; i < mg; ++i) GP[i + (size_t)mg * c] += G[i + (size_t)mg * j] * pj;
    }
  std::vector<double> Q((size_t)mg * kk), R((size_t)kk * kk), Ri((size_t)kk * kk);
  dense::qr_thin(mg, kk, GP.data(), Q.data(), R.data());
  if (!dense::upper_inverse(kk, R.data(), Ri.data())) {
    if (st) st->host_eig_ms += te.ms();
    return set_err(ctx, KRS_ERR_EIG, "recycle update: singular R");
  }
  std::vector<double> Mu((size_t)ng * kk, 0.0);
  for (int c = 0; c < kk; ++c)
    for (int i = 0; i < ng; ++i) {
      double sum = 0;
      for (int q = 0; q <= c; ++q) sum += P[i + (size_t)ng * q] * Ri[q + (size_t)kk * c];
      Mu[i + (size_t)ng * c] = (i < kc ? dvec[i] : 1.0) * sum;
    }
  if (st) {
    st->host_eig_ms += te.ms();
    st->eig_ties += ties;
  }
  std::vector<double> both(Mu);
  both.insert(both.end(), Q.begin(), Q.end());
  int rc = upload(ctx, sc + Ws<T>::kM, both.data(), (int)both.size());
  if (rc) return rc;
  const double NWt = (double)n * sizeof(T);
  KRS_LAUNCH(ctx, KRS_K_ROW_TRANSFORM, NWt * (kc + jj + kk),
             row_transform<T>(s, cols<T>(U, ldr, kc, V, ld, jj), sc + Ws<T>::kM, kk, U, ldr, n));
  KRS_LAUNCH(ctx, KRS_K_ROW_TRANSFORM, NWt * (kc + jj + 1 + kk),
             row_transform<T>(s, cols<T>(C, ldr, kc, V, ld, jj + 1),
                              sc + Ws<T>::kM + (size_t)ng * kk, kk, C, ldr, n));
  rec->dim = kk;
  return 0;
}

template <class T>
int cholqr2(krs_ctx* ctx, krs_recycle* rec, T* part, double* sc, const char* fail);

struct GcrotPar {
  int kt, s, p;
};

// ---------------------------------------------------------------------------
// recycle-space update at a cycle end of Alg. 3 (GCROT rule; a reading, since the
// paper names the rule and its parameters only): the outer space gains the
// cycle's correction y and the p directions of this cycle's selection space
// (images of the last s inner vectors) closest to the previous cycle's one
// (prevQ, prev_dim columns, kept within a solve); above k it is first cut
// to kt columns, those closest to A~ range(V_j); Cholesky-QR twice.
// ---------------------------------------------------------------------------
template <class T>
int gcrot_update(krs_ctx* ctx, krs_recycle* rec, const T* V, int64_t ld, int jj,
                 const std::vector<double>& Hbar, int ldh, const std::vector<double>& Bm,
                 int ldb, const std::vector<double>& yv, int k, const GcrotPar& par, T* prevQ,
                 int& prev_dim, T* part, double* sc, krs_stats* st) {
  hipStream_t s = ctx->stream;
  const int64_t n = rec->n;
  const int kc = rec->dim;
  if (jj == 0) return 0;
  T* U = (T*)rec->U;
  T* C = (T*)rec->C;
  const int64_t ldr = rec->ld;
  const int mg = jj + 1;
  const int sj = std::min(par.s, jj);
  const double NW = (double)n * sizeof(T);
  const bool select = prev_dim > 0 && par.p > 0;
  std::vector<double> PV;
  if (select) {
    // prev^T V_{j+1}: prev_dim x (jj + 1)
    const int gb = gram_blocks(prev_dim, mg, n);
    KRS_LAUNCH(ctx, KRS_K_GRAM, NW * (prev_dim + mg),
               gram<T>(s, cols<T>(prevQ, ld, prev_dim), cols<T>(V, ld, mg), n, part, gb));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0,
               finish_sum<T>(s, part, gb, prev_dim * mg, sc + Ws<T>::kGram1));
    int rc = read_dev(ctx, sc + Ws<T>::kGram1, prev_dim * mg);
    if (rc) return rc;
    PV.assign(ctx->pin, ctx->pin + (size_t)prev_dim * mg);   // PV[a * mg + b]
  }
  Timer te;
  int ties = 0;
  auto hb = [&](int i, int j) { return Hbar[i + (size_t)ldh * j]; };
  // selection space of this cycle: Hbar[:, jj-sj:jj] = Qs Rs
  std::vector<double> S((size_t)mg * sj), Qs((size_t)mg * sj), Rs((size_t)sj * sj);
  for (int c = 0; c < sj; ++c)
    for (int i = 0; i < mg; ++i) S[i + (size_t)mg * c] = hb(i, jj - sj + c);
  dense::qr_thin(mg, sj, S.data(), Qs.data(), Rs.data());
  // candidate coefficient vectors (length jj): y, then the selected ones
  std::vector<std::vector<double>> cand;
  cand.push_back(std::vector<double>(yv.begin(), yv.begin() + jj));
  if (select) {
    // cosines: singular values of Mx = (prev^T V) Qs; right singular vectors
    // from the eigenvectors of Mx^T Mx
    std::vector<double> Mx((size_t)prev_dim * sj, 0.0), MtM((size_t)sj * sj, 0.0), w, Z;
    for (int a = 0; a < prev_dim; ++a)
      for (int c = 0; c < sj; ++c) {
        double sum = 0;
        for (int b = 0; b < mg; ++b) sum += PV[(size_t)a * mg + b] * Qs[b + (size_t)mg * c];
        Mx[a + (size_t)prev_dim * c] = sum;
      }
    for (int c1 = 0; c1 < sj; ++c1)
      for (int c2 = 0; c2 < sj; ++c2) {
        double sum = 0;
        for (int a = 0; a < prev_dim; ++a)
          sum += Mx[a + (size_t)prev_dim * c1] * Mx[a + (size_t)prev_dim * c2];
        MtM[c1 + (size_t)sj * c2] = sum;
      }
    if (!dense::sym_eig(sj, MtM.data(), w, Z)) {
      if (st) st->host_eig_ms += te.ms();
      return set_err(ctx, KRS_ERR_EIG, "GCROT selection: eigen-solver failed");
    }
    // only directions with a nonzero cosine are defined
    auto sv = [&](int i) { return i < std::min(prev_dim, sj) ? std::sqrt(std::max(w[i], 0.0)) : 0.0; };
    // with the cycle's correction, at most k new columns
    int npick = std::min(std::min(par.p, sj), std::min(prev_dim, k - 1));
    while (npick > 0 && sv(npick - 1) <= 1e-12) --npick;
    if (npick > 0 && npick < std::min(prev_dim, sj) &&
        (sv(npick - 1) - sv(npick)) / sv(npick - 1) < 1e-8)
      ++ties;
    for (int i = 0; i < npick; ++i) {
      std::vector<double> r(Z.begin() + (size_t)sj * i, Z.begin() + (size_t)sj * (i + 1));
      int big = 0;
      for (int t = 1; t < sj; ++t)
        if (std::fabs(r[t]) > std::fabs(r[big])) big = t;
      if (r[big] < 0)
        for (double& v : r) v = -v;
      std::vector<double> g(jj, 0.0), sol(sj);
      dense::upper_solve(sj, Rs.data(), sj, r.data(), sol.data());
      for (int t = 0; t < sj; ++t) g[jj - sj + t] = sol[t];
      cand.push_back(g);
    }
  }
  // orthonormalise the images Hbar g in order (Gram-Schmidt twice, dropping
  // dependent ones): Hbar Gc = Qn
  std::vector<std::vector<double>> Qn, Gc;
  for (const auto& g0 : cand) {
    std::vector<double> g = g0, h(mg, 0.0);
    for (int i = 0; i < mg; ++i) {
      double sum = 0;
      for (int j = 0; j < jj; ++j) sum += hb(i, j) * g[j];
      h[i] = sum;
    }
    double h0 = 0;
    for (double v : h) h0 += v * v;
    h0 = std::sqrt(h0);
    if (h0 == 0) continue;
    for (int pass = 0; pass < 2; ++pass)
      for (size_t l = 0; l < Qn.size(); ++l) {
        double t = 0;
        for (int i = 0; i < mg; ++i) t += Qn[l][i] * h[i];
        for (int i = 0; i < mg; ++i) h[i] -= t * Qn[l][i];
        for (int j = 0; j < jj; ++j) g[j] -= t * Gc[l][j];
      }
    double nrm = 0;
    for (double v : h) nrm += v * v;
    nrm = std::sqrt(nrm);
    if (nrm <= 1e-10 * h0) continue;
    for (double& v : h) v /= nrm;
    for (double& v : g) v /= nrm;
    Qn.push_back(h);
    Gc.push_back(g);
  }
  const int q = (int)Qn.size();
  // cut of the outer space: keep the columns closest to A~ range(V_j)
  std::vector<int> keep;
  for (int i = 0; i < kc; ++i) keep.push_back(i);
  if (kc + q > k) {
    const int ktp = std::max(0, std::min(par.kt, k - q));
    const int mk = kc + mg;
    std::vector<double> K((size_t)mk * jj), Qk((size_t)mk * jj), Rk((size_t)jj * jj);
    for (int j = 0; j < jj; ++j) {
      for (int i = 0; i < kc; ++i) K[i + (size_t)mk * j] = Bm[i + (size_t)ldb * j];
      for (int i = 0; i < mg; ++i) K[kc + i + (size_t)mk * j] = hb(i, j);
    }
    dense::qr_thin(mk, jj, K.data(), Qk.data(), Rk.data());
    std::vector<double> cosv(kc);
    for (int i = 0; i < kc; ++i) {
      double sum = 0;
      for (int j = 0; j < jj; ++j) sum += Qk[i + (size_t)mk * j] * Qk[i + (size_t)mk * j];
      cosv[i] = std::sqrt(sum);
    }
    std::vector<int> order(kc);
    for (int i = 0; i < kc; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
      return cosv[a] != cosv[b] ? cosv[a] > cosv[b] : a > b;
    });
    if (ktp > 0 && ktp < kc && cosv[order[ktp - 1]] > 0 &&
        (cosv[order[ktp - 1]] - cosv[order[ktp]]) / cosv[order[ktp - 1]] < 1e-8)
      ++ties;
    keep.assign(order.begin(), order.begin() + ktp);
    std::sort(keep.begin(), keep.end());
  }
  const int nk = (int)keep.size(), nout = nk + q;
  if (nout > k || nout > rec->kmax)
    return set_err(ctx, KRS_ERR_STATE, "GCROT update: outer space above k");
  // U <- [U_keep, (V_j - U B) Gc] from In = [U, V_j]; C <- [C_keep, V_{j+1} Qn]
  // from In = [C, V_{j+1}]; the next selection basis V_{j+1} Qs into prevQ
  const int nu = kc + jj, ncin = kc + mg;
  std::vector<double> Mu((size_t)nu * nout, 0.0), Mc((size_t)ncin * nout, 0.0);
  for (int o = 0; o < nk; ++o) {
    Mu[keep[o] + (size_t)nu * o] = 1.0;
    Mc[keep[o] + (size_t)ncin * o] = 1.0;
  }
  for (int l = 0; l < q; ++l) {
    const int o = nk + l;
    for (int c = 0; c < kc; ++c) {
      double sum = 0;
      for (int j = 0; j < jj; ++j) sum += Bm[c + (size_t)ldb * j] * Gc[l][j];
      Mu[c + (size_t)nu * o] = -sum;
    }
    for (int j = 0; j < jj; ++j) Mu[kc + j + (size_t)nu * o] = Gc[l][j];
    for (int i = 0; i < mg; ++i) Mc[kc + i + (size_t)ncin * o] = Qn[l][i];
  }
  if (st) {
    st->host_eig_ms += te.ms();
    st->eig_ties += ties;
  }
  std::vector<double> all(Mu);
  all.insert(all.end(), Mc.begin(), Mc.end());
  all.insert(all.end(), Qs.begin(), Qs.end());
  int rc = upload(ctx, sc + Ws<T>::kM, all.data(), (int)all.size());
  if (rc) return rc;
  const double* dMu = sc + Ws<T>::kM;
  const double* dMc = dMu + Mu.size();
  const double* dQs = dMc + Mc.size();
  KRS_LAUNCH(ctx, KRS_K_ROW_TRANSFORM, NW * (mg + sj),
             row_transform<T>(s, cols<T>(V, ld, mg), dQs, sj, prevQ, ld, n));
  if (nout > 0) {
    KRS_LAUNCH(ctx, KRS_K_ROW_TRANSFORM, NW * (nu + nout),
               row_transform<T>(s, cols<T>(U, ldr, kc, V, ld, jj), dMu, nout, U, ldr, n));
    KRS_LAUNCH(ctx, KRS_K_ROW_TRANSFORM, NW * (ncin + nout),
               row_transform<T>(s, cols<T>(C, ldr, kc, V, ld, mg), dMc, nout, C, ldr, n));
  }
  prev_dim = sj;
  rec->dim = nout;
  return cholqr2<T>(ctx, rec, part, sc, "GCROT update: C is rank deficient");
}

// ---------------------------------------------------------------------------
// GMRES(m) and rGCROT(m,k)
// ---------------------------------------------------------------------------
template <class T>
int gmres_rgcrot_t(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                   bool update, const T* b, T* x, const krs_opts* o, void* ws, size_t wsb,
                   krs_stats* st) {
  Timer tm;
  const double bytes0 = ctx->bytes;
  hipStream_t s = ctx->stream;
  const int64_t n = A->n;
  const int64_t ld = vec_ld(n);
  const int m = o->m;
  const double tol = o->tol;
  const int64_t maxit = o->max_matvecs > 0 ? o->max_matvecs : 2000;
  Carver cv(ws, wsb);
  T* V = cv.vec<T>(ld * (m + 1));
  T* z = cv.vec<T>(ld);
  T* w = cv.vec<T>(ld);  // A~ v_j; doubles as the preconditioner temporary
  T* part = (T*)cv.take(partials_bytes(sizeof(T)));
  double* sc = cv.vec<double>(kScalarDoubles);
  const bool left = (o->flags & KRS_FLAG_LEFT_PRECOND) != 0 && M && M->d.type != KRS_PC_NONE;
  T* bl = left ? cv.vec<T>(ld) : nullptr;     // M^-1 b
  T* ptmp = left ? cv.vec<T>(ld) : nullptr;   // preconditioner temporary
  // GCROT rule: the previous cycle's selection space (up to m columns)
  const bool gcrot = update && rec && o->recycle_rule == KRS_RECYCLE_GCROT;
  T* prevQ = gcrot ? cv.vec<T>(ld * m) : nullptr;
  int prev_dim = 0;
  const GcrotPar gpar{o->gcrot_kt > 0 ? o->gcrot_kt : std::max(1, o->k - 10),
                      o->gcrot_s > 0 ? o->gcrot_s : std::max(1, m / 2), o->gcrot_p};
  if (!ws || !cv.ok) return set_err(ctx, KRS_ERR_WORKSPACE, "workspace missing or too small");
  double* d_h1 = sc + Ws<T>::kH1;
  double* d_h2 = sc + Ws<T>::kH2;
  double* d_hcol = sc + Ws<T>::kHcol;
  double* d_inv = sc + Ws<T>::kInv;
  int* d_flag = (int*)(sc + Ws<T>::kFlagOff);
  int* d_skip = d_flag + 1;
  int64_t n_one_pass = 0, n_two_pass = 0;
  double* d_coef = sc + Ws<T>::kCoef;
  double* d_xi = sc + Ws<T>::kXi;
  double* d_nrm = sc + Ws<T>::kNrm;
  const int nblk = red_blocks(n);
  Op<T> op{ctx, A, M, grid3(A), z, w};
  const double NW = (double)n * sizeof(T);
  // the operator of the iteration: A M^-1 (right) or M^-1 A (left, into w
  // through z, with ptmp as the preconditioner's temporary)
  auto apply = [&](const T* v, T* out) -> int {
    if (!left) return op.apply(v, out);
    KRS_LAUNCH(ctx, KRS_K_STENCIL, (op.g.pts + 2) * NW,
               stencil<T>(s, op.g, op.bands(), v, z, 1.0, 0.0, nullptr, 0));
    return op.minv_s(z, out, ptmp);
  };

  init_stats(st);
  const T* b_orig = b;
  double nb_orig = 0;
  if (left) {
    double nbo2 = 0;
    int e = norm2<T>(ctx, b, n, part, d_nrm, nbo2);
    if (e) return e;
    nb_orig = std::sqrt(nbo2);
    e = op.minv_s(b, bl, ptmp);   // the system M^-1 A x = M^-1 b
    if (e) return e;
    b = bl;
  }
  double nb2 = 0;
  int rc = norm2<T>(ctx, b, n, part, d_nrm, nb2);
  if (rc) return rc;
  const double nb = std::sqrt(nb2);
  if (nb == 0 || !std::isfinite(nb)) {
    KRS_LAUNCH(ctx, KRS_K_OTHER, NW, fill<T>(s, x, n, 0.0));
    KRS_CHECK_HIP(ctx, hipStreamSynchronize(s));
    timing_flush(ctx);
    if (st) {
      st->status = std::isfinite(nb) ? KRS_OK : KRS_DIVERGED;
      st->rel_res_true = 0;
      st->time_ms = tm.ms();
    }
    return std::isfinite(nb) ? KRS_OK : KRS_DIVERGED;
  }
  T* U = rec ? (T*)rec->U : nullptr;
  T* C = rec ? (T*)rec->C : nullptr;
  const int64_t ldr = rec ? rec->ld : 0;
  int kc = rec ? rec->dim : 0;
  T* r0 = V;  // the residual lives in the first basis column
  double rho2 = 0;
  // project b against C: xi = C^T b, r = b - C xi, y = U xi
  if (kc > 0) {
    KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW * (kc + 1),
               block_dot<T>(s, cols<T>(C, ldr, kc), b, n, 0, part, nblk));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, kc, d_xi));
    KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (kc + 2),
               block_update<T>(s, cols<T>(C, ldr, kc), d_xi, -1.0, b, r0, n, nullptr, 1, part,
                               nblk));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, 1, d_nrm));
    KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (kc + 1),
               block_update<T>(s, cols<T>(U, ldr, kc), d_xi, 1.0, nullptr, x, n, nullptr, 0, part,
                               nblk));
    rc = read_dev(ctx, d_nrm, 1);
    if (rc) return rc;
    rho2 = ctx->pin[0];
  } else {
    KRS_LAUNCH(ctx, KRS_K_OTHER, 2 * NW, copy<T>(s, b, r0, n));
    KRS_LAUNCH(ctx, KRS_K_OTHER, NW, fill<T>(s, x, n, 0.0));
    rho2 = nb2;
  }
  double rho = std::sqrt(rho2);

  const int ldh = m + 1;
  const int ldb = kMaxK;
  std::vector<double> Hbar((size_t)ldh * m), Rr((size_t)ldh * m), Bm((size_t)ldb * m);
  std::vector<double> cs(m), sn(m), gv(m + 1), hc(m + 1), yv(m), coef(m + kMaxK);
  int64_t its = 0, mv = 0, cycles = 0, hlen = 0;
  int status = KRS_NOT_CONVERGED;
  double est = rho;
  const bool trust_est = (o->flags & KRS_FLAG_TRUST_ESTIMATE) != 0;
  // host-tested loop (one read per step) or device-driven batches of steps
  const bool host_loop = (o->flags & KRS_FLAG_HOST_LOOP) != 0;
  double* d_arn = sc + Ws<T>::kArn;
  const int bcap = n <= (int64_t(1) << 18) ? 32 : (n <= (int64_t(1) << 21) ? 8 : 4);
  int batch = std::min(2, bcap);
  bool est_converged = false;
  while (rho > tol * nb && its < maxit && !est_converged) {
    kc = rec ? rec->dim : 0;
    // v_1 = r / rho
    const double inv_rho = 1.0 / rho;
    rc = upload(ctx, d_inv, &inv_rho, 1);
    if (rc) return rc;
    KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, 2 * NW,
               block_update<T>(s, Cols<T>{}, nullptr, 0.0, r0, V, n, d_inv, 0, part, nblk));
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = rho;
    std::fill(Hbar.begin(), Hbar.end(), 0.0);
    std::fill(Bm.begin(), Bm.end(), 0.0);
    int jj = 0;
    // one Arnoldi step: w = A~ v_j, Gram-Schmidt against [C, V_j] (second
    // pass on the device's decision), v_{j+1} = (w - Q h) / h_{j+1,j}.  With
    // `dev` the explicit-norm fallback is enqueued as launches that do
    // nothing unless the device flag asks for them; otherwise the host reads
    // the flag and launches them when needed.
    auto step = [&](int j, bool dev) -> int {
      T* vj = V + (int64_t)j * ld;
      T* vn = V + (int64_t)(j + 1) * ld;
      int e = apply(vj, w);
      if (e) return e;
      const int ncols = kc + j + 1;
      const Cols<T> Q = cols<T>(C, ldr, kc, V, ld, j + 1);
      KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW * (ncols + 1), block_dot<T>(s, Q, w, n, 1, part, nblk));
      KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, ncols + 1, d_h1));
      KRS_LAUNCH(ctx, KRS_K_OTHER, 0, cgs_decide(s, ncols, d_h1, d_hcol, d_inv, d_flag, d_skip));
      KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT2, 0,
                 block_dot_after_update<T>(s, Q, d_h1, w, n, part, nblk, d_skip));
      KRS_LAUNCH(ctx, KRS_K_OTHER, 0,
                 finish_cgs2<T>(s, part, nblk, ncols, d_h1, d_h2, d_hcol, d_inv, d_flag, d_skip));
      KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (ncols + 2),
                 block_update<T>(s, Q, d_hcol, -1.0, w, vn, n, d_inv, 0, part, nblk));
      if (dev)
        KRS_LAUNCH(ctx, KRS_K_OTHER, 0,
                   arnoldi_givens(s, d_arn, d_hcol, d_skip, d_flag, j, kc, m));
      return 0;
    };
    // the explicit norm of w - Q h and the rescale of v_{j+1}, for a step
    // whose norm from the Pythagorean identity is unreliable (flag set)
    auto explicit_norm = [&](int j) -> int {
      const int ncols = kc + j + 1;
      T* vn = V + (int64_t)(j + 1) * ld;
      const Cols<T> Q = cols<T>(C, ldr, kc, V, ld, j + 1);
      KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (ncols + 2),
                 block_update<T>(s, Q, d_hcol, -1.0, w, vn, n, nullptr, 1, part, nblk));
      KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, 1, d_nrm));
      KRS_LAUNCH(ctx, KRS_K_OTHER, 0, set_norm_from_sum(s, d_nrm, d_hcol + ncols, d_inv));
      KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, 2 * NW,
                 block_update<T>(s, Cols<T>{}, nullptr, 0.0, vn, vn, n, d_inv, 0, part, nblk));
      return 0;
    };
    if (host_loop) {
      for (int j = 0; j < m; ++j) {
        rc = step(j, false);
        if (rc) return rc;
        ++its;
        ++mv;
        const int ncols = kc + j + 1;
        rc = read_dev(ctx, sc, Ws<T>::kFlagOff + 1);
        if (rc) return rc;
        std::vector<double> hv(ctx->pin + Ws<T>::kHcol, ctx->pin + Ws<T>::kHcol + ncols + 1);
        int flag = *(int*)(ctx->pin + Ws<T>::kFlagOff);
        const int skipped = ((int*)(ctx->pin + Ws<T>::kFlagOff))[1];
        if (!skipped) timing_add_bytes(ctx, KRS_K_BLOCK_DOT2, NW * (ncols + 1));
        ++(skipped ? n_one_pass : n_two_pass);
        if (flag) {
          // norm from the Pythagorean identity unreliable: recompute explicitly
          rc = explicit_norm(j);
          if (rc) return rc;
          rc = read_dev(ctx, d_hcol + ncols, 1);
          if (rc) return rc;
          hv[ncols] = ctx->pin[0];
        }
        for (int i = 0; i < kc; ++i) Bm[i + (size_t)ldb * j] = hv[i];
        for (int i = 0; i <= j; ++i) Hbar[i + (size_t)ldh * j] = hv[kc + i];
        Hbar[(j + 1) + (size_t)ldh * j] = hv[ncols];
        // Givens rotations for the least-squares problem of the cycle (the
        // same arithmetic, term by term, as the device-side step end)
        for (int i = 0; i <= j + 1; ++i) hc[i] = Hbar[i + (size_t)ldh * j];
        for (int i = 0; i < j; ++i) {
          const double a = hc[i], bb = hc[i + 1];
          hc[i] = cs[i] * a + sn[i] * bb;
          hc[i + 1] = -sn[i] * a + cs[i] * bb;
        }
        const double a = hc[j], bb = hc[j + 1];
        const double rr = std::sqrt(a * a + bb * bb);
        cs[j] = rr > 0 ? a / rr : 1.0;
        sn[j] = rr > 0 ? bb / rr : 0.0;
        hc[j] = rr;
        hc[j + 1] = 0;
        gv[j + 1] = -sn[j] * gv[j];
        gv[j] = cs[j] * gv[j];
        for (int i = 0; i <= j + 1; ++i) Rr[i + (size_t)ldh * j] = hc[i];
        est = std::fabs(gv[j + 1]);
        if (o->history && hlen < o->history_cap) o->history[hlen] = est / nb;
        ++hlen;
        jj = j + 1;
        if (!std::isfinite(est)) break;
        if (est <= tol * nb || hv[ncols] == 0.0 || its >= maxit) break;
      }
    } else {
      // Device-driven cycle: the step ends (Givens, estimate, stopping
      // tests) run on the device; the host enqueues batches of steps and
      // reads the cycle state once per batch.  Steps enqueued after the stop
      // run on values nobody reads (the device state no longer changes), so
      // the batch length follows the observed convergence rate.
      std::vector<double> st0(kArnG + m + 1, 0.0);
      st0[kArnTolAbs] = tol * nb;
      st0[kArnMaxIts] = (double)maxit;
      st0[kArnIts] = (double)its;
      st0[kArnG] = rho;
      rc = upload(ctx, d_arn, st0.data(), (int)st0.size());
      if (rc) return rc;
      int j = 0;
      int64_t its0 = its;
      double last = rho;
      while (j < m) {
        const int kb = std::min(batch, m - j);
        for (int q = 0; q < kb; ++q) {
          rc = step(j + q, true);
          if (rc) return rc;
        }
        rc = read_dev(ctx, d_arn, kArnHist + kArnHistRing);
        if (rc) return rc;
        const double* d = ctx->pin;
        const int jdone = (int)d[kArnJ];
        for (int64_t h = its; h < (int64_t)d[kArnIts]; ++h) {
          if (o->history && hlen < o->history_cap)
            o->history[hlen] = d[kArnHist + h % kArnHistRing] / nb;
          ++hlen;
        }
        its = (int64_t)d[kArnIts];
        const double e_now = d[kArnEst];
        j += kb;
        if (d[kArnStop] == 2.0) {
          // step jdone needs an explicit norm: the steps enqueued after it
          // ran on a v_{j+1} that is about to change, so run the step again
          // (same kernels, same inputs: V_{j+1} is intact), with the
          // explicit norm pass, end it on the device and go on from there
          const double zero = 0.0;
          rc = upload(ctx, d_arn + kArnStop, &zero, 1);
          if (rc) return rc;
          rc = step(jdone, false);
          if (rc) return rc;
          rc = explicit_norm(jdone);
          if (rc) return rc;
          KRS_LAUNCH(ctx, KRS_K_OTHER, 0,
                     arnoldi_givens(s, d_arn, d_hcol, d_skip, nullptr, jdone, kc, m));
          rc = read_dev(ctx, d_arn, kArnHist + kArnHistRing);
          if (rc) return rc;
          const double* d2 = ctx->pin;
          for (int64_t h = its; h < (int64_t)d2[kArnIts]; ++h) {
            if (o->history && hlen < o->history_cap)
              o->history[hlen] = d2[kArnHist + h % kArnHistRing] / nb;
            ++hlen;
          }
          its = (int64_t)d2[kArnIts];
          j = jdone + 1;
          if (d2[kArnStop] != 0.0) break;
          its0 = its;
          last = d2[kArnEst];
          continue;
        }
        if (d[kArnStop] != 0.0) {
          j = jdone;
          break;
        }
        // next batch: about half the steps the recent rate still needs
        const int64_t dj = its - its0;
        if (dj > 0 && e_now > 0 && e_now < last) {
          const double rate = std::pow(e_now / last, 1.0 / (double)dj);
          const double need = std::log(tol * nb / e_now) / std::log(rate);
          batch = (int)std::max(1.0, std::min((double)bcap, 0.5 * need));
        }
        its0 = its;
        last = e_now;
      }
      jj = j;
      mv += jj;
      // the cycle's least-squares data and the recycle-update inputs
      rc = read_dev(ctx, d_arn, kArnB + kc * jj);
      if (rc) return rc;
      const double* d = ctx->pin;
      // column c holds rows 0..c+1 (the device never writes below the
      // subdiagonal; those host entries stay zero)
      for (int c = 0; c < jj; ++c) {
        for (int i = 0; i <= c + 1; ++i) {
          Hbar[i + (size_t)ldh * c] = d[kArnH + i + (m + 1) * c];
          Rr[i + (size_t)ldh * c] = d[kArnR + i + (m + 1) * c];
        }
        for (int i = 0; i < kc; ++i) Bm[i + (size_t)ldb * c] = d[kArnB + i + kc * c];
      }
      for (int i = 0; i <= jj; ++i) gv[i] = d[kArnG + i];
      est = jj > 0 ? std::fabs(gv[jj]) : rho;
      // second Gram-Schmidt passes of the cycle (the state restarts per
      // cycle); the Pythagorean-norm fallbacks that ran (rare: a norm pass
      // and a rescale) are not in the byte model
      n_two_pass += (int64_t)d[kArnTwo];
      timing_add_bytes(ctx, KRS_K_BLOCK_DOT2, NW * d[kArnTwoCols]);
    }
    est_converged = trust_est && est <= tol * nb;
    // y = R^-1 g ; z = -B y ; y_acc += V y + U z
    dense::upper_solve(jj, Rr.data(), ldh, gv.data(), yv.data());
    for (int i = 0; i < jj; ++i) coef[i] = yv[i];
    for (int c = 0; c < kc; ++c) {
      double sum = 0;
      for (int j = 0; j < jj; ++j) sum += Bm[c + (size_t)ldb * j] * yv[j];
      coef[jj + c] = -sum;
    }
    rc = upload(ctx, d_coef, coef.data(), jj + kc);
    if (rc) return rc;
    KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (jj + kc + 2),
               block_update<T>(s, cols<T>(V, ld, jj, U, ldr, kc), d_coef, 1.0, x, x, n, nullptr,
                               0, part, nblk));
    ++cycles;
    // recycle-space update
    if (gcrot) {
      rc = gcrot_update<T>(ctx, rec, V, ld, jj, Hbar, ldh, Bm, ldb, yv, o->k, gpar, prevQ,
                           prev_dim, part, sc, st);
      if (rc) return rc;
    } else if (update && rec) {
      rc = harmonic_update<T>(ctx, rec, V, ld, jj, Hbar, ldh, Bm, ldb, o->k, part, sc, st);
      if (rc) return rc;
    }
    // true residual r = b - A~ y (into the first basis column)
    if (left) {
      // r = M^-1 (b - A x) = M^-1 b - M^-1 A x
      KRS_LAUNCH(ctx, KRS_K_RESIDUAL, (op.g.pts + 3) * NW,
                 residual_norm<T>(s, op.g, op.bands(), x, b_orig, z, part));
      rc = op.minv_s(z, r0, ptmp);
      if (rc) return rc;
      KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW, block_dot<T>(s, Cols<T>{}, r0, n, 1, part, nblk));
    } else {
      rc = op.minv(x, z);
      if (rc) return rc;
      KRS_LAUNCH(ctx, KRS_K_RESIDUAL, (op.g.pts + 3) * NW,
                 residual_norm<T>(s, op.g, op.bands(), z, b, r0, part));
    }
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, 1, d_nrm));
    ++mv;
    kc = rec ? rec->dim : 0;
    if (kc > 0) {
      // re-project against the (new) C: xi = C^T r, r -= C xi, y += U xi
      KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW * (kc + 1),
                 block_dot<T>(s, cols<T>(C, ldr, kc), r0, n, 0, part, nblk));
      KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, kc, d_xi));
      KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (kc + 2),
                 block_update<T>(s, cols<T>(C, ldr, kc), d_xi, -1.0, r0, r0, n, nullptr, 1, part,
                                 nblk));
      KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, 1, d_nrm));
      KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (kc + 2),
                 block_update<T>(s, cols<T>(U, ldr, kc), d_xi, 1.0, x, x, n, nullptr, 0, part,
                                 nblk));
    }
    rc = read_dev(ctx, d_nrm, 1);
    if (rc) return rc;
    rho = std::sqrt(ctx->pin[0]);
    if (!std::isfinite(rho)) {
      status = KRS_DIVERGED;
      break;
    }
  }
  if (status != KRS_DIVERGED && (rho <= tol * nb || est_converged)) status = KRS_OK;
  double rel_true = rho / nb;
  if (left) {
    // x is the iterate itself; report the unpreconditioned residual
    KRS_LAUNCH(ctx, KRS_K_RESIDUAL, (op.g.pts + 3) * NW,
               residual_norm<T>(s, op.g, op.bands(), x, b_orig, z, part));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, 1, d_nrm));
    rc = read_dev(ctx, d_nrm, 1);
    if (rc) return rc;
    rel_true = nb_orig > 0 ? std::sqrt(ctx->pin[0]) / nb_orig : 0.0;
  } else {
    // x = M^-1 y
    rc = op.minv(x, z);
    if (rc) return rc;
    KRS_LAUNCH(ctx, KRS_K_OTHER, 2 * NW, copy<T>(s, z, x, n));
  }
  KRS_CHECK_HIP(ctx, hipStreamSynchronize(s));
  timing_flush(ctx);
  if (st) {
    st->status = status;
    st->matvecs = mv;
    st->iterations = its;
    st->cycles = cycles;
    st->history_len = hlen;
    st->rel_res_true = rel_true;
    st->rel_res_est = left ? rho / nb : est / nb;
    st->time_ms = tm.ms();
    st->bytes_model = ctx->bytes - bytes0;
    st->second_passes = n_two_pass;
  }
  (void)n_one_pass;
  return status;
}

// ---------------------------------------------------------------------------
// recycle-space setup of Alg. 3: C~ = A~ U, C~ = C R (Cholesky QR, twice), U <- U R^-1
// ---------------------------------------------------------------------------
// Two Cholesky-QR passes over C (U alongside): G = C^T C = R^T R,
// C <- C R^-1, U <- U R^-1, so C^T C = I and A~ U = C are kept.
template <class T>
int cholqr2(krs_ctx* ctx, krs_recycle* rec, T* part, double* sc, const char* fail) {
  hipStream_t s = ctx->stream;
  const int64_t n = rec->n;
  const int kc = rec->dim;
  if (kc == 0) return 0;
  T* U = (T*)rec->U;
  T* C = (T*)rec->C;
  const int64_t ldr = rec->ld;
  std::vector<double> G((size_t)kc * kc), R((size_t)kc * kc), Ri((size_t)kc * kc);
  const double NW = (double)n * sizeof(T);
  for (int pass = 0; pass < 2; ++pass) {
    const int gb = gram_blocks(kc, kc, n);
    KRS_LAUNCH(ctx, KRS_K_GRAM, NW * kc,
               gram<T>(s, cols<T>(C, ldr, kc), cols<T>(C, ldr, kc), n, part, gb));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, gb, kc * kc, sc + Ws<T>::kGram1));
    int rc = read_dev(ctx, sc + Ws<T>::kGram1, kc * kc);
    if (rc) return rc;
    for (int a = 0; a < kc; ++a)
      for (int b = 0; b < kc; ++b) G[a + (size_t)kc * b] = ctx->pin[a * kc + b];
    if (!dense::cholesky_upper(kc, G.data(), R.data()) ||
        !dense::upper_inverse(kc, R.data(), Ri.data()))
      return set_err(ctx, KRS_ERR_STATE, fail);
    rc = upload(ctx, sc + Ws<T>::kM, Ri.data(), kc * kc);
    if (rc) return rc;
    KRS_LAUNCH(ctx, KRS_K_ROW_TRANSFORM, NW * 2 * kc,
               row_transform<T>(s, cols<T>(C, ldr, kc), sc + Ws<T>::kM, kc, C, ldr, n));
    KRS_LAUNCH(ctx, KRS_K_ROW_TRANSFORM, NW * 2 * kc,
               row_transform<T>(s, cols<T>(U, ldr, kc), sc + Ws<T>::kM, kc, U, ldr, n));
  }
  return 0;
}

template <class T>
int recycle_setup_t(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                    void* ws, size_t wsb) {
  hipStream_t s = ctx->stream;
  const int64_t n = A->n, ld = vec_ld(n);
  Carver cv(ws, wsb);
  T* z = cv.vec<T>(ld);
  T* tmp = cv.vec<T>(ld);
  T* part = (T*)cv.take(partials_bytes(sizeof(T)));
  double* sc = cv.vec<double>(kScalarDoubles);
  if (!ws || !cv.ok) return set_err(ctx, KRS_ERR_WORKSPACE, "workspace missing or too small");
  const int kc = rec->dim;
  if (kc == 0) return 0;
  T* U = (T*)rec->U;
  T* C = (T*)rec->C;
  const int64_t ldr = rec->ld;
  Op<T> op{ctx, A, M, grid3(A), z, tmp};
  for (int c = 0; c < kc; ++c) {
    int rc = op.apply(U + (int64_t)c * ldr, C + (int64_t)c * ldr);
    if (rc) return rc;
  }
  int rc = cholqr2<T>(ctx, rec, part, sc, "recycle setup: A~ U is rank deficient");
  if (rc) return rc;
  KRS_CHECK_HIP(ctx, hipStreamSynchronize(s));
  timing_flush(ctx);
  return 0;
}

// ---------------------------------------------------------------------------
// rBiCGStab with one recycle space (Alg. 4); Alg. 2 when the space is empty
// ---------------------------------------------------------------------------
template <class T>
int rbicgstab_t(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, const krs_recycle* rec,
                const T* b, T* x, const krs_opts* o, void* ws, size_t wsb, krs_stats* st) {
  Timer tm;
  const double bytes0 = ctx->bytes;
  hipStream_t s = ctx->stream;
  const int64_t n = A->n, ld = vec_ld(n);
  Carver cv(ws, wsb);
  T* r = cv.vec<T>(ld);
  T* rt = cv.vec<T>(ld);
  T* p = cv.vec<T>(ld);
  T* v = cv.vec<T>(ld);
  T* sv = cv.vec<T>(ld);
  T* t = cv.vec<T>(ld);
  T* z = cv.vec<T>(ld);
  T* y = cv.vec<T>(ld);   // iterate of A~ y = b (x = M^-1 y at the end)
  T* part = (T*)cv.take(partials_bytes(sizeof(T)));
  double* sc = cv.vec<double>(kScalarDoubles);
  if (!ws || !cv.ok) return set_err(ctx, KRS_ERR_WORKSPACE, "workspace missing or too small");
  const int kSums = kBSums, kEta1 = kBEta1, kEta2 = kBEta2, kXi = kBXi, kCtrt = kBCtrt,
            kNrm = kBNrm;
  // the BiCGStab passes run on at most 512 blocks (2048 waves: the whole grid
  // is resident at once at the passes' 2 waves per SIMD); the fused update
  // passes stream 2-3% faster than on 1024 blocks (measured at 256^3)
  const int nblk = std::min(red_blocks(n), 512);
  const double NW = (double)n * sizeof(T);
  const double tol = o->tol;
  const int64_t maxmv = o->max_matvecs > 0 ? o->max_matvecs : 2000;
  Op<T> op{ctx, A, M, grid3(A), z, nullptr};
  init_stats(st);
  double nb2 = 0;
  int rc = norm2<T>(ctx, b, n, part, sc + kNrm, nb2);
  if (rc) return rc;
  const double nb = std::sqrt(nb2);
  if (nb == 0 || !std::isfinite(nb)) {
    KRS_LAUNCH(ctx, KRS_K_OTHER, NW, fill<T>(s, x, n, 0.0));
    KRS_CHECK_HIP(ctx, hipStreamSynchronize(s));
    timing_flush(ctx);
    if (st) {
      st->status = std::isfinite(nb) ? KRS_OK : KRS_DIVERGED;
      st->rel_res_true = 0;
      st->time_ms = tm.ms();
    }
    return std::isfinite(nb) ? KRS_OK : KRS_DIVERGED;
  }
  const int kc = rec ? rec->dim : 0;
  // partials of the fused sv pass (|s|^2) after the dot pass's kc + 2
  // columns, then those of the yr pass (r~.r, |r|^2)
  T* const part2 = part + (size_t)nblk * (kc + 2);
  T* const part3 = part2 + nblk;
  const T* U = rec ? (const T*)rec->U : nullptr;
  const T* C = rec ? (const T*)rec->C : nullptr;
  const int64_t ldr = rec ? rec->ld : 0;
  const Cols<T> Cc = cols<T>(C, ldr, kc);
  std::vector<double> slots(kSlots, 0.0);
  double rn2 = nb2;
  // project b: eta1 = C^T b, r0 = b - C eta1, xi = -eta1
  if (kc > 0) {
    KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW * (kc + 1), block_dot<T>(s, Cc, b, n, 0, part, nblk));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, kc, sc + kEta1));
    KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (kc + 2),
               block_update<T>(s, Cc, sc + kEta1, -1.0, b, r, n, nullptr, 1, part, nblk));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, 1, sc + kNrm));
    rc = read_dev(ctx, sc + kEta1, kc);
    if (rc) return rc;
    std::vector<double> xi(kc);
    for (int c = 0; c < kc; ++c) xi[c] = -ctx->pin[c];
    rc = upload(ctx, sc + kXi, xi.data(), kc);
    if (rc) return rc;
    rc = read_dev(ctx, sc + kNrm, 1);
    if (rc) return rc;
    rn2 = ctx->pin[0];
  } else {
    KRS_LAUNCH(ctx, KRS_K_OTHER, 2 * NW, copy<T>(s, b, r, n));
  }
  // r~ = r_0 ; C^T r~ for the alpha denominator
  KRS_LAUNCH(ctx, KRS_K_OTHER, 2 * NW, copy<T>(s, r, rt, n));
  if (kc > 0) {
    KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW * (kc + 1), block_dot<T>(s, Cc, rt, n, 0, part, nblk));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, nblk, kc, sc + kCtrt));
  }
  // p_0 = r_0 (the full step of each iteration forms the next p)
  KRS_LAUNCH(ctx, KRS_K_OTHER, 2 * NW, copy<T>(s, r, p, n));
  KRS_LAUNCH(ctx, KRS_K_OTHER, NW, fill<T>(s, y, n, 0.0));
  slots[kRho] = rn2;  // r~ = r
  slots[kRhoNew] = rn2;
  slots[kOmega] = 1.0;
  slots[kBeta] = 0.0;
  slots[kRnorm2] = rn2;
  slots[kTolAbs] = tol * nb;
  slots[kDivAbs] = o->div_factor > 0 ? o->div_factor * nb : INFINITY;
  rc = upload(ctx, sc, slots.data(), kSlots);
  if (rc) return rc;
  double rnorm = std::sqrt(rn2);
  double rho = rn2;
  int64_t its = 0, mv = 0, hlen = 0;
  int status = KRS_NOT_CONVERGED;
  const double div = o->div_factor;
  auto hist = [&](double val) {
    if (o->history && hlen < o->history_cap) o->history[hlen] = val;
    ++hlen;
  };
  // one pass of the while loop of Alg. 4 up to the half-step test / after it
  // In the device-driven mode the passes that may be skipped after the stop
  // are charged to the byte model from the counts read back (dev = true).
  const double bytes_p = 4 * NW, bytes_sv = NW * (kc + (kc > 0 ? 4 : 3)), bytes_yr = NW * (kc + 7);
  auto first_half = [&](bool dev) -> int {
    int e = op.apply(p, v);
    if (e) return e;
    // eta1 = C^T v, v -= C eta1, alpha = rho / r~^T v, s = r - alpha v
    KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW * (kc + 2),
               block_dot<T>(s, cols<T>(C, ldr, kc, rt, ld, 1), v, n, 0, part, nblk));
    // the alpha step runs in front of the sv pass (each block sums the dot
    // partials itself), whose |s|^2 partials go to part2
    KRS_LAUNCH(ctx, KRS_K_BICG_SV, dev ? 0 : bytes_sv,
               bicg_sv_fused<T>(s, Cc, r, v, sv, sc, kEta1, kCtrt, sc + kSums, n, part, part2,
                                nblk));
    // host-tested loop: the half-step |s| tests in a launch of their own (on
    // convergence xi += alpha eta1 and, in the same launch, y += alpha p,
    // r = s), so that the host reads them before the second half
    if (!dev)
      KRS_LAUNCH(ctx, KRS_K_BICG_P, 0,
                 bicg_half_exit<T>(s, p, y, sv, r, sc, kEta1, kXi, kc, part2, nblk, n));
    return 0;
  };
  auto second_half = [&](bool dev) -> int {
    int e = op.apply(sv, t);
    if (e) return e;
    // eta2 = C^T t, omega = t^T s / |t - C eta2|^2, xi update
    KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW * (kc + 2),
               block_dot<T>(s, cols<T>(C, ldr, kc, sv, ld, 1), t, n, 1, part, nblk));
    // the omega step in front of the y and r updates (with the partials of
    // the next rho = r~^T r), then the loop tests and the next p.  In the
    // device-driven loop the half-step tests run in front of the omega step
    // (on convergence the pass applies the exit instead; A~ s and its dot
    // pass have then run for nothing, once per solve)
    KRS_LAUNCH(ctx, KRS_K_BICG_YR, dev ? 0 : bytes_yr,
               bicg_yr_fused<T>(s, Cc, t, sv, p, y, r, rt, sc, kEta1, kEta2, kXi, sc + kSums, n,
                                part, dev ? part2 : nullptr, part3, nblk));
    // (its p update is charged once the state read back shows it ran)
    KRS_LAUNCH(ctx, KRS_K_BICG_P, 0,
               bicg_finish_p<T>(s, part3, nblk, sc + kSums, sc, r, p, v, n));
    return 0;
  };
  if (o->flags & KRS_FLAG_HOST_LOOP) {
    while (rnorm > tol * nb && mv < maxmv) {
      if (rho == 0.0) {                                      // breakdown
        status = KRS_BREAKDOWN;
        break;
      }
      rc = first_half(false);
      if (rc) return rc;
      ++mv;
      rc = read_dev(ctx, sc, kSlots);
      if (rc) return rc;
      std::copy(ctx->pin, ctx->pin + kSlots, slots.begin());
      ++its;
      if (slots[kFlag] != 0.0) {
        status = KRS_BREAKDOWN;
        break;
      }
      const double snorm = std::sqrt(slots[kSnorm2]);
      hist(snorm / nb);
      if (!std::isfinite(snorm)) {
        status = KRS_DIVERGED;
        break;
      }
      if (snorm <= tol * nb) {                              // half-step exit (applied)
        timing_add_bytes(ctx, KRS_K_BICG_P, 5 * NW);
        rnorm = snorm;
        break;
      }
      rc = second_half(false);
      if (rc) return rc;
      ++mv;
      rc = read_dev(ctx, sc, kSlots);
      if (rc) return rc;
      std::copy(ctx->pin, ctx->pin + kSlots, slots.begin());
      rnorm = std::sqrt(slots[kRnorm2]);
      rho = slots[kRhoNew];
      if (slots[kDone] == kRunning) timing_add_bytes(ctx, KRS_K_BICG_P, bytes_p);
      hist(rnorm / nb);
      if (slots[kFlag] != 0.0 || slots[kFlagT] != 0.0) {
        status = KRS_BREAKDOWN;
        break;
      }
      if (!std::isfinite(rnorm) || (div > 0 && rnorm > div * nb)) {
        status = KRS_DIVERGED;
        break;
      }
    }
  } else if (rnorm > tol * nb) {
    auto one_pass = [&]() -> int {
      int e = first_half(true);
      if (e) return e;
      return second_half(true);
    };
    // optionally replay one captured pass per iteration
    krs_ctx::Graph* graph = nullptr;
    if ((o->flags & KRS_FLAG_GRAPH) && !ctx->timing && n <= kGraphMaxN) {
      const krs_precond* Mp = M;
      std::vector<uint64_t> key = {
          sizeof(T), (uint64_t)n, (uint64_t)kc, (uint64_t)(uintptr_t)A->bands,
          (uint64_t)A->g.nx, (uint64_t)A->g.ny, (uint64_t)A->g.nz,
          (uint64_t)(A->g.periodic[0] | (A->g.periodic[1] << 1) | (A->g.periodic[2] << 2)),
          (uint64_t)(uintptr_t)Mp, (uint64_t)(uintptr_t)(Mp ? Mp->pack : nullptr),
          (uint64_t)(Mp ? Mp->d.type : -1), (uint64_t)(Mp ? Mp->d.tile : 0),
          (uint64_t)(Mp ? Mp->d.overlap : 0), (uint64_t)(Mp ? Mp->d.local_sweeps : 0),
          (uint64_t)(Mp ? Mp->d.global_sweeps : 0), 0, 0, (uint64_t)(uintptr_t)C,
          (uint64_t)ldr, (uint64_t)(uintptr_t)ws};
      if (Mp) {
        std::memcpy(&key[15], &Mp->d.omega_local, 8);
        std::memcpy(&key[16], &Mp->d.omega_global, 8);
      }
      for (auto& g : ctx->graphs)
        if (g.key == key) graph = &g;
      if (!graph) {
        if (!ctx->capture)
          KRS_CHECK_HIP(ctx, hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
        const hipStream_t saved = ctx->stream;
        const double b0 = ctx->bytes;
        ctx->stream = ctx->capture;
        s = ctx->capture;
        hipGraph_t gr = nullptr;
        hipError_t eb = hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal);
        int e = eb == hipSuccess ? one_pass() : 0;
        hipError_t ee = eb == hipSuccess ? hipStreamEndCapture(ctx->capture, &gr) : eb;
        ctx->stream = saved;
        s = saved;
        const double gbytes = ctx->bytes - b0;
        ctx->bytes = b0;
        if (e || ee != hipSuccess) {
          if (gr) (void)hipGraphDestroy(gr);
          if (e) return e;
          return set_err(ctx, KRS_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ee));
        }
        hipGraphExec_t ex = nullptr;
        hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (ei != hipSuccess)
          return set_err(ctx, KRS_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
        if ((int)ctx->graphs.size() >= kMaxGraphs) {
          auto lru = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                      [](const krs_ctx::Graph& a, const krs_ctx::Graph& b) {
                                        return a.used < b.used;
                                      });
          (void)hipGraphExecDestroy(lru->exec);
          ctx->graphs.erase(lru);
        }
        krs_ctx::Graph g;
        g.key = key;
        g.exec = ex;
        g.bytes = gbytes;
        ctx->graphs.push_back(g);
        graph = &ctx->graphs.back();
      }
      graph->used = ++ctx->clock;
    }
    // Device-driven: the stopping tests run in single-thread kernels and the
    // host reads the state once per batch of iterations.  The batch length
    // follows the observed convergence rate so that few iterations run past
    // the stop (they are no-ops: every pass returns once kDone != 0).
    const int64_t allowed = (maxmv + 1) / 2;                // passes with mv < maxmv at entry
    const int kcap = n <= (int64_t(1) << 18) ? 32 : (n <= (int64_t(1) << 21) ? 8 : 4);
    int batch = std::min(2, kcap);
    int64_t hseen = 0;
    double last = rnorm;
    int64_t its_prev = 0;
    while (its < allowed) {
      const int kb = (int)std::min<int64_t>(batch, allowed - its);
      for (int q = 0; q < kb; ++q) {
        if (graph) {
          KRS_CHECK_HIP(ctx, hipGraphLaunch(graph->exec, s));
          ctx->bytes += graph->bytes;
        } else {
          rc = one_pass();
          if (rc) return rc;
        }
      }
      rc = read_dev(ctx, sc, kHistOff + kHistRing);
      if (rc) return rc;
      const double* d = ctx->pin;
      const int64_t started = (int64_t)d[kIts] - its;
      const int done_now = (int)d[kDone];
      const bool half = done_now != kRunning && d[kEndHalf] != 0.0;
      const bool exited = done_now == kExited || done_now == kConvHalf;
      // p is formed at the end of every iteration that goes on
      const int64_t p_updates = started - (done_now != kRunning ? 1 : 0);
      timing_add_bytes(ctx, KRS_K_BICG_P, p_updates * bytes_p + (exited ? 5 * NW : 0.0));
      timing_add_bytes(ctx, KRS_K_BICG_SV, started * bytes_sv);
      timing_add_bytes(ctx, KRS_K_BICG_YR, (started - (half ? 1 : 0)) * bytes_yr);
      its = (int64_t)d[kIts];
      const int64_t hl = (int64_t)d[kHlen];
      for (int64_t h = hseen; h < hl; ++h) hist(d[kHistOff + h % kHistRing] / nb);
      hseen = hl;
      const int done = (int)d[kDone];
      if (done != kRunning) {
        mv = 2 * its - (d[kEndHalf] != 0.0 ? 1 : 0);
        rnorm = std::sqrt(d[kRnorm2]);
        if (done == kBreak) status = KRS_BREAKDOWN;
        else if (done == kDiverge) status = KRS_DIVERGED;
        break;
      }
      mv = 2 * its;
      rnorm = std::sqrt(d[kRnorm2]);
      // next batch: about half the iterations the recent rate still needs
      const int64_t dits = its - its_prev;
      its_prev = its;
      if (dits > 0 && rnorm > 0 && rnorm < last) {
        const double rate = std::pow(rnorm / last, 1.0 / (double)dits);
        const double need = std::log(tol * nb / rnorm) / std::log(rate);
        batch = (int)std::max(1.0, std::min((double)kcap, 0.5 * need));
      } else {
        batch = std::min(kcap, std::max(1, batch));
      }
      last = rnorm;
    }
  }
  if (status == KRS_NOT_CONVERGED && rnorm <= tol * nb) status = KRS_OK;
  int64_t site = 0;
  if (status == KRS_BREAKDOWN) {
    // the flag the scalar steps left (1: alpha, 2: omega), else rho = 0
    int e = read_dev(ctx, sc, kSlots);
    if (e) return e;
    site = ctx->pin[kFlag] != 0.0 ? (int64_t)ctx->pin[kFlag]
                                  : (ctx->pin[kFlagT] != 0.0 ? (int64_t)ctx->pin[kFlagT] : 3);
  }
  // postponed U-update: y -= U xi ; then x = M^-1 y
  if (kc > 0) {
    KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (kc + 2),
               block_update<T>(s, cols<T>(U, ldr, kc), sc + kXi, -1.0, y, y, n, nullptr, 0, part,
                               nblk));
  }
  rc = op.minv_s(y, x, z);
  if (rc) return rc;
  // true residual of x (the residual kernel writes one partial per block of
  // its own grid, red_blocks(n), which can exceed the passes' nblk)
  KRS_LAUNCH(ctx, KRS_K_RESIDUAL, (op.g.pts + 3) * NW,
             residual_norm<T>(s, op.g, op.bands(), x, b, t, part));
  KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<T>(s, part, red_blocks(n), 1, sc + kNrm));
  rc = read_dev(ctx, sc + kNrm, 1);
  if (rc) return rc;
  if (st) {
    st->status = status;
    st->matvecs = mv;
    st->iterations = its;
    st->history_len = hlen;
    st->rel_res_true = std::sqrt(ctx->pin[0]) / nb;
    st->rel_res_est = rnorm / nb;
    st->time_ms = tm.ms();
    st->bytes_model = ctx->bytes - bytes0;
    st->breakdown_site = site;
  }
  return status;
}

}  // namespace

// ---------------------------------------------------------------------------
// dtype dispatch
// ---------------------------------------------------------------------------
int workspace_bytes(krs_solver solver, int64_t n, int m, int k, krs_dtype dt, size_t* bytes) {
  (void)k;
  const bool f64 = dt == KRS_F64;
  size_t v = 0;
  switch (solver) {
    case KRS_SOLVER_GMRES:
    case KRS_SOLVER_RGCROT:
      v = f64 ? std::max(ws_gmres<double>(n, m), ws_bicg<double>(n))
              : std::max(ws_gmres<float>(n, m), ws_bicg<float>(n));
      break;
    case KRS_SOLVER_RGCROT_T: {
      const size_t extra = (size_t)vec_ld(n) * m * (f64 ? sizeof(double) : sizeof(float));
      v = f64 ? std::max(ws_gmres<double>(n, m) + extra + 256, ws_bicg<double>(n))
              : std::max(ws_gmres<float>(n, m) + extra + 256, ws_bicg<float>(n));
      break;
    }
    case KRS_SOLVER_RBICGSTAB:
      v = f64 ? ws_bicg<double>(n) : ws_bicg<float>(n);
      break;
    case KRS_SOLVER_IR:
      v = ws_ir(n, m);
      break;
    default:
      return KRS_ERR_ARG;
  }
  *bytes = v;
  return KRS_OK;
}

size_t precond_pack_bytes(const krs_matrix* A, const krs_precond_desc* d) {
  // the packed coefficients serve 7-point bands; 19-point local solves read the bands
  if (!d || d->type != KRS_PC_SCHWARZ_JACOBI || d->tile <= 0 || A->pts != 7) return 0;
  return (size_t)schwarz_pack_values(grid3(A), d->tile) *
         (A->dt == KRS_F64 ? sizeof(double) : sizeof(float));
}

int precond_pack(krs_ctx* ctx, const krs_precond* M) {
  if (!M->pack) return 0;
  const krs_matrix* A = M->A;
  const Grid3 g = grid3(A);
  const double bytes = (double)precond_pack_bytes(A, &M->d) + 7.0 * A->n *
                       (A->dt == KRS_F64 ? 8 : 4);
  if (A->dt == KRS_F64)
    KRS_LAUNCH(ctx, KRS_K_OTHER, bytes,
               schwarz_pack<double>(ctx->stream, g, M->d.tile, (const double*)A->bands,
                                    (double*)M->pack, M->d.omega_local));
  else
    KRS_LAUNCH(ctx, KRS_K_OTHER, bytes,
               schwarz_pack<float>(ctx->stream, g, M->d.tile, (const float*)A->bands,
                                   (float*)M->pack, M->d.omega_local));
  return 0;
}

int precond_apply(krs_ctx* ctx, const krs_precond* M, const void* r, void* z, void* tmp) {
  const krs_matrix* A = M->A;
  if (A->dt == KRS_F64) {
    Op<double> op{ctx, A, M, grid3(A), nullptr, (double*)tmp};
    return op.minv((const double*)r, (double*)z);
  }
  Op<float> op{ctx, A, M, grid3(A), nullptr, (float*)tmp};
  return op.minv((const float*)r, (float*)z);
}

int operator_apply(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, const void* v, void* w,
                   void* tmp) {
  if (A->dt == KRS_F64) {
    Op<double> op{ctx, A, M, grid3(A), (double*)tmp, nullptr};
    return op.apply((const double*)v, (double*)w);
  }
  Op<float> op{ctx, A, M, grid3(A), (float*)tmp, nullptr};
  return op.apply((const float*)v, (float*)w);
}

int gmres_rgcrot(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                 bool update, const void* b, void* x, const krs_opts* o, void* ws, size_t wsb,
                 krs_stats* st) {
  ctx->bytes = 0;
  if (A->dt == KRS_F64)
    return gmres_rgcrot_t<double>(ctx, A, M, rec, update, (const double*)b, (double*)x, o, ws, wsb,
                                  st);
  return gmres_rgcrot_t<float>(ctx, A, M, rec, update, (const float*)b, (float*)x, o, ws, wsb, st);
}

int rbicgstab(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, const krs_recycle* rec,
              const void* b, void* x, const krs_opts* o, void* ws, size_t wsb, krs_stats* st) {
  ctx->bytes = 0;
  if (A->dt == KRS_F64)
    return rbicgstab_t<double>(ctx, A, M, rec, (const double*)b, (double*)x, o, ws, wsb, st);
  return rbicgstab_t<float>(ctx, A, M, rec, (const float*)b, (float*)x, o, ws, wsb, st);
}

int recycle_setup(krs_ctx* ctx, const krs_matrix* A, const krs_precond* M, krs_recycle* rec,
                  void* ws, size_t wsb) {
  ctx->bytes = 0;
  if (A->dt == KRS_F64) return recycle_setup_t<double>(ctx, A, M, rec, ws, wsb);
  return recycle_setup_t<float>(ctx, A, M, rec, ws, wsb);
}

// ---------------------------------------------------------------------------
// FP64 iterative refinement around an FP32 inner solver
// ---------------------------------------------------------------------------
int ir_solve(krs_ctx* ctx, const krs_matrix* A64, const krs_matrix* A32, const krs_precond* M32,
             krs_recycle* rec32, const void* bv, void* xv, const krs_opts* o, void* ws,
             size_t wsb, krs_stats* st) {
  Timer tm;
  hipStream_t s = ctx->stream;
  const int64_t n = A64->n, ld = vec_ld(n);
  const double* b = (const double*)bv;
  double* x = (double*)xv;
  const size_t inner_bytes = std::max(ws_gmres<float>(n, o->m), ws_bicg<float>(n));
  Carver cv(ws, wsb);
  void* inner = cv.take(inner_bytes);
  double* r64 = cv.vec<double>(ld);
  float* b32 = cv.vec<float>(ld);
  float* d32 = cv.vec<float>(ld);
  double* part = (double*)cv.take(partials_bytes(sizeof(double)));
  double* sc = cv.vec<double>(kScalarDoubles);
  if (!ws || !cv.ok) return set_err(ctx, KRS_ERR_WORKSPACE, "workspace missing or too small");
  const int nblk = red_blocks(n);
  const Grid3 g = grid3(A64);
  init_stats(st);
  double total_bytes = 0;
  double nb2 = 0;
  ctx->bytes = 0;
  int rc = norm2<double>(ctx, b, n, part, sc, nb2);
  if (rc) return rc;
  const double nb = std::sqrt(nb2);
  KRS_LAUNCH(ctx, KRS_K_OTHER, 8.0 * n, fill<double>(s, x, n, 0.0));
  KRS_LAUNCH(ctx, KRS_K_OTHER, 16.0 * n, copy<double>(s, b, r64, n));
  total_bytes += ctx->bytes;
  double rn = nb;
  int status = KRS_NOT_CONVERGED;
  int64_t outer = 0, its = 0, mv = 0, cycles = 0;
  krs_opts io = *o;
  const double inner_floor = o->inner_tol > 0 ? o->inner_tol : 1e-5;
  io.flags |= KRS_FLAG_TRUST_ESTIMATE;
  io.history = nullptr;
  io.history_cap = 0;
  const int max_outer = o->max_outer > 0 ? o->max_outer : 20;
  double host_eig = 0;
  int ties = 0;
  int64_t second = 0;
  if (!(nb > 0)) {
    if (st) {
      st->status = std::isfinite(nb) ? KRS_OK : KRS_DIVERGED;
      st->rel_res_true = 0;
    }
    return std::isfinite(nb) ? KRS_OK : KRS_DIVERGED;
  }
  while (rn > o->tol * nb && outer < max_outer) {
    // scaled FP32 right-hand side r / ||r||; solve no tighter than needed
    io.tol = std::max(inner_floor, 0.5 * o->tol * nb / rn);
    const double sv[2] = {1.0 / rn, rn};
    rc = upload(ctx, sc + 16, sv, 2);
    if (rc) return rc;
    ctx->bytes = 0;
    KRS_LAUNCH(ctx, KRS_K_OTHER, 12.0 * n, cast_scale_f64_f32(s, r64, b32, n, sc + 16));
    total_bytes += ctx->bytes;
    krs_stats ist;
    int irc;
    if (o->inner_solver == KRS_SOLVER_RBICGSTAB) {
      irc = rbicgstab(ctx, A32, M32, rec32, b32, d32, &io, inner, inner_bytes, &ist);
      if (irc == KRS_BREAKDOWN || irc == KRS_DIVERGED) {
        // switch back to rGCROT for this correction (Sec. 2.4)
        its += ist.iterations;
        mv += ist.matvecs;
        total_bytes += ist.bytes_model;
        irc = gmres_rgcrot(ctx, A32, M32, rec32, true, b32, d32, &io, inner, inner_bytes, &ist);
      }
    } else {
      irc = gmres_rgcrot(ctx, A32, M32, rec32, o->update_recycle != 0, b32, d32, &io, inner,
                         inner_bytes, &ist);
    }
    if (irc < 0) return irc;
    its += ist.iterations;
    mv += ist.matvecs;
    cycles += ist.cycles;
    host_eig += ist.host_eig_ms;
    ties += ist.eig_ties;
    second += ist.second_passes;
    total_bytes += ist.bytes_model;
    // x += ||r|| d ; r = b - A x in FP64
    ctx->bytes = 0;
    KRS_LAUNCH(ctx, KRS_K_OTHER, 20.0 * n, axpy_f32_into_f64(s, d32, x, n, sc + 17));
    KRS_LAUNCH(ctx, KRS_K_RESIDUAL, (8.0 * g.pts + 24.0) * n,
               residual_norm<double>(s, g, (const double*)A64->bands, x, b, r64, part));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<double>(s, part, nblk, 1, sc));
    total_bytes += ctx->bytes;
    rc = read_dev(ctx, sc, 1);
    if (rc) return rc;
    const double rn_new = std::sqrt(ctx->pin[0]);
    ++outer;
    if (o->history && outer - 1 < o->history_cap) o->history[outer - 1] = rn_new / nb;
    if (!std::isfinite(rn_new)) {
      status = KRS_DIVERGED;
      rn = rn_new;
      break;
    }
    const bool stalled = rn_new > 0.9 * rn;
    rn = rn_new;
    if (stalled && rn > o->tol * nb) break;
  }
  if (status != KRS_DIVERGED && rn <= o->tol * nb) status = KRS_OK;
  if (st) {
    st->status = status;
    st->iterations = its;
    st->matvecs = mv;
    st->cycles = cycles;
    st->outer = outer;
    st->history_len = outer;
    st->rel_res_true = rn / nb;
    st->rel_res_est = rn / nb;
    st->time_ms = tm.ms();
    st->host_eig_ms = host_eig;
    st->eig_ties = ties;
    st->bytes_model = total_bytes;
    st->second_passes = second;
  }
  return status;
}

// ---------------------------------------------------------------------------
// FP64 iterative refinement of several independent systems at once, with the
// inner rBiCGStab iterations of all of them in grouped launches
// ---------------------------------------------------------------------------
namespace {

// Whether the grouped rBiCGStab passes can run system i exactly as its own
// launches would: FP32 7-point bands, Schwarz-Jacobi with packed Jacobi local
// sweeps on 8^3 tiles in bricks of 2^3, one global sweep, 16-byte packs.
bool batchable(const krs_ir_system& q) {
  const krs_matrix* A = q.A32;
  const krs_precond* M = q.M32;
  if (!A || !M || A->pts != 7 || A->dt != KRS_F32) return false;
  if (M->d.type != KRS_PC_SCHWARZ_JACOBI || !M->pack || M->d.tile != 8 || M->d.overlap != 1 ||
      M->d.local_sweeps < 1 || M->d.global_sweeps != 1 ||
      M->d.local_solver != KRS_LOCAL_JACOBI)
    return false;
  const Grid3 g = grid3(A);
  if (g.nx % 8 || g.ny % 8 || g.nz % 8 || schwarz_brick(g, 8) != 2 || g.nx % 4) return false;
  auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  if (!al(A->bands) || !al(M->pack)) return false;
  if (q.rec32 && q.rec32->dim > 0 && (!al(q.rec32->C) || q.rec32->ld % 4)) return false;
  return true;
}

// Per-system state of the batched refinement: the layout of its workspace
// (that of ir_solve, with rbicgstab_t's inside the inner part), its FP64
// residual and the counters ir_solve keeps.
struct IrSys {
  const krs_ir_system* q;
  int64_t n = 0, ld = 0;
  void* inner = nullptr;
  size_t inner_bytes = 0;
  double* r64 = nullptr;
  float* b32 = nullptr;
  float* d32 = nullptr;
  double* part = nullptr;
  double* sc = nullptr;      // refinement scalars
  // the inner rBiCGStab workspace
  float *r = nullptr, *rt = nullptr, *p = nullptr, *v = nullptr, *sv = nullptr, *t = nullptr,
        *z = nullptr, *y = nullptr, *ipart = nullptr;
  double* isc = nullptr;
  double nb = 0, rn = 0;
  int status = KRS_NOT_CONVERGED;
  bool active = false;
  int64_t outer = 0, its = 0, mv = 0;
  double bytes = 0;
  // inner solve
  double itol = 0, inb = 0, irnorm = 0;
  int istatus = KRS_NOT_CONVERGED;
  int64_t iits = 0, imv = 0;
  bool inner_running = false;
};

}  // namespace

int ir_solve_batched(krs_ctx* ctx, int nsys, const krs_ir_system* sys, const krs_opts* o,
                     void* ws, size_t wsb) {
  hipStream_t s = ctx->stream;
  if (nsys < 1) return KRS_OK;
  if (!ws || wsb < align_up(sizeof(BatchTable)))
    return set_err(ctx, KRS_ERR_WORKSPACE, "batch workspace missing or too small");
  BatchTable* d_tb = (BatchTable*)ws;
  const double inner_floor = o->inner_tol > 0 ? o->inner_tol : 1e-5;
  const int max_outer = o->max_outer > 0 ? o->max_outer : 20;
  const int64_t maxmv = o->max_matvecs > 0 ? o->max_matvecs : 2000;
  const int64_t allowed = (maxmv + 1) / 2;
  const bool use_graph = (o->flags & KRS_FLAG_GRAPH) != 0 && !ctx->timing;
  krs_opts io = *o;
  io.flags |= KRS_FLAG_TRUST_ESTIMATE;
  io.flags &= ~(KRS_FLAG_GRAPH | KRS_FLAG_HOST_LOOP);
  io.history = nullptr;
  io.history_cap = 0;
  // systems the grouped passes cannot run exactly as alone: solved alone
  std::vector<IrSys> st;
  std::vector<int> alone;
  int kc_all = -1;
  for (int i = 0; i < nsys; ++i) {
    const krs_ir_system& q = sys[i];
    const int kc = q.rec32 ? q.rec32->dim : 0;
    if (batchable(q) && (kc_all < 0 || kc == kc_all) && (int)st.size() < kMaxBatch) {
      kc_all = kc;
      IrSys x;
      x.q = &q;
      st.push_back(x);
    } else {
      alone.push_back(i);
    }
  }
  // refinement setup of every grouped system (as ir_solve)
  for (IrSys& x : st) {
    const krs_ir_system& q = *x.q;
    x.n = q.A64->n;
    x.ld = vec_ld(x.n);
    x.inner_bytes = std::max(ws_gmres<float>(x.n, o->m), ws_bicg<float>(x.n));
    Carver cv(q.ws, q.ws_bytes);
    x.inner = cv.take(x.inner_bytes);
    x.r64 = cv.vec<double>(x.ld);
    x.b32 = cv.vec<float>(x.ld);
    x.d32 = cv.vec<float>(x.ld);
    x.part = (double*)cv.take(partials_bytes(sizeof(double)));
    x.sc = cv.vec<double>(kScalarDoubles);
    if (!q.ws || !cv.ok) return set_err(ctx, KRS_ERR_WORKSPACE, "system workspace too small");
    Carver ci(x.inner, x.inner_bytes);
    x.r = ci.vec<float>(x.ld);
    x.rt = ci.vec<float>(x.ld);
    x.p = ci.vec<float>(x.ld);
    x.v = ci.vec<float>(x.ld);
    x.sv = ci.vec<float>(x.ld);
    x.t = ci.vec<float>(x.ld);
    x.z = ci.vec<float>(x.ld);
    x.y = ci.vec<float>(x.ld);
    x.ipart = (float*)ci.take(partials_bytes(sizeof(float)));
    x.isc = ci.vec<double>(kScalarDoubles);
    init_stats(q.stats);
    double nb2 = 0;
    int rc = norm2<double>(ctx, (const double*)q.b, x.n, x.part, x.sc, nb2);
    if (rc) return rc;
    x.nb = std::sqrt(nb2);
    KRS_LAUNCH(ctx, KRS_K_OTHER, 8.0 * x.n, fill<double>(s, (double*)q.x, x.n, 0.0));
    KRS_LAUNCH(ctx, KRS_K_OTHER, 16.0 * x.n, copy<double>(s, (const double*)q.b, x.r64, x.n));
    x.rn = x.nb;
    if (!(x.nb > 0)) {
      x.status = std::isfinite(x.nb) ? KRS_OK : KRS_DIVERGED;
      if (q.stats) {
        q.stats->status = x.status;
        q.stats->rel_res_true = 0;
      }
    } else {
      x.active = x.rn > o->tol * x.nb;
      if (!x.active) x.status = KRS_OK;
    }
  }
  BatchTable tb;
  std::vector<int> in_table;
  // one device-driven batch of rBiCGStab inner solves of the active systems
  auto inner_batch = [&](std::vector<IrSys*>& act) -> int {
    // setup of each inner solve, enqueued for all systems before one
    // synchronisation: the kernels rbicgstab_t runs (||b||, projection of b
    // against C, r~, C^T r~, p = r, zero y) and the starting state it forms on
    // the host, formed on the device (same values)
    std::vector<IrSys*> run;
    for (IrSys* x : act) {
      const krs_recycle* rec = x->q->rec32;
      const int kc = rec ? rec->dim : 0;
      const Cols<float> Cc = cols<float>(rec ? (const float*)rec->C : nullptr, rec ? rec->ld : 0,
                                         kc);
      const int nblk = std::min(red_blocks(x->n), 512);
      const int nred = red_blocks(x->n);
      const double NW = (double)x->n * sizeof(float);
      x->iits = 0;
      x->imv = 0;
      x->istatus = KRS_NOT_CONVERGED;
      x->inner_running = false;
      KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW,
                 block_dot<float>(s, Cols<float>{}, x->b32, x->n, 1, x->ipart, nred));
      KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<float>(s, x->ipart, nred, 1, x->isc + kBNb2));
      if (kc > 0) {
        KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW * (kc + 1),
                   block_dot<float>(s, Cc, x->b32, x->n, 0, x->ipart, nblk));
        KRS_LAUNCH(ctx, KRS_K_OTHER, 0,
                   finish_sum<float>(s, x->ipart, nblk, kc, x->isc + kBEta1));
        KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (kc + 2),
                   block_update<float>(s, Cc, x->isc + kBEta1, -1.0, x->b32, x->r, x->n, nullptr,
                                       1, x->ipart, nblk));
        KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<float>(s, x->ipart, nblk, 1, x->isc + kBNrm));
      } else {
        KRS_LAUNCH(ctx, KRS_K_OTHER, 2 * NW, copy<float>(s, x->b32, x->r, x->n));
      }
      KRS_LAUNCH(ctx, KRS_K_OTHER, 2 * NW, copy<float>(s, x->r, x->rt, x->n));
      if (kc > 0) {
        KRS_LAUNCH(ctx, KRS_K_BLOCK_DOT, NW * (kc + 1),
                   block_dot<float>(s, Cc, x->rt, x->n, 0, x->ipart, nblk));
        KRS_LAUNCH(ctx, KRS_K_OTHER, 0,
                   finish_sum<float>(s, x->ipart, nblk, kc, x->isc + kBCtrt));
      }
      KRS_LAUNCH(ctx, KRS_K_OTHER, 2 * NW, copy<float>(s, x->r, x->p, x->n));
      KRS_LAUNCH(ctx, KRS_K_OTHER, NW, fill<float>(s, x->y, x->n, 0.0));
      KRS_LAUNCH(ctx, KRS_K_OTHER, 0, bicg_setup(s, x->isc, kc, x->itol, io.div_factor));
    }
    for (size_t i = 0; i < act.size(); ++i)
      KRS_CHECK_HIP(ctx, hipMemcpyAsync(ctx->pin + 2 * i, act[i]->isc + kBNrm,
                                        2 * sizeof(double), hipMemcpyDeviceToHost, s));
    KRS_CHECK_HIP(ctx, hipStreamSynchronize(s));
    timing_flush(ctx);
    for (size_t i = 0; i < act.size(); ++i) {
      IrSys* x = act[i];
      const krs_recycle* rec = x->q->rec32;
      const int kc = rec ? rec->dim : 0;
      const double nb2 = ctx->pin[2 * i + 1];
      const double rn2 = kc > 0 ? ctx->pin[2 * i] : nb2;
      x->inb = std::sqrt(nb2);
      if (x->inb == 0 || !std::isfinite(x->inb)) {
        KRS_LAUNCH(ctx, KRS_K_OTHER, (double)x->n * sizeof(float),
                   fill<float>(s, x->d32, x->n, 0.0));
        x->istatus = std::isfinite(x->inb) ? KRS_OK : KRS_DIVERGED;
        continue;
      }
      x->irnorm = std::sqrt(rn2);
      if (x->irnorm > x->itol * x->inb) {
        x->inner_running = true;
        run.push_back(x);
      }
    }
    // the grouped iterations
    int64_t passes = 0;
    int batch = 2;
    double last = 0;
    for (IrSys* x : run) last = std::max(last, x->irnorm / x->inb);
    int64_t prev = 0;
    while (!run.empty() && passes < allowed) {
      tb.nsys = (int)run.size();
      for (int i = 0; i < tb.nsys; ++i) {
        IrSys* x = run[i];
        const krs_ir_system& q = *x->q;
        BatchSys& b = tb.sys[i];
        b.g = grid3(q.A32);
        b.bands = (const float*)q.A32->bands;
        b.pk = (const float*)q.M32->pack;
        b.nbx = b.g.nx / 16;
        b.nby = b.g.ny / 16;
        b.omega_l = (float)q.M32->d.omega_local;
        b.omega_g = (float)q.M32->d.omega_global;
        b.sweeps = q.M32->d.local_sweeps;
        const krs_recycle* rec = q.rec32;
        b.C = cols<float>(rec ? (const float*)rec->C : nullptr, rec ? rec->ld : 0,
                          rec ? rec->dim : 0);
        b.rt = x->rt;
        b.r = x->r;
        b.p = x->p;
        b.v = x->v;
        b.sv = x->sv;
        b.t = x->t;
        b.z = x->z;
        b.y = x->y;
        b.part = x->ipart;
        b.sc = x->isc;
        b.nblk = std::min(red_blocks(x->n), 512);
        // as in rbicgstab_t: after the dot passes' k_c + 2 columns
        b.part2 = b.part + (size_t)b.nblk * (b.C.n1 + 2);
        b.part3 = b.part2 + b.nblk;
        b.n = x->n;
        b.ld = x->ld;
      }
      batch_layout(tb);
      KRS_CHECK_HIP(ctx, hipStreamSynchronize(s));
      std::memcpy(ctx->pin + kPinDoubles / 2, &tb, sizeof(BatchTable));
      KRS_CHECK_HIP(ctx, hipMemcpyAsync(d_tb, ctx->pin + kPinDoubles / 2, sizeof(BatchTable),
                                        hipMemcpyHostToDevice, s));
      // optionally one pass of the table captured as a graph and replayed
      // (its launches read everything from the table and the scalar areas)
      hipGraphExec_t gexec = nullptr;
      if (use_graph) {
        if (!ctx->capture)
          KRS_CHECK_HIP(ctx, hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          hipError_t e1 = batch_bicg_first_half(ctx->capture, d_tb, tb, kc_all);
          hipError_t e2 = batch_bicg_second_half(ctx->capture, d_tb, tb, kc_all);
          e = hipStreamEndCapture(ctx->capture, &gr);
          if (e == hipSuccess) e = e1 != hipSuccess ? e1 : e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&gexec, gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
        if (e != hipSuccess)
          return set_err(ctx, KRS_ERR_HIP, std::string("batched graph: ") + hipGetErrorString(e));
      }
      struct GraphGuard {
        hipGraphExec_t& g;
        ~GraphGuard() {
          if (g) (void)hipGraphExecDestroy(g);
        }
      } guard{gexec};
      // passes until the active set changes (read once per batch of passes)
      while (passes < allowed) {
        const int kb = (int)std::min<int64_t>(batch, allowed - passes);
        for (int q = 0; q < kb; ++q) {
          if (gexec) {
            KRS_CHECK_HIP(ctx, hipGraphLaunch(gexec, s));
          } else {
            KRS_LAUNCH(ctx, KRS_K_OTHER, 0, batch_bicg_first_half(s, d_tb, tb, kc_all));
            KRS_LAUNCH(ctx, KRS_K_OTHER, 0, batch_bicg_second_half(s, d_tb, tb, kc_all));
          }
        }
        passes += kb;
        // the state of every system of the table, one synchronisation
        const int per = kHistOff + kHistRing;
        for (int i = 0; i < tb.nsys; ++i)
          KRS_CHECK_HIP(ctx, hipMemcpyAsync(ctx->pin + (size_t)i * per, run[i]->isc,
                                            sizeof(double) * per, hipMemcpyDeviceToHost, s));
        KRS_CHECK_HIP(ctx, hipStreamSynchronize(s));
        timing_flush(ctx);
        bool changed = false;
        double worst = 0;
        for (int i = 0; i < tb.nsys; ++i) {
          IrSys* x = run[i];
          const double* d = ctx->pin + (size_t)i * per;
          x->iits = (int64_t)d[kIts];
          const int done = (int)d[kDone];
          x->irnorm = std::sqrt(d[kRnorm2]);
          if (done != kRunning) {
            x->imv = 2 * x->iits - (d[kEndHalf] != 0.0 ? 1 : 0);
            if (done == kBreak) x->istatus = KRS_BREAKDOWN;
            else if (done == kDiverge) x->istatus = KRS_DIVERGED;
            x->inner_running = false;
            changed = true;
          } else {
            x->imv = 2 * x->iits;
            worst = std::max(worst, x->irnorm / x->inb);
          }
        }
        if (changed) break;
        // next batch: about half the iterations the slowest system still needs
        const int64_t dits = passes - prev;
        prev = passes;
        if (dits > 0 && worst > 0 && worst < last) {
          const double rate = std::pow(worst / last, 1.0 / (double)dits);
          double tmin = 1.0;
          for (IrSys* x : run) tmin = std::min(tmin, x->itol);
          const double need = std::log(tmin / worst) / std::log(rate);
          batch = (int)std::max(1.0, std::min(32.0, 0.5 * need));
        }
        last = worst;
      }
      std::vector<IrSys*> still;
      for (IrSys* x : run)
        if (x->inner_running) still.push_back(x);
      run.swap(still);
    }
    // finish every inner solve (as rbicgstab_t): status, postponed U-update,
    // x = M^-1 y
    for (IrSys* x : act) {
      if (x->inb == 0 || !std::isfinite(x->inb)) continue;
      if (x->istatus == KRS_NOT_CONVERGED && x->irnorm <= x->itol * x->inb) x->istatus = KRS_OK;
      const krs_recycle* rec = x->q->rec32;
      const int kc = rec ? rec->dim : 0;
      const int nblk = std::min(red_blocks(x->n), 512);
      const double NW = (double)x->n * sizeof(float);
      if (kc > 0) {
        KRS_LAUNCH(ctx, KRS_K_BLOCK_UPDATE, NW * (kc + 2),
                   block_update<float>(s, cols<float>((const float*)rec->U, rec->ld, kc),
                                       x->isc + kBXi, -1.0, x->y, x->y, x->n, nullptr, 0,
                                       x->ipart, nblk));
      }
      Op<float> op{ctx, x->q->A32, x->q->M32, grid3(x->q->A32), x->z, nullptr};
      int rc = op.minv_s(x->y, x->d32, x->z);
      if (rc) return rc;
    }
    return 0;
  };
  // refinement rounds over the systems still active
  while (true) {
    std::vector<IrSys*> act;
    for (IrSys& x : st)
      if (x.active) act.push_back(&x);
    if (act.empty()) break;
    for (IrSys* x : act) {
      x->itol = std::max(inner_floor, 0.5 * o->tol * x->nb / x->rn);
      const double sv[2] = {1.0 / x->rn, x->rn};
      int rc = upload(ctx, x->sc + 16, sv, 2);
      if (rc) return rc;
      KRS_LAUNCH(ctx, KRS_K_OTHER, 12.0 * x->n, cast_scale_f64_f32(s, x->r64, x->b32, x->n,
                                                                   x->sc + 16));
    }
    int rc = inner_batch(act);
    if (rc) return rc;
    for (IrSys* x : act) {
      x->its += x->iits;
      x->mv += x->imv;
      if (x->istatus == KRS_BREAKDOWN || x->istatus == KRS_DIVERGED) {
        // switch back to rGCROT for this correction (Sec. 2.4), as ir_solve
        krs_opts jo = io;
        jo.tol = x->itol;
        krs_stats ist;
        const int irc = gmres_rgcrot(ctx, x->q->A32, x->q->M32, x->q->rec32, true, x->b32,
                                     x->d32, &jo, x->inner, x->inner_bytes, &ist);
        if (irc < 0) return irc;
        x->its += ist.iterations;
        x->mv += ist.matvecs;
      }
      const Grid3 g = grid3(x->q->A64);
      const int nblk = red_blocks(x->n);
      KRS_LAUNCH(ctx, KRS_K_OTHER, 20.0 * x->n,
                 axpy_f32_into_f64(s, x->d32, (double*)x->q->x, x->n, x->sc + 17));
      KRS_LAUNCH(ctx, KRS_K_RESIDUAL, (8.0 * g.pts + 24.0) * x->n,
                 residual_norm<double>(s, g, (const double*)x->q->A64->bands,
                                       (const double*)x->q->x, (const double*)x->q->b, x->r64,
                                       x->part));
      KRS_LAUNCH(ctx, KRS_K_OTHER, 0, finish_sum<double>(s, x->part, nblk, 1, x->sc));
    }
    for (size_t i = 0; i < act.size(); ++i)
      KRS_CHECK_HIP(ctx, hipMemcpyAsync(ctx->pin + i, act[i]->sc, sizeof(double),
                                        hipMemcpyDeviceToHost, s));
    KRS_CHECK_HIP(ctx, hipStreamSynchronize(s));
    timing_flush(ctx);
    for (size_t i = 0; i < act.size(); ++i) {
      IrSys* x = act[i];
      const double rn_new = std::sqrt(ctx->pin[i]);
      ++x->outer;
      if (!std::isfinite(rn_new)) {
        x->status = KRS_DIVERGED;
        x->rn = rn_new;
        x->active = false;
        continue;
      }
      const bool stalled = rn_new > 0.9 * x->rn;
      x->rn = rn_new;
      if (x->rn <= o->tol * x->nb) {
        x->status = KRS_OK;
        x->active = false;
      } else if (stalled || x->outer >= max_outer) {
        x->active = false;
      }
    }
  }
  int worst = KRS_OK;
  for (IrSys& x : st) {
    if (x.q->stats && x.nb > 0) {
      krs_stats* so = x.q->stats;
      so->status = x.status;
      so->iterations = x.its;
      so->matvecs = x.mv;
      so->outer = x.outer;
      so->history_len = 0;
      so->rel_res_true = x.rn / x.nb;
      so->rel_res_est = x.rn / x.nb;
      so->solver = KRS_SOLVER_RBICGSTAB;
    }
    worst = std::max(worst, x.status);
  }
  for (int i : alone) {
    const krs_ir_system& q = sys[i];
    const int rc = ir_solve(ctx, q.A64, q.A32, q.M32, q.rec32, q.b, q.x, o, q.ws, q.ws_bytes,
                            q.stats);
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
  }
  return worst;
}

}  // namespace krs
