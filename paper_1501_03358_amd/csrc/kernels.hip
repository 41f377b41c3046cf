// HIP kernels for the recycling Krylov solvers on gfx950 (MI355X).
//
// Everything on the solve path is bound by HBM bandwidth (well under one
// flop per byte), so the kernels are written for coalesced streaming with
// wave64 shuffles and LDS for reductions; the Schwarz-Jacobi kernel keeps a
// (tile+2)^3 extended tile in LDS for its local sweeps.  Large launches remap
// block ids so that each of the 8 XCDs (each with its own L2) processes a
// contiguous range of the grid, which keeps stencil neighbours and tile halos
// in the same L2.
#include "kernels.hpp"

#include <cmath>

namespace krs {

namespace {

constexpr int kXcd = 8;

// Block b runs on XCD b % 8; give every XCD a contiguous range of work ids.
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int q = G / kXcd, r = G % kXcd;
  const int x = b % kXcd, s = b / kXcd;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + s;
}

template <class T>
__device__ __forceinline__ const T* col_ptr(const Cols<T>& Q, int c) {
  return c < Q.n1 ? Q.p1 + (int64_t)c * Q.ld1 : Q.p2 + (int64_t)(c - Q.n1) * Q.ld2;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 256 threads of a block; fixed order; result valid in all threads.
template <class T>
__device__ __forceinline__ T block_sum(T v) {
  __shared__ T sh[kThreads / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Block-reduce nv (<= NV) accumulators and store partials[c*nblk + blockIdx.x].
template <class T, int NV>
__device__ __forceinline__ void reduce_store(T (&acc)[NV], int nv, T* partials, int nblk) {
  __shared__ T sh[NV][kThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    if (c < nv) {
      T v = wave_sum(acc[c]);
      if (lane == 0) sh[c][wid] = v;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < nv; c += kThreads)
    partials[(int64_t)c * nblk + blockIdx.x] = (sh[c][0] + sh[c][1]) + (sh[c][2] + sh[c][3]);
}

// ---------------------------------------------------------------------------
// 7-point stencil: (A u)_i over the 7 bands, periodic wrap or dropped term
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T apply_row(const Grid3& g, const T* __restrict__ A,
                                       const T* __restrict__ x, int64_t i) {
  const int64_t N = g.n;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ii = (int)i;
  const int ix = ii % nx;
  const int t = ii / nx;
  const int iy = t % ny;
  const int iz = t / ny;
  const int64_t sxy = (int64_t)nx * ny;
  T ax = A[i] * x[i];
  if (ix > 0) ax += A[N + i] * x[i - 1];
  else if (g.px) ax += A[N + i] * x[i + nx - 1];
  if (ix < nx - 1) ax += A[2 * N + i] * x[i + 1];
  else if (g.px) ax += A[2 * N + i] * x[i - (nx - 1)];
  if (iy > 0) ax += A[3 * N + i] * x[i - nx];
  else if (g.py) ax += A[3 * N + i] * x[i + (int64_t)(ny - 1) * nx];
  if (iy < ny - 1) ax += A[4 * N + i] * x[i + nx];
  else if (g.py) ax += A[4 * N + i] * x[i - (int64_t)(ny - 1) * nx];
  if (iz > 0) ax += A[5 * N + i] * x[i - sxy];
  else if (g.pz) ax += A[5 * N + i] * x[i + (int64_t)(nz - 1) * sxy];
  if (iz < nz - 1) ax += A[6 * N + i] * x[i + sxy];
  else if (g.pz) ax += A[6 * N + i] * x[i - (int64_t)(nz - 1) * sxy];
  return ax;
}

// MODE 0: y = a*Ax; 1: y = a*Ax + b0*bv; 2: y = a*Ax + b0*y; 3: y = x + a*(bv - Ax)/C
template <class T, int MODE>
__global__ __launch_bounds__(kThreads) void k_stencil(Grid3 g, const T* __restrict__ A,
                                                       const T* __restrict__ x, T* y, T alpha,
                                                       T beta, const T* __restrict__ bv) {
  const int64_t i = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (i >= g.n) return;
  const T ax = apply_row(g, A, x, i);
  T out;
  if constexpr (MODE == 0) out = alpha * ax;
  else if constexpr (MODE == 1) out = alpha * ax + beta * bv[i];
  else if constexpr (MODE == 2) out = alpha * ax + beta * y[i];
  else out = x[i] + alpha * (bv[i] - ax) / A[i];
  y[i] = out;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_residual_norm(Grid3 g, const T* __restrict__ A,
                                                            const T* __restrict__ x,
                                                            const T* __restrict__ b,
                                                            T* __restrict__ y, T* partials) {
  T acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < g.n;
       i += (int64_t)gridDim.x * kThreads) {
    const T v = b[i] - apply_row(g, A, x, i);
    y[i] = v;
    acc += v * v;
  }
  const T s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_point_jacobi(int64_t n, const T* __restrict__ A,
                                                           const T* __restrict__ r,
                                                           T* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) z[i] = r[i] / A[i];
}

// ---------------------------------------------------------------------------
// Schwarz-Jacobi local solves: one block per tile, (TILE+2)^3 cells in LDS
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool wrap_coord(int& c, int n, int periodic) {
  if (c < 0) {
    if (!periodic) return false;
    c += n;
  } else if (c >= n) {
    if (!periodic) return false;
    c -= n;
  }
  return true;
}

template <class T, int TILE>
__global__ __launch_bounds__(kThreads) void k_schwarz_local(Grid3 g, const T* __restrict__ A,
                                                            const T* __restrict__ r,
                                                            T* __restrict__ z, T omega,
                                                            int sweeps, int ntx, int nty) {
  constexpr int E = TILE + 2;
  constexpr int NE = E * E * E;
  constexpr int PER = (NE + kThreads - 1) / kThreads;
  __shared__ T zs[2][NE];
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = tile % ntx;
  const int ty = (tile / ntx) % nty;
  const int tz = tile / (ntx * nty);
  const int64_t N = g.n;

  T a[PER][7];
  T rr[PER];
  T idg[PER];
  int gi[PER];
  unsigned nbm[PER];   // bit d: neighbour d (W,E,S,N,B,T) inside the extended tile
  unsigned ownm = 0;   // bit q: cell q is owned by this tile
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + kThreads * q;
#pragma unroll
    for (int d = 0; d < 7; ++d) a[q][d] = 0;
    rr[q] = 0;
    idg[q] = 0;
    gi[q] = -1;
    nbm[q] = 0;
    if (e < NE) {
      const int ex = e % E, ey = (e / E) % E, ez = e / (E * E);
      int gx = tx * TILE + ex - 1, gy = ty * TILE + ey - 1, gz = tz * TILE + ez - 1;
      const bool ok = wrap_coord(gx, g.nx, g.px) && wrap_coord(gy, g.ny, g.py) &&
                      wrap_coord(gz, g.nz, g.pz);
      nbm[q] = (ex > 0 ? 1u : 0u) | (ex < E - 1 ? 2u : 0u) | (ey > 0 ? 4u : 0u) |
               (ey < E - 1 ? 8u : 0u) | (ez > 0 ? 16u : 0u) | (ez < E - 1 ? 32u : 0u);
      if (ex >= 1 && ex <= TILE && ey >= 1 && ey <= TILE && ez >= 1 && ez <= TILE)
        ownm |= 1u << q;
      if (ok) {
        const int64_t i = gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz);
        gi[q] = (int)i;
#pragma unroll
        for (int d = 0; d < 7; ++d) a[q][d] = A[d * N + i];
        rr[q] = r[i];
        idg[q] = T(1) / a[q][0];
      }
      zs[0][e] = 0;
    }
  }
  __syncthreads();
  int cur = 0;
  for (int s = 0; s < sweeps; ++s) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + kThreads * q;
      if (e < NE) {
        const T* zc = zs[cur];
        const T zv = zc[e];
        T az = a[q][0] * zv;
        const unsigned m = nbm[q];
        if (m & 1u) az += a[q][1] * zc[e - 1];
        if (m & 2u) az += a[q][2] * zc[e + 1];
        if (m & 4u) az += a[q][3] * zc[e - E];
        if (m & 8u) az += a[q][4] * zc[e + E];
        if (m & 16u) az += a[q][5] * zc[e - E * E];
        if (m & 32u) az += a[q][6] * zc[e + E * E];
        zs[cur ^ 1][e] = zv + omega * (rr[q] - az) * idg[q];
      }
    }
    __syncthreads();
    cur ^= 1;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + kThreads * q;
    if (e < NE && ((ownm >> q) & 1u)) z[gi[q]] = zs[cur][e];
  }
}

// ---------------------------------------------------------------------------
// tall-skinny block products
// ---------------------------------------------------------------------------
template <class T, int NC>
__global__ __launch_bounds__(kThreads) void k_block_dot(Cols<T> Q, const T* __restrict__ w,
                                                        int64_t n, int self_dot, T* partials,
                                                        int nblk) {
  const int nc = Q.n1 + Q.n2;
  T acc[NC + 1];
#pragma unroll
  for (int c = 0; c <= NC; ++c) acc[c] = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    const T wi = w[i];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < nc) acc[c] += col_ptr(Q, c)[i] * wi;
    acc[NC] += wi * wi;
  }
  if (self_dot) {
    // move the self product next to the column products
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c == nc) acc[c] = acc[NC];
    if (nc == NC) { /* already in place at index NC */ }
  }
  reduce_store<T, NC + 1>(acc, nc + (self_dot ? 1 : 0), partials, nblk);
}

template <class T, int NC, bool NORM, bool SCALE, bool HAS_IN>
__global__ __launch_bounds__(kThreads) void k_block_update(Cols<T> Q, const double* coef, T sgn,
                                                           const T* w_in, T* w_out, int64_t n,
                                                           const double* scale, T* partials,
                                                           int nblk) {
  __shared__ T cf[NC];
  const int nc = Q.n1 + Q.n2;
  for (int c = threadIdx.x; c < nc; c += kThreads) cf[c] = sgn * (T)coef[c];
  __syncthreads();
  T sc = 1;
  if constexpr (SCALE) sc = (T)scale[0];
  T acc[1] = {0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    T v = 0;
    if constexpr (HAS_IN) v = w_in[i];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < nc) v += cf[c] * col_ptr(Q, c)[i];
    if constexpr (SCALE) v *= sc;
    w_out[i] = v;
    if constexpr (NORM) acc[0] += v * v;
  }
  if constexpr (NORM) reduce_store<T, 1>(acc, 1, partials, nblk);
}

template <class T, int NC>
__global__ __launch_bounds__(kThreads) void k_block_dot_after_update(Cols<T> Q,
                                                                     const double* coef,
                                                                     const T* __restrict__ w,
                                                                     int64_t n, T* partials,
                                                                     int nblk) {
  __shared__ T cf[NC];
  const int nc = Q.n1 + Q.n2;
  for (int c = threadIdx.x; c < nc; c += kThreads) cf[c] = (T)coef[c];
  __syncthreads();
  T acc[NC + 1];
#pragma unroll
  for (int c = 0; c <= NC; ++c) acc[c] = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    T q[NC];
    T v = w[i];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      q[c] = c < nc ? col_ptr(Q, c)[i] : T(0);
      v -= cf[c < nc ? c : 0] * q[c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] += q[c] * v;
    acc[NC] += v * v;
  }
  // place |v|^2 at index nc
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (c == nc) acc[c] = acc[NC];
  reduce_store<T, NC + 1>(acc, nc + 1, partials, nblk);
}

// Gram partials X^T Y: one wave per block; chunks of kGramRows rows of all
// columns are staged in LDS and every lane accumulates up to two 4 x 4 tiles
// of (a, b) pairs in registers (8 LDS reads per 16 FMAs).
constexpr int kGramRows = 16;
constexpr int kGramTile = 4;

template <class T>
__global__ __launch_bounds__(64) void k_gram(Cols<T> X, Cols<T> Y, int64_t n, T* partials,
                                             int nblk) {
  extern __shared__ unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);
  const int na = X.n1 + X.n2, nb = Y.n1 + Y.n2;
  const int nta = (na + kGramTile - 1) / kGramTile, ntb = (nb + kGramTile - 1) / kGramTile;
  const int lda = nta * kGramTile, ldb = ntb * kGramTile;
  T* ys = xs + kGramRows * lda;
  const int lane = threadIdx.x;
  T acc[2][kGramTile][kGramTile];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int i = 0; i < kGramTile; ++i)
#pragma unroll
      for (int j = 0; j < kGramTile; ++j) acc[q][i][j] = 0;
  const int t0 = lane, t1 = lane + 64;
  const int ta0 = t0 / ntb, tb0 = t0 % ntb, ta1 = t1 / ntb, tb1 = t1 % ntb;
  const bool v0 = t0 < nta * ntb, v1 = t1 < nta * ntb;
  for (int64_t r0 = (int64_t)blockIdx.x * kGramRows; r0 < n; r0 += (int64_t)gridDim.x * kGramRows) {
    for (int idx = lane; idx < kGramRows * lda; idx += 64) {
      const int c = idx / kGramRows, rr = idx % kGramRows;
      const int64_t i = r0 + rr;
      xs[rr * lda + c] = (c < na && i < n) ? col_ptr(X, c)[i] : T(0);
    }
    for (int idx = lane; idx < kGramRows * ldb; idx += 64) {
      const int c = idx / kGramRows, rr = idx % kGramRows;
      const int64_t i = r0 + rr;
      ys[rr * ldb + c] = (c < nb && i < n) ? col_ptr(Y, c)[i] : T(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < kGramRows; ++rr) {
      if (v0) {
        T xa[kGramTile], yb[kGramTile];
#pragma unroll
        for (int i = 0; i < kGramTile; ++i) xa[i] = xs[rr * lda + ta0 * kGramTile + i];
#pragma unroll
        for (int j = 0; j < kGramTile; ++j) yb[j] = ys[rr * ldb + tb0 * kGramTile + j];
#pragma unroll
        for (int i = 0; i < kGramTile; ++i)
#pragma unroll
          for (int j = 0; j < kGramTile; ++j) acc[0][i][j] += xa[i] * yb[j];
      }
      if (v1) {
        T xa[kGramTile], yb[kGramTile];
#pragma unroll
        for (int i = 0; i < kGramTile; ++i) xa[i] = xs[rr * lda + ta1 * kGramTile + i];
#pragma unroll
        for (int j = 0; j < kGramTile; ++j) yb[j] = ys[rr * ldb + tb1 * kGramTile + j];
#pragma unroll
        for (int i = 0; i < kGramTile; ++i)
#pragma unroll
          for (int j = 0; j < kGramTile; ++j) acc[1][i][j] += xa[i] * yb[j];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const bool v = q == 0 ? v0 : v1;
    if (!v) continue;
    const int ta = q == 0 ? ta0 : ta1, tb = q == 0 ? tb0 : tb1;
#pragma unroll
    for (int i = 0; i < kGramTile; ++i)
#pragma unroll
      for (int j = 0; j < kGramTile; ++j) {
        const int a = ta * kGramTile + i, b = tb * kGramTile + j;
        if (a < na && b < nb) partials[((int64_t)a * nb + b) * nblk + blockIdx.x] = acc[q][i][j];
      }
  }
}

template <class T, int NIN>
__global__ __launch_bounds__(kThreads) void k_row_transform(Cols<T> In, const double* M,
                                                            int nout, T* out, int64_t ldo,
                                                            int64_t n) {
  extern __shared__ unsigned char smem_raw[];
  T* Ms = reinterpret_cast<T*>(smem_raw);
  const int nin = In.n1 + In.n2;
  for (int idx = threadIdx.x; idx < nin * nout; idx += kThreads) Ms[idx] = (T)M[idx];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    T v[NIN];
#pragma unroll
    for (int c = 0; c < NIN; ++c) v[c] = c < nin ? col_ptr(In, c)[i] : T(0);
    for (int o = 0; o < nout; ++o) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < NIN; ++c)
        if (c < nin) s += v[c] * Ms[c + nin * o];
      out[(int64_t)o * ldo + i] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// finishing reductions (FP64, fixed order)
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kThreads) void k_finish_sum(const T* partials, int nblk,
                                                         double* out) {
  const int c = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) s += (double)partials[(int64_t)c * nblk + b];
  s = block_sum(s);
  if (threadIdx.x == 0) out[c] = s;
}

__global__ void k_cgs2_combine(int ncols, const double* h1, const double* h2, double* hcol,
                               double* inv, int* flag) {
  if (threadIdx.x != 0) return;
  double q = 0;
  for (int c = 0; c < ncols; ++c) {
    hcol[c] = h1[c] + h2[c];
    q += h2[c] * h2[c];
  }
  const double nrm2 = h2[ncols];
  double hn2 = nrm2 - q;
  int f = 0;
  if (!(hn2 > 0.5 * nrm2)) f = 1;  // second pass removed a large part: norm needs a pass
  if (hn2 < 0) hn2 = 0;
  const double hn = sqrt(hn2);
  hcol[ncols] = hn;
  inv[0] = hn > 0 ? 1.0 / hn : 0.0;
  flag[0] = f;
}

__global__ void k_set_norm(const double* nrm2, double* hcol_last, double* inv) {
  if (threadIdx.x != 0) return;
  const double hn = sqrt(nrm2[0] > 0 ? nrm2[0] : 0.0);
  hcol_last[0] = hn;
  inv[0] = hn > 0 ? 1.0 / hn : 0.0;
}

// ---------------------------------------------------------------------------
// BiCGStab passes
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kThreads) void k_bicg_p(const T* __restrict__ r, T* __restrict__ p,
                                                     const T* __restrict__ v, const double* sc,
                                                     int64_t n) {
  const T beta = (T)sc[kBeta], omega = (T)sc[kOmega];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

__global__ void k_bicg_alpha(const double* sums, int kc, double* sc, int off_eta1, int off_ctrt) {
  if (threadIdx.x != 0) return;
  double corr = 0;
  for (int c = 0; c < kc; ++c) {
    sc[off_eta1 + c] = sums[c];
    corr += sc[off_ctrt + c] * sums[c];
  }
  const double rtv = sums[kc] - corr;
  sc[kRtv] = rtv;
  if (rtv == 0.0 || !isfinite(rtv)) {
    sc[kAlpha] = 0.0;   // breakdown: leave s = r, the host stops
    sc[kFlag] = 1.0;
  } else {
    sc[kAlpha] = sc[kRho] / rtv;
  }
}

template <class T, int NC>
__global__ __launch_bounds__(kThreads) void k_bicg_sv(Cols<T> C, const T* __restrict__ r, T* v,
                                                      T* __restrict__ sv, const double* sc,
                                                      int off_eta1, int64_t n, T* partials,
                                                      int nblk) {
  __shared__ T cf[NC > 0 ? NC : 1];
  const int kc = C.n1;
  for (int c = threadIdx.x; c < kc; c += kThreads) cf[c] = (T)sc[off_eta1 + c];
  __syncthreads();
  const T alpha = (T)sc[kAlpha];
  T acc[1] = {0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    T vi = v[i];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < kc) vi -= cf[c] * C.p1[(int64_t)c * C.ld1 + i];
    if (NC > 0) v[i] = vi;
    const T si = r[i] - alpha * vi;
    sv[i] = si;
    acc[0] += si * si;
  }
  reduce_store<T, 1>(acc, 1, partials, nblk);
}

__global__ void k_bicg_omega(const double* sums, int kc, double* sc, int off_eta1, int off_eta2,
                             int off_xi) {
  if (threadIdx.x != 0) return;
  double q = 0;
  for (int c = 0; c < kc; ++c) {
    sc[off_eta2 + c] = sums[c];
    q += sums[c] * sums[c];
  }
  const double ts = sums[kc];
  const double tt = sums[kc + 1] - q;  // |t - C eta2|^2 with C^T C = I
  sc[kTs] = ts;
  sc[kTt] = tt;
  double omega = 0.0;  // t = 0 (breakdown): y += alpha p, r = s, the host stops
  if (tt > 0.0 && isfinite(tt)) omega = ts / tt;
  else sc[kFlag] = 2.0;
  sc[kOmega] = omega;
  const double alpha = sc[kAlpha];
  for (int c = 0; c < kc; ++c) sc[off_xi + c] += alpha * sc[off_eta1 + c] + omega * sc[off_eta2 + c];
}

template <class T, int NC>
__global__ __launch_bounds__(kThreads) void k_bicg_yr(Cols<T> C, const T* __restrict__ t,
                                                      const T* __restrict__ sv,
                                                      const T* __restrict__ p, T* __restrict__ y,
                                                      T* __restrict__ r, const T* __restrict__ rt,
                                                      const double* sc, int off_eta2, int64_t n,
                                                      T* partials, int nblk) {
  __shared__ T cf[NC > 0 ? NC : 1];
  const int kc = C.n1;
  for (int c = threadIdx.x; c < kc; c += kThreads) cf[c] = (T)sc[off_eta2 + c];
  __syncthreads();
  const T alpha = (T)sc[kAlpha], omega = (T)sc[kOmega];
  T acc[2] = {0, 0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    T ti = t[i];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < kc) ti -= cf[c] * C.p1[(int64_t)c * C.ld1 + i];
    const T si = sv[i];
    y[i] += alpha * p[i] + omega * si;
    const T ri = si - omega * ti;
    r[i] = ri;
    acc[0] += rt[i] * ri;
    acc[1] += ri * ri;
  }
  reduce_store<T, 2>(acc, 2, partials, nblk);
}

__global__ void k_bicg_rho(const double* sums, double* sc) {
  if (threadIdx.x != 0) return;
  const double rho = sums[0];
  sc[kRnorm2] = sums[1];
  sc[kRhoOld] = sc[kRho];
  sc[kBeta] = sc[kOmega] != 0.0 ? (rho / sc[kRho]) * (sc[kAlpha] / sc[kOmega]) : 0.0;
  sc[kRho] = rho;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_bicg_exit_s(const T* __restrict__ p, T* y,
                                                          const T* __restrict__ sv, T* r,
                                                          const double* sc, int64_t n) {
  const T alpha = (T)sc[kAlpha];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) {
    y[i] += alpha * p[i];
    r[i] = sv[i];
  }
}

__global__ void k_bicg_exit_xi(double* sc, int off_eta1, int off_xi, int kc) {
  if (threadIdx.x != 0) return;
  const double alpha = sc[kAlpha];
  for (int c = 0; c < kc; ++c) sc[off_xi + c] += alpha * sc[off_eta1 + c];
  sc[kRnorm2] = sc[kSnorm2];
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_fill(T* x, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) x[i] = v;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_copy(const T* __restrict__ x, T* __restrict__ y,
                                                   int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = x[i];
}

__global__ __launch_bounds__(kThreads) void k_cast_scale(const double* __restrict__ x,
                                                         float* __restrict__ y, int64_t n,
                                                         const double* scale) {
  const double s = scale[0];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = (float)(x[i] * s);
}

__global__ __launch_bounds__(kThreads) void k_axpy_f32_f64(const float* __restrict__ d,
                                                           double* __restrict__ x, int64_t n,
                                                           const double* scale) {
  const double s = scale[0];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) x[i] += s * (double)d[i];
}

inline int grid_for(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

template <int NC>
constexpr bool fits(int n) { return n <= NC; }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class T>
hipError_t stencil(hipStream_t s, const Grid3& g, const T* bands, const T* x, T* y, double alpha,
                   double beta, const T* b, int mode) {
  const int grid = grid_for(g.n);
  if (g.n == 0) return hipSuccess;
  switch (mode) {
    case 0: k_stencil<T, 0><<<grid, kThreads, 0, s>>>(g, bands, x, y, (T)alpha, (T)beta, b); break;
    case 1: k_stencil<T, 1><<<grid, kThreads, 0, s>>>(g, bands, x, y, (T)alpha, (T)beta, b); break;
    default: k_stencil<T, 2><<<grid, kThreads, 0, s>>>(g, bands, x, y, (T)alpha, (T)beta, b); break;
  }
  return hipGetLastError();
}

template <class T>
hipError_t residual_norm(hipStream_t s, const Grid3& g, const T* bands, const T* x, const T* b,
                         T* y, T* partials) {
  k_residual_norm<T><<<red_blocks(g.n), kThreads, 0, s>>>(g, bands, x, b, y, partials);
  return hipGetLastError();
}

template <class T>
hipError_t jacobi_sweep(hipStream_t s, const Grid3& g, const T* bands, const T* r, const T* zin,
                        T* zout, double omega) {
  if (g.n == 0) return hipSuccess;
  k_stencil<T, 3><<<grid_for(g.n), kThreads, 0, s>>>(g, bands, zin, zout, (T)omega, T(0), r);
  return hipGetLastError();
}

template <class T>
hipError_t point_jacobi(hipStream_t s, const Grid3& g, const T* bands, const T* r, T* z) {
  if (g.n == 0) return hipSuccess;
  k_point_jacobi<T><<<grid_for(g.n), kThreads, 0, s>>>(g.n, bands, r, z);
  return hipGetLastError();
}

template <class T>
hipError_t schwarz_local(hipStream_t s, const Grid3& g, int tile, const T* bands, const T* r, T* z,
                         double omega, int sweeps) {
  const int ntx = g.nx / tile, nty = g.ny / tile, ntz = g.nz / tile;
  const int nt = ntx * nty * ntz;
  if (nt == 0) return hipSuccess;
  if (tile == 8)
    k_schwarz_local<T, 8><<<nt, kThreads, 0, s>>>(g, bands, r, z, (T)omega, sweeps, ntx, nty);
  else if (tile == 4)
    k_schwarz_local<T, 4><<<nt, kThreads, 0, s>>>(g, bands, r, z, (T)omega, sweeps, ntx, nty);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

#define KRS_NC_DISPATCH(ncount, KERNEL_CALL) \
  do {                                       \
    const int _n = (ncount);                 \
    if (_n <= 8) { constexpr int NCB = 8; KERNEL_CALL; }          \
    else if (_n <= 16) { constexpr int NCB = 16; KERNEL_CALL; }   \
    else if (_n <= 32) { constexpr int NCB = 32; KERNEL_CALL; }   \
    else if (_n <= 64) { constexpr int NCB = 64; KERNEL_CALL; }   \
    else return hipErrorInvalidValue;        \
  } while (0)

template <class T>
hipError_t block_dot(hipStream_t s, const Cols<T>& Q, const T* w, int64_t n, int self_dot,
                     T* partials, int nblk) {
  KRS_NC_DISPATCH(Q.count() > 0 ? Q.count() : 1,
                  (k_block_dot<T, NCB><<<nblk, kThreads, 0, s>>>(Q, w, n, self_dot, partials, nblk)));
  return hipGetLastError();
}

template <class T>
hipError_t block_update(hipStream_t s, const Cols<T>& Q, const double* coef, double sgn,
                        const T* w_in, T* w_out, int64_t n, const double* scale, int dots,
                        T* partials, int nblk) {
  const bool norm = dots > 0, sc = scale != nullptr, in = w_in != nullptr;
  const int nc = Q.count() > 0 ? Q.count() : 1;
#define KRS_BU(NORM, SC, IN)                                                                   \
  KRS_NC_DISPATCH(nc, (k_block_update<T, NCB, NORM, SC, IN><<<nblk, kThreads, 0, s>>>(        \
                          Q, coef, (T)sgn, w_in, w_out, n, scale, partials, nblk)))
  if (norm) {
    if (sc) { if (in) KRS_BU(true, true, true); else KRS_BU(true, true, false); }
    else { if (in) KRS_BU(true, false, true); else KRS_BU(true, false, false); }
  } else {
    if (sc) { if (in) KRS_BU(false, true, true); else KRS_BU(false, true, false); }
    else { if (in) KRS_BU(false, false, true); else KRS_BU(false, false, false); }
  }
#undef KRS_BU
  return hipGetLastError();
}

template <class T>
hipError_t block_dot_after_update(hipStream_t s, const Cols<T>& Q, const double* coef,
                                  const T* w, int64_t n, T* partials, int nblk) {
  KRS_NC_DISPATCH(Q.count() > 0 ? Q.count() : 1,
                  (k_block_dot_after_update<T, NCB><<<nblk, kThreads, 0, s>>>(Q, coef, w, n,
                                                                               partials, nblk)));
  return hipGetLastError();
}

template <class T>
hipError_t gram(hipStream_t s, const Cols<T>& X, const Cols<T>& Y, int64_t n, T* partials,
                int nblk) {
  const int na = X.count(), nb = Y.count();
  if (na == 0 || nb == 0) return hipSuccess;
  const int nta = (na + kGramTile - 1) / kGramTile, ntb = (nb + kGramTile - 1) / kGramTile;
  if (nta * ntb > 128) return hipErrorInvalidValue;   // two 4 x 4 tiles per lane
  const size_t smem = sizeof(T) * kGramRows * kGramTile * (nta + ntb);
  k_gram<T><<<nblk, 64, smem, s>>>(X, Y, n, partials, nblk);
  return hipGetLastError();
}

template <class T>
hipError_t row_transform(hipStream_t s, const Cols<T>& In, const double* M, int nout, T* out,
                         int64_t ldo, int64_t n) {
  const int nin = In.count();
  if (nout == 0 || n == 0) return hipSuccess;
  const size_t smem = sizeof(T) * (size_t)nin * nout;
  if (smem > 64 * 1024) return hipErrorInvalidValue;
  int grid = grid_for(n);
  if (grid > 4 * kMaxRedBlocks) grid = 4 * kMaxRedBlocks;
  if (nin <= 8) k_row_transform<T, 8><<<grid, kThreads, smem, s>>>(In, M, nout, out, ldo, n);
  else if (nin <= 16) k_row_transform<T, 16><<<grid, kThreads, smem, s>>>(In, M, nout, out, ldo, n);
  else if (nin <= 32) k_row_transform<T, 32><<<grid, kThreads, smem, s>>>(In, M, nout, out, ldo, n);
  else if (nin <= 64) k_row_transform<T, 64><<<grid, kThreads, smem, s>>>(In, M, nout, out, ldo, n);
  else if (nin <= 96) k_row_transform<T, 96><<<grid, kThreads, smem, s>>>(In, M, nout, out, ldo, n);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class T>
hipError_t finish_sum(hipStream_t s, const T* partials, int nblk, int ncols, double* out) {
  if (ncols == 0) return hipSuccess;
  k_finish_sum<T><<<ncols, kThreads, 0, s>>>(partials, nblk, out);
  return hipGetLastError();
}

template <class T>
hipError_t finish_cgs2(hipStream_t s, const T* partials, int nblk, int ncols, const double* h1,
                       double* h2, double* hcol, double* inv, int* flag) {
  k_finish_sum<T><<<ncols + 1, kThreads, 0, s>>>(partials, nblk, h2);
  k_cgs2_combine<<<1, 64, 0, s>>>(ncols, h1, h2, hcol, inv, flag);
  return hipGetLastError();
}

hipError_t set_norm_from_sum(hipStream_t s, const double* nrm2, double* hcol_last, double* inv) {
  k_set_norm<<<1, 64, 0, s>>>(nrm2, hcol_last, inv);
  return hipGetLastError();
}

template <class T>
hipError_t bicg_p(hipStream_t s, const T* r, T* p, const T* v, const double* sc, int64_t n) {
  if (n == 0) return hipSuccess;
  k_bicg_p<T><<<grid_for(n), kThreads, 0, s>>>(r, p, v, sc, n);
  return hipGetLastError();
}

template <class T>
hipError_t bicg_sv(hipStream_t s, const Cols<T>& C, const T* r, T* v, T* sv, const double* sc,
                   int off_eta1, int64_t n, T* partials, int nblk) {
  const int kc = C.n1;
  if (kc == 0) k_bicg_sv<T, 0><<<nblk, kThreads, 0, s>>>(C, r, v, sv, sc, off_eta1, n, partials, nblk);
  else if (kc <= 8) k_bicg_sv<T, 8><<<nblk, kThreads, 0, s>>>(C, r, v, sv, sc, off_eta1, n, partials, nblk);
  else if (kc <= 16) k_bicg_sv<T, 16><<<nblk, kThreads, 0, s>>>(C, r, v, sv, sc, off_eta1, n, partials, nblk);
  else if (kc <= 32) k_bicg_sv<T, 32><<<nblk, kThreads, 0, s>>>(C, r, v, sv, sc, off_eta1, n, partials, nblk);
  else if (kc <= 64) k_bicg_sv<T, 64><<<nblk, kThreads, 0, s>>>(C, r, v, sv, sc, off_eta1, n, partials, nblk);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class T>
hipError_t bicg_yr(hipStream_t s, const Cols<T>& C, const T* t, const T* sv, const T* p, T* y,
                   T* r, const T* rt, const double* sc, int off_eta2, int64_t n, T* partials,
                   int nblk) {
  const int kc = C.n1;
#define KRS_YR(NCV) k_bicg_yr<T, NCV><<<nblk, kThreads, 0, s>>>(C, t, sv, p, y, r, rt, sc, off_eta2, n, partials, nblk)
  if (kc == 0) KRS_YR(0);
  else if (kc <= 8) KRS_YR(8);
  else if (kc <= 16) KRS_YR(16);
  else if (kc <= 32) KRS_YR(32);
  else if (kc <= 64) KRS_YR(64);
  else return hipErrorInvalidValue;
#undef KRS_YR
  return hipGetLastError();
}

hipError_t bicg_alpha(hipStream_t s, const double* sums, int kc, double* sc, int off_eta1,
                      int off_ctrt) {
  k_bicg_alpha<<<1, 64, 0, s>>>(sums, kc, sc, off_eta1, off_ctrt);
  return hipGetLastError();
}
hipError_t bicg_omega(hipStream_t s, const double* sums, int kc, double* sc, int off_eta1,
                      int off_eta2, int off_xi) {
  k_bicg_omega<<<1, 64, 0, s>>>(sums, kc, sc, off_eta1, off_eta2, off_xi);
  return hipGetLastError();
}
hipError_t bicg_rho(hipStream_t s, const double* sums, double* sc) {
  k_bicg_rho<<<1, 64, 0, s>>>(sums, sc);
  return hipGetLastError();
}

template <class T>
hipError_t bicg_exit_s(hipStream_t s, const T* p, T* y, const T* sv, T* r, double* sc,
                       int off_eta1, int off_xi, int kc, int64_t n) {
  if (n > 0) k_bicg_exit_s<T><<<grid_for(n), kThreads, 0, s>>>(p, y, sv, r, sc, n);
  k_bicg_exit_xi<<<1, 64, 0, s>>>(sc, off_eta1, off_xi, kc);
  return hipGetLastError();
}

template <class T>
hipError_t fill(hipStream_t s, T* x, int64_t n, double v) {
  if (n == 0) return hipSuccess;
  k_fill<T><<<grid_for(n), kThreads, 0, s>>>(x, n, (T)v);
  return hipGetLastError();
}

template <class T>
hipError_t copy(hipStream_t s, const T* x, T* y, int64_t n) {
  if (n == 0) return hipSuccess;
  k_copy<T><<<grid_for(n), kThreads, 0, s>>>(x, y, n);
  return hipGetLastError();
}

hipError_t cast_scale_f64_f32(hipStream_t s, const double* x, float* y, int64_t n,
                              const double* scale) {
  if (n == 0) return hipSuccess;
  k_cast_scale<<<grid_for(n), kThreads, 0, s>>>(x, y, n, scale);
  return hipGetLastError();
}

hipError_t axpy_f32_into_f64(hipStream_t s, const float* d, double* x, int64_t n,
                             const double* scale) {
  if (n == 0) return hipSuccess;
  k_axpy_f32_f64<<<grid_for(n), kThreads, 0, s>>>(d, x, n, scale);
  return hipGetLastError();
}

#define KRS_INSTANTIATE(T)                                                                        \
  template hipError_t stencil<T>(hipStream_t, const Grid3&, const T*, const T*, T*, double,       \
                                 double, const T*, int);                                          \
  template hipError_t residual_norm<T>(hipStream_t, const Grid3&, const T*, const T*, const T*,   \
                                       T*, T*);                                                   \
  template hipError_t jacobi_sweep<T>(hipStream_t, const Grid3&, const T*, const T*, const T*,    \
                                      T*, double);                                                \
  template hipError_t point_jacobi<T>(hipStream_t, const Grid3&, const T*, const T*, T*);         \
  template hipError_t schwarz_local<T>(hipStream_t, const Grid3&, int, const T*, const T*, T*,    \
                                       double, int);                                              \
  template hipError_t block_dot<T>(hipStream_t, const Cols<T>&, const T*, int64_t, int, T*, int); \
  template hipError_t block_update<T>(hipStream_t, const Cols<T>&, const double*, double,         \
                                      const T*, T*, int64_t, const double*, int, T*, int);        \
  template hipError_t block_dot_after_update<T>(hipStream_t, const Cols<T>&, const double*,       \
                                                const T*, int64_t, T*, int);                      \
  template hipError_t gram<T>(hipStream_t, const Cols<T>&, const Cols<T>&, int64_t, T*, int);     \
  template hipError_t row_transform<T>(hipStream_t, const Cols<T>&, const double*, int, T*,       \
                                       int64_t, int64_t);                                         \
  template hipError_t finish_sum<T>(hipStream_t, const T*, int, int, double*);                    \
  template hipError_t finish_cgs2<T>(hipStream_t, const T*, int, int, const double*, double*,     \
                                     double*, double*, int*);                                     \
  template hipError_t bicg_p<T>(hipStream_t, const T*, T*, const T*, const double*, int64_t);     \
  template hipError_t bicg_sv<T>(hipStream_t, const Cols<T>&, const T*, T*, T*, const double*,    \
                                 int, int64_t, T*, int);                                          \
  template hipError_t bicg_yr<T>(hipStream_t, const Cols<T>&, const T*, const T*, const T*, T*,   \
                                 T*, const T*, const double*, int, int64_t, T*, int);             \
  template hipError_t bicg_exit_s<T>(hipStream_t, const T*, T*, const T*, T*, double*, int, int,  \
                                     int, int64_t);                                               \
  template hipError_t fill<T>(hipStream_t, T*, int64_t, double);                                  \
  template hipError_t copy<T>(hipStream_t, const T*, T*, int64_t);

KRS_INSTANTIATE(double)
KRS_INSTANTIATE(float)

}  // namespace krs
