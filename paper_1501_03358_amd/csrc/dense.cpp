// Small dense FP64 linear algebra for the cycle-end steps (host).
#include "dense.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace krs {
namespace dense {

namespace {
constexpr double kEps = std::numeric_limits<double>::epsilon();
}

void qr_thin(int m, int n, const double* A, double* Q, double* R) {
  std::vector<double> W(A, A + (size_t)m * n);
  std::vector<double> V((size_t)m * n, 0.0);  // Householder vectors (unit)
  auto w = [&](int i, int j) -> double& { return W[i + (size_t)m * j]; };
  for (int j = 0; j < n; ++j) {
    double nx = 0;
    for (int i = j; i < m; ++i) nx += w(i, j) * w(i, j);
    nx = std::sqrt(nx);
    double* v = &V[(size_t)m * j];
    if (nx == 0) continue;
    const double alpha = w(j, j) > 0 ? -nx : nx;
    for (int i = j; i < m; ++i) v[i] = w(i, j);
    v[j] -= alpha;
    double vn = 0;
    for (int i = j; i < m; ++i) vn += v[i] * v[i];
    vn = std::sqrt(vn);
    if (vn == 0) continue;
    for (int i = j; i < m; ++i) v[i] /= vn;
    for (int c = j; c < n; ++c) {
      double s = 0;
      for (int i = j; i < m; ++i) s += v[i] * w(i, c);
      for (int i = j; i < m; ++i) w(i, c) -= 2 * s * v[i];
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) R[i + (size_t)n * j] = i <= j ? w(i, j) : 0.0;
  // Q = H_0 ... H_{n-1} [I; 0]
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) Q[i + (size_t)m * j] = (i == j) ? 1.0 : 0.0;
  for (int h = n - 1; h >= 0; --h) {
    const double* v = &V[(size_t)m * h];
    for (int c = 0; c < n; ++c) {
      double s = 0;
      for (int i = h; i < m; ++i) s += v[i] * Q[i + (size_t)m * c];
      for (int i = h; i < m; ++i) Q[i + (size_t)m * c] -= 2 * s * v[i];
    }
  }
  for (int i = 0; i < n; ++i) {
    if (R[i + (size_t)n * i] < 0) {
      for (int j = 0; j < n; ++j) R[i + (size_t)n * j] = -R[i + (size_t)n * j];
      for (int r = 0; r < m; ++r) Q[r + (size_t)m * i] = -Q[r + (size_t)m * i];
    }
  }
}

bool sym_eig(int n, const double* A, std::vector<double>& w, std::vector<double>& Z) {
  std::vector<double> M(A, A + (size_t)n * n);
  auto m = [&](int i, int j) -> double& { return M[i + (size_t)n * j]; };
  Z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Z[i + (size_t)n * i] = 1.0;
  bool ok = false;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0, tot = 0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        tot += m(i, j) * m(i, j);
        if (i != j) off += m(i, j) * m(i, j);
      }
    if (off <= (n * kEps) * (n * kEps) * tot || off == 0) {
      ok = true;
      break;
    }
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = m(p, q);
        if (apq == 0) continue;
        // rotation that zeroes (p, q): tan of the angle from the classical formula
        const double theta = (m(q, q) - m(p, p)) / (2 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        const double c = 1 / std::sqrt(t * t + 1), sn = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double mkp = m(k, p), mkq = m(k, q);
          m(k, p) = c * mkp - sn * mkq;
          m(k, q) = sn * mkp + c * mkq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double mpk = m(p, k), mqk = m(q, k);
          m(p, k) = c * mpk - sn * mqk;
          m(q, k) = sn * mpk + c * mqk;
        }
        for (int k = 0; k < n; ++k) {
          const double zkp = Z[k + (size_t)n * p], zkq = Z[k + (size_t)n * q];
          Z[k + (size_t)n * p] = c * zkp - sn * zkq;
          Z[k + (size_t)n * q] = sn * zkp + c * zkq;
        }
      }
  }
  // sort descending
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return m(a, a) > m(b, b); });
  std::vector<double> Zs((size_t)n * n);
  w.assign(n, 0.0);
  for (int c = 0; c < n; ++c) {
    w[c] = m(idx[c], idx[c]);
    for (int i = 0; i < n; ++i) Zs[i + (size_t)n * c] = Z[i + (size_t)n * idx[c]];
  }
  Z.swap(Zs);
  return ok;
}

bool cholesky_upper(int n, const double* A, double* R) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) R[i + (size_t)n * j] = 0;
  for (int j = 0; j < n; ++j) {
    double d = A[j + (size_t)n * j];
    for (int k = 0; k < j; ++k) d -= R[k + (size_t)n * j] * R[k + (size_t)n * j];
    if (!(d > 0)) return false;
    const double rjj = std::sqrt(d);
    R[j + (size_t)n * j] = rjj;
    for (int c = j + 1; c < n; ++c) {
      double s = A[j + (size_t)n * c];
      for (int k = 0; k < j; ++k) s -= R[k + (size_t)n * j] * R[k + (size_t)n * c];
      R[j + (size_t)n * c] = s / rjj;
    }
  }
  return true;
}

bool upper_inverse(int n, const double* R, double* Ri) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) Ri[i + (size_t)n * j] = 0;
  for (int j = 0; j < n; ++j) {
    if (R[j + (size_t)n * j] == 0) return false;
    // column j of R^-1: solve R x = e_j
    Ri[j + (size_t)n * j] = 1.0 / R[j + (size_t)n * j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0;
      for (int k = i + 1; k <= j; ++k) s += R[i + (size_t)n * k] * Ri[k + (size_t)n * j];
      Ri[i + (size_t)n * j] = -s / R[i + (size_t)n * i];
    }
  }
  return true;
}

void upper_solve(int n, const double* R, int ldr, const double* g, double* y) {
  for (int i = n - 1; i >= 0; --i) {
    double s = g[i];
    for (int k = i + 1; k < n; ++k) s -= R[i + (size_t)ldr * k] * y[k];
    y[i] = s / R[i + (size_t)ldr * i];
  }
}

namespace {

// P = I - beta v v^T with P x = alpha e1 for x of length len (2 or 3).
void reflector(const double* x, int len, double* v, double& beta) {
  double nx = 0;
  for (int i = 0; i < len; ++i) nx += x[i] * x[i];
  nx = std::sqrt(nx);
  for (int i = 0; i < len; ++i) v[i] = x[i];
  if (nx == 0) {
    beta = 0;
    return;
  }
  const double alpha = x[0] > 0 ? -nx : nx;
  v[0] -= alpha;
  double vv = 0;
  for (int i = 0; i < len; ++i) vv += v[i] * v[i];
  beta = vv > 0 ? 2.0 / vv : 0.0;
}

void eig2(double a, double b, double c, double d, cplx& l1, cplx& l2) {
  const double p = 0.5 * (a - d);
  const double disc = p * p + b * c;
  const double mid = 0.5 * (a + d);
  if (disc >= 0) {
    const double sq = std::sqrt(disc);
    const double big = mid + (mid >= 0 ? sq : -sq);
    const double det = a * d - b * c;
    const double small = big != 0 ? det / big : mid - (mid >= 0 ? sq : -sq);
    l1 = cplx(big, 0);
    l2 = cplx(small, 0);
  } else {
    const double sq = std::sqrt(-disc);
    l1 = cplx(mid, sq);
    l2 = cplx(mid, -sq);
  }
}

}  // namespace

bool eigenvalues(int n, const double* A, std::vector<cplx>& lam) {
  lam.assign(n, cplx(0, 0));
  if (n == 0) return true;
  std::vector<double> H(A, A + (size_t)n * n);
  auto h = [&](int i, int j) -> double& { return H[i + (size_t)n * j]; };
  double anorm = 0;
  for (double v : H) anorm = std::max(anorm, std::fabs(v));
  if (anorm == 0) return true;
  // Householder reduction to upper Hessenberg form
  std::vector<double> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    double nx = 0;
    for (int i = k + 1; i < n; ++i) nx += h(i, k) * h(i, k);
    nx = std::sqrt(nx);
    if (nx == 0) continue;
    const double alpha = h(k + 1, k) > 0 ? -nx : nx;
    std::fill(v.begin(), v.end(), 0.0);
    for (int i = k + 1; i < n; ++i) v[i] = h(i, k);
    v[k + 1] -= alpha;
    double vv = 0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0) continue;
    const double beta = 2.0 / vv;
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int i = k + 1; i < n; ++i) s += v[i] * h(i, j);
      s *= beta;
      for (int i = k + 1; i < n; ++i) h(i, j) -= s * v[i];
    }
    for (int i = 0; i < n; ++i) {
      double s = 0;
      for (int j = k + 1; j < n; ++j) s += h(i, j) * v[j];
      s *= beta;
      for (int j = k + 1; j < n; ++j) h(i, j) -= s * v[j];
    }
    for (int i = k + 2; i < n; ++i) h(i, k) = 0;
  }
  // implicit double-shift QR on the active window [lo, hi]
  int hi = n - 1;
  int iter = 0, total = 0;
  while (hi >= 0) {
    if (hi == 0) {
      lam[0] = cplx(h(0, 0), 0);
      --hi;
      continue;
    }
    int l = hi;
    while (l > 0) {
      double s = std::fabs(h(l - 1, l - 1)) + std::fabs(h(l, l));
      if (s == 0) s = anorm;
      if (std::fabs(h(l, l - 1)) <= kEps * s) {
        h(l, l - 1) = 0;
        break;
      }
      --l;
    }
    if (l == hi) {
      lam[hi] = cplx(h(hi, hi), 0);
      --hi;
      iter = 0;
      continue;
    }
    if (l == hi - 1) {
      eig2(h(hi - 1, hi - 1), h(hi - 1, hi), h(hi, hi - 1), h(hi, hi), lam[hi - 1], lam[hi]);
      hi -= 2;
      iter = 0;
      continue;
    }
    ++iter;
    if (++total > 60 * n) return false;
    double s, t;
    if (iter % 11 == 10) {  // exceptional shift
      const double w = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
      s = 1.5 * w;
      t = w * w;
    } else {
      s = h(hi - 1, hi - 1) + h(hi, hi);
      t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
    }
    double x[3];
    x[0] = h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - s * h(l, l) + t;
    x[1] = h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - s);
    x[2] = h(l + 1, l) * h(l + 2, l + 1);
    for (int k = l; k <= hi - 2; ++k) {
      double vr[3], beta;
      reflector(x, 3, vr, beta);
      if (beta != 0) {
        const int q = std::max(l, k - 1);
        for (int j = q; j <= hi; ++j) {
          double sdot = vr[0] * h(k, j) + vr[1] * h(k + 1, j) + vr[2] * h(k + 2, j);
          sdot *= beta;
          h(k, j) -= sdot * vr[0];
          h(k + 1, j) -= sdot * vr[1];
          h(k + 2, j) -= sdot * vr[2];
        }
        const int r = std::min(k + 3, hi);
        for (int i = l; i <= r; ++i) {
          double sdot = h(i, k) * vr[0] + h(i, k + 1) * vr[1] + h(i, k + 2) * vr[2];
          sdot *= beta;
          h(i, k) -= sdot * vr[0];
          h(i, k + 1) -= sdot * vr[1];
          h(i, k + 2) -= sdot * vr[2];
        }
      }
      x[0] = h(k + 1, k);
      x[1] = h(k + 2, k);
      if (k < hi - 2) x[2] = h(k + 3, k);
    }
    double vr[3], beta;
    reflector(x, 2, vr, beta);
    if (beta != 0) {
      for (int j = hi - 2; j <= hi; ++j) {
        if (j < l) continue;
        double sdot = vr[0] * h(hi - 1, j) + vr[1] * h(hi, j);
        sdot *= beta;
        h(hi - 1, j) -= sdot * vr[0];
        h(hi, j) -= sdot * vr[1];
      }
      for (int i = l; i <= hi; ++i) {
        double sdot = h(i, hi - 1) * vr[0] + h(i, hi) * vr[1];
        sdot *= beta;
        h(i, hi - 1) -= sdot * vr[0];
        h(i, hi) -= sdot * vr[1];
      }
    }
  }
  return true;
}

void eigenvector(int n, const double* A, cplx mu, const std::vector<cplx>& start,
                 const std::vector<cplx>& against, int na, std::vector<cplx>& v) {
  double anorm = 0;
  for (int i = 0; i < n * n; ++i) anorm = std::max(anorm, std::fabs(A[i]));
  const double tiny = kEps * std::max(anorm, 1e-300);
  // LU with partial pivoting of (A - mu I)
  std::vector<cplx> M((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) M[i + (size_t)n * j] = cplx(A[i + (size_t)n * j], 0) - (i == j ? mu : 0.0);
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(M[k + (size_t)n * k]);
    for (int i = k + 1; i < n; ++i)
      if (std::abs(M[i + (size_t)n * k]) > best) {
        best = std::abs(M[i + (size_t)n * k]);
        p = i;
      }
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(M[k + (size_t)n * j], M[p + (size_t)n * j]);
    if (std::abs(M[k + (size_t)n * k]) < tiny) M[k + (size_t)n * k] = tiny;
    for (int i = k + 1; i < n; ++i) {
      const cplx f = M[i + (size_t)n * k] / M[k + (size_t)n * k];
      M[i + (size_t)n * k] = f;
      for (int j = k + 1; j < n; ++j) M[i + (size_t)n * j] -= f * M[k + (size_t)n * j];
    }
  }
  auto project = [&](std::vector<cplx>& x) {
    for (int a = 0; a < na; ++a) {
      cplx d = 0;
      for (int i = 0; i < n; ++i) d += std::conj(against[i + (size_t)n * a]) * x[i];
      for (int i = 0; i < n; ++i) x[i] -= d * against[i + (size_t)n * a];
    }
  };
  auto normalize = [&](std::vector<cplx>& x) {
    double s = 0;
    for (auto& c : x) s += std::norm(c);
    s = std::sqrt(s);
    if (s > 0)
      for (auto& c : x) c /= s;
  };
  v = start;
  project(v);
  normalize(v);
  for (int it = 0; it < 3; ++it) {
    for (int k = 0; k < n; ++k) std::swap(v[k], v[piv[k]]);
    for (int i = 1; i < n; ++i)
      for (int k = 0; k < i; ++k) v[i] -= M[i + (size_t)n * k] * v[k];
    for (int i = n - 1; i >= 0; --i) {
      cplx s = v[i];
      for (int k = i + 1; k < n; ++k) s -= M[i + (size_t)n * k] * v[k];
      v[i] = s / M[i + (size_t)n * i];
    }
    project(v);
    normalize(v);
  }
}

bool harmonic_ritz_select(int mg, int ng, const double* G, const double* F, int k,
                          std::vector<double>& P, int& kk, int& ties) {
  ties = 0;
  std::vector<double> QG((size_t)mg * ng), RG((size_t)ng * ng), RGi((size_t)ng * ng);
  qr_thin(mg, ng, G, QG.data(), RG.data());
  if (!upper_inverse(ng, RG.data(), RGi.data())) return false;
  // S = QG^T F RG^-1 ; the pencil G^T G z = theta G^T F z becomes S w = (1/theta) w, z = RG^-1 w
  std::vector<double> X((size_t)ng * ng, 0.0), S((size_t)ng * ng, 0.0);
  for (int j = 0; j < ng; ++j)
    for (int i = 0; i < ng; ++i) {
      double s = 0;
      for (int r = 0; r < mg; ++r) s += QG[r + (size_t)mg * i] * F[r + (size_t)mg * j];
      X[i + (size_t)ng * j] = s;
    }
  for (int j = 0; j < ng; ++j)
    for (int i = 0; i < ng; ++i) {
      double s = 0;
      for (int c = 0; c <= j; ++c) s += X[i + (size_t)ng * c] * RGi[c + (size_t)ng * j];
      S[i + (size_t)ng * j] = s;
    }
  std::vector<cplx> mu;
  if (!eigenvalues(ng, S.data(), mu)) return false;
  // order by |theta| ascending == |mu| descending (mu = 0: theta infinite, last)
  std::vector<int> order(ng);
  for (int i = 0; i < ng; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double ma = std::abs(mu[a]), mb = std::abs(mu[b]);
    if (ma != mb) return ma > mb;
    return mu[a].imag() > mu[b].imag();
  });
  auto is_conj = [&](int a, int b) {
    const double sc = std::max(std::abs(mu[a]), 1e-300);
    return std::abs(mu[a] - std::conj(mu[b])) <= 1e-10 * sc && mu[a].imag() != 0;
  };
  int kk0 = std::min(k, ng);
  // tie at the cut (not a conjugate pair)
  if (kk0 < ng && std::abs(mu[order[kk0]]) > 0) {
    const int a = order[kk0 - 1], b = order[kk0];
    if (!is_conj(a, b) && std::abs(mu[a]) / std::abs(mu[b]) - 1.0 < 1e-8) ties = 1;
  }
  // keep conjugate pairs together
  std::vector<int> sel(order.begin(), order.begin() + kk0);
  std::vector<int> keep;
  for (int i : sel) {
    if (mu[i].imag() != 0) {
      bool partner = false;
      for (int j : sel)
        if (j != i && is_conj(i, j)) partner = true;
      if (!partner) continue;
    }
    keep.push_back(i);
  }
  // eigenvectors (one per conjugate pair), real basis of the span
  std::vector<double> cols;
  std::vector<cplx> found;  // previous vectors of nearly equal eigenvalues
  int nfound = 0;
  std::vector<cplx> start(ng), w;
  std::vector<int> done(ng, 0);
  std::vector<cplx> all_vecs;
  std::vector<cplx> all_mu;
  for (size_t q = 0; q < keep.size(); ++q) {
    const int i = keep[q];
    if (done[i]) continue;
    if (mu[i].imag() < 0) {
      // handled by its partner with positive imaginary part
      bool has_partner = false;
      for (int j : keep)
        if (!done[j] && is_conj(j, i) && mu[j].imag() > 0) has_partner = true;
      if (has_partner) continue;
    }
    // cluster of previously computed vectors with nearly the same eigenvalue
    found.clear();
    nfound = 0;
    for (size_t a = 0; a < all_mu.size(); ++a)
      if (std::abs(all_mu[a] - mu[i]) <= 1e-8 * std::max(std::abs(mu[i]), 1e-300)) {
        found.insert(found.end(), all_vecs.begin() + a * ng, all_vecs.begin() + (a + 1) * ng);
        ++nfound;
      }
    for (int r = 0; r < ng; ++r)
      start[r] = cplx(1.0 + 0.37 * std::sin(1.3 * r + 0.7 * nfound),
                      mu[i].imag() != 0 ? 0.21 * std::cos(0.9 * r) : 0.0);
    eigenvector(ng, S.data(), mu[i], start, found, nfound, w);
    all_mu.push_back(mu[i]);
    all_vecs.insert(all_vecs.end(), w.begin(), w.end());
    // z = RG^-1 w
    std::vector<cplx> z(ng, 0.0);
    for (int r = 0; r < ng; ++r) {
      cplx s = 0;
      for (int c = r; c < ng; ++c) s += RGi[r + (size_t)ng * c] * w[c];
      z[r] = s;
    }
    for (int r = 0; r < ng; ++r) cols.push_back(z[r].real());
    if (mu[i].imag() != 0) {
      for (int r = 0; r < ng; ++r) cols.push_back(z[r].imag());
      for (int j : keep)
        if (j != i && is_conj(i, j)) done[j] = 1;
    }
    done[i] = 1;
  }
  kk = (int)(cols.size() / ng);
  P.swap(cols);
  return kk > 0;
}

}  // namespace dense
}  // namespace krs
