// Test driver for the host dense linear algebra (paper_1501_03358_amd/csrc/
// dense.cpp): reads cases from stdin, writes results to stdout, one line per
// case; tests/test_host_dense.py builds it with the address and undefined-
// behaviour sanitizers and checks the results against NumPy/SciPy.
//
// Input cases (values in full precision, column-major):
//   qr m n <A>            -> "qr" Q (m*n) R (n*n)
//   chol n <A>            -> "chol ok|fail" R (n*n)
//   uinv n <R>            -> "uinv ok|fail" Rinv (n*n)
//   usolve n <R> <g>      -> "usolve" y (n)
//   symeig n <A>          -> "symeig ok|fail" w (n) Z (n*n)
//   eig n <A>             -> "eig ok|fail" (re im) x n
//   hr mg ng k <G> <F>    -> "hr ok|fail kk ties" P (ng*kk)
#include <cstdio>
#include <iostream>
#include <string>
#include <vector>

#include "../paper_1501_03358_amd/csrc/dense.hpp"

using namespace krs::dense;

static std::vector<double> read_vals(size_t n) {
  std::vector<double> v(n);
  for (size_t i = 0; i < n; ++i) std::cin >> v[i];
  return v;
}

static void put(const char* tag, const std::vector<double>& a) {
  std::printf("%s", tag);
  for (double x : a) std::printf(" %.17g", x);
}

int main() {
  std::string kind;
  while (std::cin >> kind) {
    if (kind == "qr") {
      int m, n;
      std::cin >> m >> n;
      auto A = read_vals((size_t)m * n);
      std::vector<double> Q((size_t)m * n), R((size_t)n * n);
      qr_thin(m, n, A.data(), Q.data(), R.data());
      put("qr", Q);
      put("", R);
    } else if (kind == "chol") {
      int n;
      std::cin >> n;
      auto A = read_vals((size_t)n * n);
      std::vector<double> R((size_t)n * n, 0.0);
      const bool ok = cholesky_upper(n, A.data(), R.data());
      put(ok ? "chol ok" : "chol fail", R);
    } else if (kind == "uinv") {
      int n;
      std::cin >> n;
      auto R = read_vals((size_t)n * n);
      std::vector<double> Ri((size_t)n * n, 0.0);
      const bool ok = upper_inverse(n, R.data(), Ri.data());
      put(ok ? "uinv ok" : "uinv fail", Ri);
    } else if (kind == "usolve") {
      int n;
      std::cin >> n;
      auto R = read_vals((size_t)n * n);
      auto g = read_vals(n);
      std::vector<double> y(n, 0.0);
      upper_solve(n, R.data(), n, g.data(), y.data());
      put("usolve", y);
    } else if (kind == "symeig") {
      int n;
      std::cin >> n;
      auto A = read_vals((size_t)n * n);
      std::vector<double> w, Z;
      const bool ok = sym_eig(n, A.data(), w, Z);
      put(ok ? "symeig ok" : "symeig fail", w);
      put("", Z);
    } else if (kind == "eig") {
      int n;
      std::cin >> n;
      auto A = read_vals((size_t)n * n);
      std::vector<cplx> lam;
      const bool ok = eigenvalues(n, A.data(), lam);
      std::vector<double> out;
      for (const cplx& l : lam) {
        out.push_back(l.real());
        out.push_back(l.imag());
      }
      put(ok ? "eig ok" : "eig fail", out);
    } else if (kind == "hr") {
      int mg, ng, k;
      std::cin >> mg >> ng >> k;
      auto G = read_vals((size_t)mg * ng);
      auto F = read_vals((size_t)mg * ng);
      std::vector<double> P;
      int kk = 0, ties = 0;
      const bool ok = harmonic_ritz_select(mg, ng, G.data(), F.data(), k, P, kk, ties);
      std::printf("%s %d %d", ok ? "hr ok" : "hr fail", kk, ties);
      put("", P);
    } else {
      std::fprintf(stderr, "unknown case %s\n", kind.c_str());
      return 2;
    }
    std::printf("\n");
  }
  return 0;
}
