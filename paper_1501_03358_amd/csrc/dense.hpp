// Small dense FP64 linear algebra on the host (column-major), used by the
// cycle-end steps of the Krylov solvers: least squares by Givens rotations,
// thin QR, Cholesky, and the harmonic-Ritz eigenproblem of the recycle-space
// update.  Sizes are at most a few dozen.
#pragma once
#include <complex>
#include <vector>

namespace krs {
namespace dense {

using cplx = std::complex<double>;

// Thin Householder QR of the m x n matrix A (lda = m), m >= n:
// A = Q R with Q m x n orthonormal columns, R n x n upper, diag(R) >= 0.
void qr_thin(int m, int n, const double* A, double* Q, double* R);

// Cholesky A = R^T R (A n x n SPD, upper factor R).  Returns false if not SPD.
bool cholesky_upper(int n, const double* A, double* R);

// Inverse of an n x n upper triangular matrix. Returns false on a zero pivot.
bool upper_inverse(int n, const double* R, double* Rinv);

// Solve R y = g (n x n upper triangular, ldr).
void upper_solve(int n, const double* R, int ldr, const double* g, double* y);

// Eigenvalues of a real n x n matrix (Householder Hessenberg reduction and
// the implicit double-shift QR iteration).  Returns false if it does not
// converge.
bool eigenvalues(int n, const double* A, std::vector<cplx>& lam);

// Eigenvector of A for the (computed) eigenvalue mu by inverse iteration in
// complex arithmetic, started from `start` (length n); orthogonalised against
// the columns of `against` (n x na, complex) before each solve.
void eigenvector(int n, const double* A, cplx mu, const std::vector<cplx>& start,
                 const std::vector<cplx>& against, int na, std::vector<cplx>& v);

// Eigen-decomposition of a symmetric n x n matrix by the cyclic Jacobi
// method: eigenvalues w descending, eigenvectors the columns of Z (n x n).
// Returns false if the sweeps do not converge.
bool sym_eig(int n, const double* A, std::vector<double>& w, std::vector<double>& Z);

// Harmonic-Ritz selection for the recycle-space update.
//   G: mg x ng (= ng+1 rows), F: mg x ng, both column-major.
// Solves G^T G z = theta G^T F z, keeps the k pairs of smallest |theta|
// without splitting a complex-conjugate pair, and returns a real basis P
// (ng x kk, column-major) of the span of the kept z.  ties counts a near tie
// at the cut.  Returns false on failure of the eigen-solver.
bool harmonic_ritz_select(int mg, int ng, const double* G, const double* F, int k,
                          std::vector<double>& P, int& kk, int& ties);

}  // namespace dense
}  // namespace krs
