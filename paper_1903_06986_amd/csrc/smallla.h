// Small dense complex linear algebra on the host (m <= a few hundred):
// the Hessenberg least-squares problems, harmonic Ritz eigenproblems and
// Rayleigh-Ritz steps of the restarted Krylov solvers.  Matrices are
// column-major with an explicit leading dimension.
#pragma once

#include <complex>
#include <vector>

namespace lqcd {
namespace la {

using cd = std::complex<double>;

// Column-major dense matrix.
struct Mat {
  int rows = 0, cols = 0;
  std::vector<cd> a;
  Mat() = default;
  Mat(int r, int c) : rows(r), cols(c), a(size_t(r) * c, cd(0, 0)) {}
  cd &operator()(int i, int j) { return a[size_t(j) * rows + i]; }
  const cd &operator()(int i, int j) const { return a[size_t(j) * rows + i]; }
  cd *col(int j) { return a.data() + size_t(j) * rows; }
  const cd *col(int j) const { return a.data() + size_t(j) * rows; }
};

Mat matmul(const Mat &A, const Mat &B);        // A B
Mat matmul_hn(const Mat &A, const Mat &B);     // A^H B
Mat adjoint(const Mat &A);

// Householder QR of A (rows >= cols): keeps the reflectors so that Q^H b
// and the triangular solve can be applied to many right-hand sides.
struct QR {
  int rows = 0, cols = 0;
  Mat qr;                  // R in the upper triangle, reflectors below
  std::vector<cd> tau;
  std::vector<double> beta;
  void factor(const Mat &A);
  void apply_qh(cd *b) const;           // b <- Q^H b (length rows)
  void solve_r(cd *x) const;            // x <- R^{-1} x (first cols entries)
  Mat thin_q() const;                   // rows x cols orthonormal Q
};

// x = argmin |b - A x| (A rows x cols, rows >= cols, full column rank).
std::vector<cd> lstsq(const Mat &A, const std::vector<cd> &b);

// Solve A x = b (square) by LU with partial pivoting.
std::vector<cd> solve(Mat A, std::vector<cd> b);

// Eigenvalues w and unit-norm right eigenvectors (columns of Vr) of a
// general square matrix: Householder reduction to Hessenberg form, then the
// complex shifted QR iteration (Wilkinson shifts, Givens rotations) to the
// Schur form A = Z T Z^H, then back-substitution in T.  Returns false if
// the iteration does not converge.
bool eig(const Mat &A, std::vector<cd> &w, Mat &Vr);

// Hermitian eigenproblem by cyclic complex Jacobi rotations: eigenvalues
// ascending, orthonormal eigenvectors in the columns of Vr.
void eigh(const Mat &A, std::vector<double> &w, Mat &Vr);

// Li = L^{-1} for the Cholesky factor L L^H = A of a hermitian positive
// definite A (lower triangular); false if A is not positive definite.
bool cholesky_inv(const Mat &A, Mat &Li);

}  // namespace la
}  // namespace lqcd
