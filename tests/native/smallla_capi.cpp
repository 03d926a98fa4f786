// C wrappers around the library's host dense linear algebra, built by the
// CPU test-suite with g++ (no GPU, no HIP) to check it against LAPACK.
#include <complex>
#include <cstring>
#include <vector>

#include "../../paper_1903_06986_amd/csrc/smallla.h"

using namespace lqcd::la;

static Mat load(int r, int c, const double *a) {
  Mat M(r, c);
  std::memcpy(M.a.data(), a, sizeof(cd) * r * c);
  return M;
}

extern "C" int la_eig(int n, const double *A, double *w, double *V) {
  std::vector<cd> ww;
  Mat Vr;
  if (!eig(load(n, n, A), ww, Vr)) return 1;
  std::memcpy(w, ww.data(), sizeof(cd) * n);
  std::memcpy(V, Vr.a.data(), sizeof(cd) * n * n);
  return 0;
}

extern "C" void la_eigh(int n, const double *A, double *w, double *V) {
  std::vector<double> ww;
  Mat Vr;
  eigh(load(n, n, A), ww, Vr);
  std::memcpy(w, ww.data(), sizeof(double) * n);
  std::memcpy(V, Vr.a.data(), sizeof(cd) * n * n);
}

extern "C" void la_lstsq(int r, int c, const double *A, const double *b, double *x) {
  std::vector<cd> bb(r);
  std::memcpy(bb.data(), b, sizeof(cd) * r);
  auto xx = lstsq(load(r, c, A), bb);
  std::memcpy(x, xx.data(), sizeof(cd) * c);
}

extern "C" void la_solve(int n, const double *A, const double *b, double *x) {
  std::vector<cd> bb(n);
  std::memcpy(bb.data(), b, sizeof(cd) * n);
  auto xx = solve(load(n, n, A), bb);
  std::memcpy(x, xx.data(), sizeof(cd) * n);
}

extern "C" void la_thin_q(int r, int c, const double *A, double *Q) {
  QR f;
  f.factor(load(r, c, A));
  Mat q = f.thin_q();
  std::memcpy(Q, q.a.data(), sizeof(cd) * r * c);
}

extern "C" int la_cholesky_inv(int n, const double *A, double *Li) {
  Mat L;
  if (!cholesky_inv(load(n, n, A), L)) return 1;
  std::memcpy(Li, L.a.data(), sizeof(cd) * n * n);
  return 0;
}
