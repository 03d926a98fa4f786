// Host dense linear algebra for the small projected problems of the
// Krylov solvers (see smallla.h).  Plain textbook algorithms in FP64:
// Householder QR, LU with partial pivoting, Hessenberg reduction + complex
// shifted QR (Schur form) for general eigenproblems, cyclic Jacobi for
// hermitian ones.
#include "smallla.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace lqcd {
namespace la {

namespace {
constexpr double kEps = std::numeric_limits<double>::epsilon();

// Householder vector v (length n, v[0] arbitrary) and beta with
// (I - beta v v^H) x = alpha e_1, alpha = -phase(x0) |x|.
double house(const cd *x, int n, cd *v, cd &alpha) {
  double nrm2 = 0;
  for (int i = 0; i < n; ++i) nrm2 += std::norm(x[i]);
  double nrm = std::sqrt(nrm2);
  for (int i = 0; i < n; ++i) v[i] = x[i];
  if (nrm == 0.0) {
    alpha = 0;
    return 0.0;
  }
  cd ph = std::abs(x[0]) > 0 ? x[0] / std::abs(x[0]) : cd(1, 0);
  alpha = -ph * nrm;
  v[0] = x[0] - alpha;
  double vv = nrm2 - std::norm(x[0]) + std::norm(v[0]);
  return vv > 0 ? 2.0 / vv : 0.0;
}
}  // namespace

Mat matmul(const Mat &A, const Mat &B) {
  Mat C(A.rows, B.cols);
  for (int j = 0; j < B.cols; ++j)
    for (int l = 0; l < A.cols; ++l) {
      cd b = B(l, j);
      if (b == cd(0, 0)) continue;
      for (int i = 0; i < A.rows; ++i) C(i, j) += A(i, l) * b;
    }
  return C;
}

Mat matmul_hn(const Mat &A, const Mat &B) {
  Mat C(A.cols, B.cols);
  for (int j = 0; j < B.cols; ++j)
    for (int i = 0; i < A.cols; ++i) {
      cd s = 0;
      for (int l = 0; l < A.rows; ++l) s += std::conj(A(l, i)) * B(l, j);
      C(i, j) = s;
    }
  return C;
}

Mat adjoint(const Mat &A) {
  Mat C(A.cols, A.rows);
  for (int j = 0; j < A.cols; ++j)
    for (int i = 0; i < A.rows; ++i) C(j, i) = std::conj(A(i, j));
  return C;
}

void QR::factor(const Mat &A) {
  rows = A.rows;
  cols = A.cols;
  qr = A;
  tau.assign(cols, cd(0, 0));  // R diagonal (alpha) per column
  beta.assign(cols, 0.0);
  std::vector<cd> v(rows);
  for (int k = 0; k < cols; ++k) {
    int n = rows - k;
    cd alpha;
    double b = house(qr.col(k) + k, n, v.data(), alpha);
    beta[k] = b;
    // apply to the remaining columns
    for (int j = k + 1; j < cols; ++j) {
      cd *cj = qr.col(j) + k;
      cd s = 0;
      for (int i = 0; i < n; ++i) s += std::conj(v[i]) * cj[i];
      s *= b;
      for (int i = 0; i < n; ++i) cj[i] -= s * v[i];
    }
    // store v below the diagonal (v[0] kept in place of R_kk, R_kk in tau)
    cd *ck = qr.col(k) + k;
    for (int i = 0; i < n; ++i) ck[i] = v[i];
    tau[k] = alpha;
  }
}

void QR::apply_qh(cd *b) const {
  for (int k = 0; k < cols; ++k) {
    const cd *v = qr.col(k) + k;
    int n = rows - k;
    cd s = 0;
    for (int i = 0; i < n; ++i) s += std::conj(v[i]) * b[k + i];
    s *= beta[k];
    for (int i = 0; i < n; ++i) b[k + i] -= s * v[i];
  }
}

void QR::solve_r(cd *x) const {
  for (int i = cols - 1; i >= 0; --i) {
    cd s = x[i];
    for (int j = i + 1; j < cols; ++j) s -= qr(i, j) * x[j];
    x[i] = s / tau[i];
  }
}

Mat QR::thin_q() const {
  Mat Q(rows, cols);
  for (int j = 0; j < cols; ++j) Q(j, j) = 1.0;
  for (int k = cols - 1; k >= 0; --k) {
    const cd *v = qr.col(k) + k;
    int n = rows - k;
    for (int j = 0; j < cols; ++j) {
      cd *qj = Q.col(j) + k;
      cd s = 0;
      for (int i = 0; i < n; ++i) s += std::conj(v[i]) * qj[i];
      s *= beta[k];
      for (int i = 0; i < n; ++i) qj[i] -= s * v[i];
    }
  }
  return Q;
}

std::vector<cd> lstsq(const Mat &A, const std::vector<cd> &b) {
  QR f;
  f.factor(A);
  std::vector<cd> y(b);
  f.apply_qh(y.data());
  f.solve_r(y.data());
  y.resize(A.cols);
  return y;
}

std::vector<cd> solve(Mat A, std::vector<cd> b) {
  const int n = A.rows;
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(A(k, k));
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A(i, k)) > best) {
        best = std::abs(A(i, k));
        p = i;
      }
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A(k, j), A(p, j));
      std::swap(b[k], b[p]);
    }
    cd piv = A(k, k);
    if (piv == cd(0, 0)) piv = cd(kEps, 0);
    for (int i = k + 1; i < n; ++i) {
      cd f = A(i, k) / piv;
      if (f == cd(0, 0)) continue;
      for (int j = k; j < n; ++j) A(i, j) -= f * A(k, j);
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    cd s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A(i, j) * b[j];
    cd piv = A(i, i);
    if (piv == cd(0, 0)) piv = cd(kEps, 0);
    b[i] = s / piv;
  }
  return b;
}

bool eig(const Mat &A0, std::vector<cd> &w, Mat &Vr) {
  const int n = A0.rows;
  Mat H = A0;
  Mat Z(n, n);
  for (int i = 0; i < n; ++i) Z(i, i) = 1.0;
  // 1. Hessenberg reduction H = Q^H A Q, Z = Q.
  std::vector<cd> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    int m = n - k - 1;
    cd alpha;
    double b = house(H.col(k) + k + 1, m, v.data(), alpha);
    if (b == 0.0) continue;
    // rows k+1.. : H <- (I - b v v^H) H
    for (int j = 0; j < n; ++j) {
      cd s = 0;
      for (int i = 0; i < m; ++i) s += std::conj(v[i]) * H(k + 1 + i, j);
      s *= b;
      for (int i = 0; i < m; ++i) H(k + 1 + i, j) -= s * v[i];
    }
    // columns k+1.. : H <- H (I - b v v^H), Z likewise
    for (Mat *M : {&H, &Z})
      for (int i = 0; i < n; ++i) {
        cd s = 0;
        for (int l = 0; l < m; ++l) s += (*M)(i, k + 1 + l) * v[l];
        s *= b;
        for (int l = 0; l < m; ++l) (*M)(i, k + 1 + l) -= s * std::conj(v[l]);
      }
    for (int i = k + 2; i < n; ++i) H(i, k) = 0;
  }
  // 2. Shifted QR iteration to Schur form (Givens rotations on the whole
  //    matrix so that T and Z stay complete for the eigenvectors).
  int hi = n - 1;
  int iter = 0, total = 0;
  const int max_total = 60 * std::max(n, 1);
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      double s = std::abs(H(l - 1, l - 1)) + std::abs(H(l, l));
      if (s == 0.0) s = 1.0;
      if (std::abs(H(l, l - 1)) <= kEps * s) {
        H(l, l - 1) = 0;
        break;
      }
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > max_total) return false;
    ++iter;
    // Wilkinson shift from the trailing 2x2 block of the active window
    cd a = H(hi - 1, hi - 1), bb = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
    cd mu;
    if (iter % 11 == 10) {
      mu = d + cd(std::abs(H(hi, hi - 1)), 0);  // exceptional shift
    } else {
      cd tr2 = 0.5 * (a + d);
      cd disc = std::sqrt((a - tr2) * (a - tr2) + bb * c);
      cd m1 = tr2 + disc, m2 = tr2 - disc;
      mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    }
    cd x = H(l, l) - mu, y = H(l + 1, l);
    for (int k = l; k < hi; ++k) {
      if (k > l) {
        x = H(k, k - 1);
        y = H(k + 1, k - 1);
      }
      double ax = std::abs(x), ay = std::abs(y);
      double nr = std::hypot(ax, ay);
      if (nr == 0.0) continue;
      double cc;
      cd ss;
      if (ax == 0.0) {
        cc = 0.0;
        ss = std::conj(y) / ay;
      } else {
        cc = ax / nr;
        ss = (x / ax) * std::conj(y) / nr;
      }
      // rows k, k+1 (columns k-1 .. n-1)
      for (int j = std::max(k - 1, 0); j < n; ++j) {
        cd h1 = H(k, j), h2 = H(k + 1, j);
        H(k, j) = cc * h1 + ss * h2;
        H(k + 1, j) = -std::conj(ss) * h1 + cc * h2;
      }
      if (k > l) H(k + 1, k - 1) = 0;
      // columns k, k+1 (rows 0 .. min(k+2, hi))
      int rmax = std::min(k + 2, hi);
      for (int i = 0; i <= rmax; ++i) {
        cd h1 = H(i, k), h2 = H(i, k + 1);
        H(i, k) = cc * h1 + std::conj(ss) * h2;
        H(i, k + 1) = -ss * h1 + cc * h2;
      }
      for (int i = 0; i < n; ++i) {
        cd z1 = Z(i, k), z2 = Z(i, k + 1);
        Z(i, k) = cc * z1 + std::conj(ss) * z2;
        Z(i, k + 1) = -ss * z1 + cc * z2;
      }
    }
  }
  // 3. Eigenvalues and eigenvectors of the triangular T, mapped back by Z.
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = H(i, i);
  double tnorm = 0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) tnorm = std::max(tnorm, std::abs(H(i, j)));
  const double small = kEps * std::max(tnorm, 1e-300);
  Vr = Mat(n, n);
  std::vector<cd> y(n);
  for (int k = 0; k < n; ++k) {
    std::fill(y.begin(), y.end(), cd(0, 0));
    y[k] = 1.0;
    for (int j = k - 1; j >= 0; --j) {
      cd s = 0;
      for (int l = j + 1; l <= k; ++l) s += H(j, l) * y[l];
      cd den = H(j, j) - H(k, k);
      if (std::abs(den) < small) den = cd(small, 0);
      y[j] = -s / den;
    }
    double nrm = 0;
    for (int i = 0; i < n; ++i) {
      cd s = 0;
      for (int l = 0; l <= k; ++l) s += Z(i, l) * y[l];
      Vr(i, k) = s;
      nrm += std::norm(s);
    }
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i) Vr(i, k) /= nrm;
  }
  return true;
}

void eigh(const Mat &A0, std::vector<double> &w, Mat &Vr) {
  const int n = A0.rows;
  Mat A = A0;
  // hermitise
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) {
      cd h = 0.5 * (A(i, j) + std::conj(A(j, i)));
      A(i, j) = h;
      A(j, i) = std::conj(h);
    }
  Vr = Mat(n, n);
  for (int i = 0; i < n; ++i) Vr(i, i) = 1.0;
  double fro = 0;
  for (auto &x : A.a) fro += std::norm(x);
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < j; ++i) off += std::norm(A(i, j));
    if (std::sqrt(2 * off) <= 1e-16 * fro) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = std::abs(A(p, q));
        if (apq <= 1e-300) continue;
        cd ph = A(p, q) / apq;  // e^{i phi}
        double app = A(p, p).real(), aqq = A(q, q).real();
        double tau = (aqq - app) / (2 * apq);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1 + tau * tau));
        double c = 1 / std::sqrt(1 + t * t), s = t * c;
        // J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on columns p, q
        cd em = std::conj(ph);
        for (int i = 0; i < n; ++i) {
          cd ap = A(i, p), aq = A(i, q);
          A(i, p) = c * ap - s * em * aq;
          A(i, q) = s * ap + c * em * aq;
        }
        for (int j = 0; j < n; ++j) {
          cd ap = A(p, j), aq = A(q, j);
          A(p, j) = c * ap - s * ph * aq;
          A(q, j) = s * ap + c * ph * aq;
        }
        A(p, q) = 0;
        A(q, p) = 0;
        for (int i = 0; i < n; ++i) {
          cd vp = Vr(i, p), vq = Vr(i, q);
          Vr(i, p) = c * vp - s * em * vq;
          Vr(i, q) = s * vp + c * em * vq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return A(a, a).real() < A(b, b).real(); });
  Mat V2(n, n);
  w.resize(n);
  for (int k = 0; k < n; ++k) {
    w[k] = A(idx[k], idx[k]).real();
    for (int i = 0; i < n; ++i) V2(i, k) = Vr(i, idx[k]);
  }
  Vr = V2;
}

bool cholesky_inv(const Mat &A, Mat &Li) {
  const int n = A.rows;
  Mat L(n, n);
  for (int j = 0; j < n; ++j) {
    double d = A(j, j).real();
    for (int k = 0; k < j; ++k) d -= std::norm(L(j, k));
    if (!(d > 0) || !std::isfinite(d)) return false;
    const double ljj = std::sqrt(d);
    L(j, j) = ljj;
    for (int i = j + 1; i < n; ++i) {
      cd v = A(i, j);
      for (int k = 0; k < j; ++k) v -= L(i, k) * std::conj(L(j, k));
      L(i, j) = v / ljj;
    }
  }
  // forward substitution on the identity: L Li = I
  Li = Mat(n, n);
  for (int c = 0; c < n; ++c)
    for (int i = c; i < n; ++i) {
      cd v = i == c ? cd(1, 0) : cd(0, 0);
      for (int k = c; k < i; ++k) v -= L(i, k) * Li(k, c);
      Li(i, c) = v / L(i, i);
    }
  return true;
}

}  // namespace la
}  // namespace lqcd
