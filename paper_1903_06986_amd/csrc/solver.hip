// Deflated restarted GMRES on the GPU (Sec. 7: GMRES-DR(m,k) for the first
// noise vector, super-converged, then GMRES-Proj for the rest; Sec. 5.4 for
// the hermitian M').  The algorithms are the cited ones (Morgan's GMRES-DR,
// Morgan and Wilcox's GMRES-Proj); the paper does not print them.
//
// Device work: operator applications (the stencil), classical Gram-Schmidt
// applied twice with FP64 accumulation, norms, basis updates and the
// deflation projections.  Host work: the (m+1) x m least-squares problems,
// the m x m harmonic Ritz eigenproblem and the restart matrix P_{k+1},
// once per cycle.  Within a cycle nothing waits for the host.
//
// GMRES-DR restart (per cycle): d = argmin |c - Hbar d|, x += V_m d; the k
// harmonic Ritz vectors g of smallest |theta| ((H_m + |h|^2 f e_m^T) g =
// theta g, H_m^H f = e_m) and the residual direction w = [-|h|^2 f; h]
// (parallel to c - Hbar d, but free of its cancellation) are
// orthonormalised into P_{k+1}; then V_{k+1} = V_{m+1} P_{k+1},
// Hbar_k = P_{k+1}^H Hbar_m P_k, c = P_{k+1}^H (c - Hbar d).
//
// GMRES-Proj (batched over right-hand sides): repeat { projection
// c = V_{k+1}^H r, d = argmin |c - Hbar_k d|, x += V_k d, r -= V_{k+1}
// Hbar_k d; one GMRES(m-k) cycle; true residual r = b - A x }.
//
// Mixed precision (inner = F32): FP64 iterative refinement; each refinement
// step solves A e = r with the FP32 stencil and an FP32 Krylov basis
// (Gram-Schmidt coefficients and norms still accumulated in FP64) to a
// relative tolerance inner_tol, then x += e and r = b - A x in FP64.
#include <algorithm>
#include <cmath>
#include <memory>

#include "cplx.h"
#include "fields.h"
#include "half.h"
#include "solver.h"

namespace lqcd {

namespace {

// ------------------------------------------------------------- kernels
// Reorthogonalisation test after the first Gram-Schmidt pass (Daniel,
// Gragg, Kaufman and Stewart): with |w|^2 = |w'|^2 + |h|^2 (w' orthogonal to
// the basis), a second pass runs when |w'|^2 < eta2 |w|^2.  eta2 > 1 makes
// it unconditional.
__global__ void k_dgks(const cx<double> *__restrict__ h1, size_t hrs, int J,
                       const double *__restrict__ nrm1, int *__restrict__ flag,
                       int *__restrict__ reorth_count, double eta2) {
  const int r = blockIdx.x;
  if (threadIdx.x != 0) return;
  double hh = 0;
  for (int i = 0; i < J; ++i) {
    cx<double> v = h1[r * hrs + i];
    hh += v.re * v.re + v.im * v.im;
  }
  const int need = nrm1[r] < eta2 * (nrm1[r] + hh) ? 1 : 0;
  flag[r] = need;
  if (need) reorth_count[r] += 1;
}

__global__ void k_count1(int *__restrict__ count) { count[0] += 1; }

// Selective reorthogonalisation against the kept vectors (MINRES-DR): the
// update with their second-pass coefficients runs only if one of them
// exceeds tau |w| (tau2 = tau^2, nrm1 = |w|^2 after the first pass);
// otherwise they are set to zero, so that the Hessenberg column matches the
// vector.  Counts the updates that run, and raises the second-pass flag
// when one does.
__global__ void k_kept_test(cx<double> *__restrict__ h2, int kept, const double *__restrict__ nrm1, double tau2,
                            int *__restrict__ kflag, int *__restrict__ flag, int *__restrict__ count) {
  if (threadIdx.x != 0) return;
  double mx = 0;
  for (int i = 0; i < kept; ++i) mx = fmax(mx, h2[i].re * h2[i].re + h2[i].im * h2[i].im);
  const int need = mx > tau2 * nrm1[0] ? 1 : 0;
  kflag[0] = need;
  if (need) {
    count[0] += 1;
    flag[0] = 1;  // the second pass (and |w| after it) is then needed
  } else {
    for (int i = 0; i < kept; ++i) h2[i] = mk(0.0, 0.0);
  }
}

// Column j of Hbar: h1 (+ h2 when the second pass ran); h_{j+1,j} = |w|.
__global__ void k_finish_col(cx<double> *__restrict__ Hd, size_t Hrs, int ldh, int j,
                             const cx<double> *__restrict__ h1, const cx<double> *__restrict__ h2,
                             size_t hrs, const double *__restrict__ nrm1,
                             const double *__restrict__ nrm2, const int *__restrict__ flag,
                             double *__restrict__ inv) {
  const int r = blockIdx.x;
  const bool two = flag[r] != 0;
  cx<double> *col = Hd + r * Hrs + size_t(j) * ldh;
  for (int i = threadIdx.x; i <= j; i += blockDim.x)
    col[i] = two ? h1[r * hrs + i] + h2[r * hrs + i] : h1[r * hrs + i];
  if (threadIdx.x == 0) {
    double nr = sqrt(two ? nrm2[r] : nrm1[r]);
    col[j + 1] = mk(nr, 0.0);
    inv[r] = (nr > 0 && isfinite(nr)) ? 1.0 / nr : 0.0;
  }
}

// Cholesky factor G = R^H R of the S x S Gram matrix g (layout of
// gram_pair_idx; G[l][m] = y_l^H y_m), column by column, stopping at the
// first pivot that is not above pmin times its diagonal entry (pmin = 0:
// not positive) or is not finite.  Returns the number t of pivots taken;
// R holds the columns before t and R[l][t], l < t (zero elsewhere).
template <int S>
__device__ inline int chol_gram(const double *g, cx<double> (&R)[S][S], double pmin) {
#pragma unroll
  for (int m = 0; m < S; ++m)
#pragma unroll
    for (int l = 0; l < S; ++l) R[l][m] = mk(0.0, 0.0);
  for (int m = 0; m < S; ++m) {
    for (int l = 0; l < m; ++l) {
      const int q = gram_pair_idx(S, l, m);
      cx<double> a = mk(g[q], g[q + 1]);
      for (int p = 0; p < l; ++p) a = a - cmulc(R[p][l], R[p][m]);
      R[l][m] = (1.0 / R[l][l].re) * a;
    }
    double d = g[m];
    for (int p = 0; p < m; ++p) d -= R[p][m].re * R[p][m].re + R[p][m].im * R[p][m].im;
    if (!(d > pmin * g[m]) || !(d > 0) || !isfinite(d)) return m;
    R[m][m] = mk(sqrt(d), 0.0);
  }
  return S;
}

// Sums the S^2 Gram partials of one right-hand side over nblk workgroups
// (one 64-lane block; every lane ends with the totals).
template <int S>
__device__ inline void gram_total(const double *__restrict__ part, int r, int nblk, double (&g)[S * S]) {
  constexpr int NG = S * S;
#pragma unroll
  for (int q = 0; q < NG; ++q) g[q] = 0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int q = 0; q < NG; ++q) g[q] += part[(size_t(r) * nblk + b) * NG + q];
#pragma unroll
  for (int q = 0; q < NG; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) g[q] += __shfl_xor(g[q], off, 64);
}

constexpr int kSstepMaxJ = 256;  // basis vectors before a block (J <= m + 1 <= 251)
// A block stores its basis vectors straight from the update pass only if
// every Cholesky pivot of its Gram matrix (from the dot pass) keeps this
// fraction of its diagonal entry: the difference Z^H Z - C^H C then loses
// at most three digits to cancellation, well inside the 16-bit storage
// rounding.
constexpr double kPivotMin = 1e-3;

// s-step Arnoldi (16-bit basis), after the first dot pass: the Gram matrix
// of the projected block Y = Z - V C follows from it as Z^H Z - C^H C (V
// orthonormal; gpart holds the partials of Z^H Z).  The block takes the
// direct path (flag clear; G[r] receives this Gram matrix, and the update
// pass stores the orthonormalised vectors at once) when the DGKS test
// passes on each vector (|y_k|^2 at least eta2 |z_k|^2) and each Cholesky
// pivot keeps kPivotMin of its diagonal entry; otherwise the explicit path
// (flag set, counted as a second pass): update in place, second block
// pass, Gram matrix of the final vectors.
template <int S>
__global__ void k_sstep_plan(const double *__restrict__ gpart, int nblk, const cx<double> *__restrict__ C, size_t ldc,
                             int J, double *__restrict__ G, int *__restrict__ flag, int *__restrict__ reorth_count,
                             double eta2) {
  constexpr int NG = S * S;
  constexpr int NPR = S * (S + 1) / 2;
  const int r = blockIdx.x;
  double g[NG];
  gram_total<S>(gpart, r, nblk, g);
  // C^H C over the J basis vectors, pairs l <= m in the order of gram_pair_idx
  double cc[2 * NPR];
#pragma unroll
  for (int q = 0; q < 2 * NPR; ++q) cc[q] = 0;
  for (int i = threadIdx.x; i < J; i += blockDim.x) {
    cx<double> cv[S];
#pragma unroll
    for (int l = 0; l < S; ++l) cv[l] = C[r * ldc + size_t(l) * J + i];
    int q = 0;
#pragma unroll
    for (int l = 0; l < S; ++l)
#pragma unroll
      for (int m = l; m < S; ++m, ++q) {
        const cx<double> p = cmulc(cv[l], cv[m]);
        cc[2 * q] += p.re;
        cc[2 * q + 1] += p.im;
      }
  }
#pragma unroll
  for (int q = 0; q < 2 * NPR; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cc[q] += __shfl_xor(cc[q], off, 64);
  if (threadIdx.x != 0) return;
  double gp[NG];
  int need = 0;
  {
    int q = 0;
#pragma unroll
    for (int l = 0; l < S; ++l)
#pragma unroll
      for (int m = l; m < S; ++m, ++q) {
        if (l == m) {
          gp[l] = g[l] - cc[2 * q];
          if (!(gp[l] >= eta2 * g[l])) need = 1;  // DGKS (and not finite)
        } else {
          const int k = gram_pair_idx(S, l, m);
          gp[k] = g[k] - cc[2 * q];
          gp[k + 1] = g[k + 1] - cc[2 * q + 1];
        }
      }
  }
  if (!need) {
    cx<double> R[S][S];
    if (chol_gram<S>(gp, R, kPivotMin) < S) need = 1;
  }
#pragma unroll
  for (int q = 0; q < NG; ++q) G[size_t(r) * NG + q] = gp[q];
  flag[r] = need;
  if (need) reorth_count[r] += 1;
}

// Columns j .. j + S - 1 of Hbar from the block z_k = B^k v_j, k = 1..S,
// B = A - sigma (one 64-lane block per right-hand side).  With the
// projected block Y = Z - V C = Q R (R the Cholesky factor of its Gram
// matrix, Q = [v_{j+1} .. v_{j+S}]), z_k has the coordinates
// zeta_k = (c_k; R[0..k)[k]) in the basis [V, Q], and
//   B v_j     = zeta_1,
//   B v_{j+m} = (zeta_{m+1} - B V c_m - sum_{l<m-1} B v_{j+1+l} R[l][m-1]) / R[m-1][m-1]
// (m = 1..S-1; indices of c, zeta and R from 0 in the code), where
// B V c_m = sum_{i<j} c_m[i] (Hbar[:, i] - sigma e_i) + c_m[j] B v_j.
// Column j + m of Hbar (for A) is B v_{j+m} + sigma e_{j+m}.  Runs for the
// right-hand sides of one path: EXPLICIT clear, those whose flag is clear
// (c = C1, Gram matrix G[r] from k_sstep_plan); EXPLICIT set, those whose
// flag is set (c = C1 + C2, the second pass's coefficients added; Gram
// matrix of the final vectors from the partials part).  f[r] = R^{-1} (S x
// S, upper) turns the block into Q.  Where the Cholesky factor breaks down
// at t < S (a pivot not positive), vectors t.. are zero: their F columns
// vanish, column j + t has a zero subdiagonal entry, later columns are
// zero.  Hbar's earlier columns must be Hessenberg (columns 0 .. j - 1 of
// an Arnoldi process started at column 0).
template <int S, bool EXPLICIT>
__global__ void k_sstep_finish(cx<double> *__restrict__ Hd, size_t Hrs, int ldh, int j,
                               const cx<double> *__restrict__ C1, const cx<double> *__restrict__ C2, size_t ldc,
                               const double *__restrict__ part, int nblk, const double *__restrict__ G,
                               const int *__restrict__ flag, double sigma, cx<double> *__restrict__ f) {
  constexpr int NG = S * S;
  constexpr int LDB = kSstepMaxJ + S + 1;
  __shared__ cx<double> sc[S][kSstepMaxJ];
  __shared__ cx<double> sb[S][LDB];
  __shared__ cx<double> sR[S][S];
  __shared__ int st;
  const int r = blockIdx.x, J = j + 1;
  if ((flag[r] != 0) != EXPLICIT) return;
  for (int i = threadIdx.x; i < J; i += blockDim.x)
#pragma unroll
    for (int k = 0; k < S; ++k) {
      cx<double> a = C1[r * ldc + size_t(k) * J + i];
      if (EXPLICIT) a = a + C2[r * ldc + size_t(k) * J + i];
      sc[k][i] = a;
    }
  for (int i = threadIdx.x; i < LDB; i += blockDim.x)
#pragma unroll
    for (int k = 0; k < S; ++k) sb[k][i] = mk(0.0, 0.0);
  double g[NG];
  if (EXPLICIT) {
    gram_total<S>(part, r, nblk, g);
  } else {
#pragma unroll
    for (int q = 0; q < NG; ++q) g[q] = G[size_t(r) * NG + q];
  }
  if (threadIdx.x == 0) {
    cx<double> R[S][S];
    const int t = chol_gram<S>(g, R, 0.0);
    // column j keeps |y_1| even when it is zero
    if (t == 0 && g[0] >= 0 && isfinite(g[0])) R[0][0] = mk(sqrt(g[0]), 0.0);
    // F = R^{-1} on the leading t x t block, zero elsewhere
    cx<double> F[S][S];
#pragma unroll
    for (int m = 0; m < S; ++m)
#pragma unroll
      for (int l = 0; l < S; ++l) F[l][m] = mk(0.0, 0.0);
    for (int m = 0; m < t; ++m) {
      F[m][m] = mk(1.0 / R[m][m].re, 0.0);
      for (int l = m - 1; l >= 0; --l) {
        cx<double> a = mk(0.0, 0.0);
        for (int p = l + 1; p <= m; ++p) a = a + R[l][p] * F[p][m];
        F[l][m] = (-1.0 / R[l][l].re) * a;
      }
    }
#pragma unroll
    for (int m = 0; m < S; ++m)
#pragma unroll
      for (int l = 0; l < S; ++l) {
        sR[l][m] = R[l][m];
        f[size_t(r) * NG + l * S + m] = F[l][m];
      }
    st = t;
  }
  __syncthreads();
  const int t = st;
  cx<double> *H0 = Hd + r * Hrs;
  for (int m = 0; m < S; ++m) {
    cx<double> *col = H0 + size_t(j + m) * ldh;
    const bool valid = m <= t;
    for (int k = threadIdx.x; k <= J + m; k += blockDim.x) {
      cx<double> b = mk(0.0, 0.0);
      if (m == 0) {
        b = k < J ? sc[0][k] : sR[0][0];
      } else if (valid) {
        const cx<double> *cm = sc[m - 1];
        // zeta_m
        cx<double> z = k < J ? sc[m][k] : (k - J < t ? sR[k - J][m] : mk(0.0, 0.0));
        // B V c_{m-1}: the earlier columns (Hessenberg: row k meets columns
        // k - 1 and later), less sigma on their diagonal, then B v_j
        cx<double> hc = mk(0.0, 0.0);
        for (int i = k > 0 ? k - 1 : 0; i < j; ++i) hc = hc + H0[size_t(i) * ldh + k] * cm[i];
        if (k < j) hc = hc - sigma * cm[k];
        hc = hc + sb[0][k] * cm[j];
        for (int l = 0; l + 1 < m; ++l) hc = hc + sb[l + 1][k] * sR[l][m - 1];
        b = (1.0 / sR[m - 1][m - 1].re) * (z - hc);
      }
      sb[m][k] = b;
      col[k] = (valid && k == j + m) ? b + mk(sigma, 0.0) : b;
    }
    __syncthreads();
  }
}

__global__ void k_izero(int *__restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <class R>
__global__ void k_swap(cx<R> *__restrict__ a, cx<R> *__restrict__ b, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    cx<R> t = a[i];
    a[i] = b[i];
    b[i] = t;
  }
}

// y (FP64) += x (FP32)
__global__ void k_acc_widen(const cx<float> *__restrict__ x, cx<double> *__restrict__ y, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += size_t(gridDim.x) * blockDim.x) {
    cx<float> v = x[i];
    cx<double> w = y[i];
    y[i] = mk(w.re + double(v.re), w.im + double(v.im));
  }
}

template <class R>
void swap_vec(lqcd_ctx *c, void *a, void *b, size_t n) {
  if (a == b) return;
  unsigned nb = unsigned(std::min<size_t>(nblocks(n), 4096));
  hipLaunchKernelGGL(k_swap<R>, dim3(nb), dim3(kBlock), 0, c->stream, static_cast<cx<R> *>(a),
                     static_cast<cx<R> *>(b), n);
  LQCD_HIP(hipGetLastError());
}

void copy_dev(lqcd_ctx *c, void *dst, const void *src, size_t bytes) {
  LQCD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
}

// ------------------------------------------------------------ operators
template <class R>
struct Op {
  lqcd_ctx *c;
  lqcd_op op;
  size_t n;  // vector length
  DevBuf *tmp;
  void apply(const void *in, size_t sin, void *out, size_t sout, int nb) const {
    if (nb <= 0) return;
    if (op == LQCD_OP_SCHUR) {
      const size_t hl = half_len(c->g);
      void *t = tmp->ensure(hl * size_t(nb) * sizeof(cx<R>));
      apply_schur<R>(c, in, out, t, nb, sin, sout, hl);
    } else {
      apply_full<R>(c, LQCD_OP_MG5, in, out, nb, sin, sout);
    }
  }
  // Mhat on 16-bit stored even fields (words, sin apart), FP32 output.
  template <int BK>
  void apply_h(const void *in, size_t sin, void *out, size_t sout, int nb) const {
    if (nb <= 0) return;
    const size_t hl = half_len(c->g);
    void *t = tmp->ensure(hl * size_t(nb) * sizeof(cx<float>));
    apply_schur_h<BK>(c, in, out, t, nb, sin, sout, hl);
  }
  // Mhat - 1 (= -kappa^2 D_eo D_oe) with the output in the FP32 pair
  // layout, on a 16-bit stored input and on an FP32 pair-layout input (the
  // s-step Arnoldi's shifted power basis).
  template <int BK>
  void apply_dd_h(const void *in, size_t sin, void *out, size_t sout, int nb) const {
    if (nb <= 0) return;
    const size_t hl = half_len(c->g);
    void *t = tmp->ensure(hl * size_t(nb) * sizeof(cx<float>));
    apply_dd_h_pair<BK>(c, in, out, t, nb, sin, sout, hl);
  }
  void apply_dd(const void *in, size_t sin, void *out, size_t sout, int nb) const {
    if (nb <= 0) return;
    const size_t hl = half_len(c->g);
    void *t = tmp->ensure(hl * size_t(nb) * sizeof(cx<float>));
    apply_dd_pair(c, in, out, t, nb, sin, sout, hl);
  }
  // the same from a 16-bit stored input to a 16-bit stored output (strides
  // in words)
  template <int BK>
  void apply_dd_hh(const void *in, size_t sin, void *out, size_t sout, int nb) const {
    if (nb <= 0) return;
    const size_t hl = half_len(c->g);
    void *t = tmp->ensure(hl * size_t(nb) * sizeof(cx<float>));
    ::lqcd::apply_dd_hh<BK>(c, in, out, t, nb, sin, sout, hl);
  }
};

// Device scratch for the small per-cycle matrices.
struct Small {
  DevBuf &buf;
  explicit Small(DevBuf &b) : buf(b) {}
  cdouble *Hd, *h1, *h2, *vec, *C, *E;
  double *nrm2, *inv, *nrm1;
  int *flag, *reorth, *kflag, *scratch_count;
  size_t Hrs;
  void setup(int m, int nb, int kmax) {
    Hrs = size_t(m + 1) * m;
    size_t nc = Hrs * nb + 2 * size_t(m + 1) * nb + size_t(m + 1) * nb + 2 * size_t(kmax + 1) * nb +
                size_t(m + 1) * (kmax + 1);
    size_t bytes = nc * sizeof(cdouble) + 3 * size_t(nb) * sizeof(double) + 4 * size_t(nb) * sizeof(int) + 256;
    char *p = static_cast<char *>(buf.ensure(bytes));
    Hd = reinterpret_cast<cdouble *>(p);
    h1 = Hd + Hrs * nb;
    h2 = h1 + size_t(m + 1) * nb;
    vec = h2 + size_t(m + 1) * nb;                 // LS solutions / restart matrix
    C = vec + std::max(size_t(m + 1) * nb, size_t(m + 1) * (kmax + 1));
    E = C + size_t(kmax + 1) * nb;
    nrm2 = reinterpret_cast<double *>(E + size_t(kmax + 1) * nb);
    inv = nrm2 + nb;
    nrm1 = inv + nb;
    flag = reinterpret_cast<int *>(nrm1 + nb);
    reorth = flag + nb;
    kflag = reorth + nb;
    scratch_count = kflag + nb;
  }
};

void h2d(lqcd_ctx *c, void *dst, const void *src, size_t bytes) {
  LQCD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  LQCD_HIP(hipStreamSynchronize(c->stream));
}
void d2h(lqcd_ctx *c, void *dst, const void *src, size_t bytes) {
  LQCD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream));
  LQCD_HIP(hipStreamSynchronize(c->stream));
}

// Arnoldi steps j0 .. m-1 on nb bases (vectors n apart, bases Wrs apart):
// w = A v_j; two classical Gram-Schmidt passes; h_{j+1,j} = |w|;
// v_{j+1} = w / |w|.  Column j of each Hbar goes to the device matrix.
// Second-pass thresholds: in GMRES-DR (whose harmonic Ritz vectors become
// the deflation space) the DGKS test with |w'|^2 < |w|^2 / 2, which keeps
// the basis orthogonal to working precision; in the GMRES(m-k) cycles of
// GMRES-Proj only when the first pass cancelled more than one digit
// (|w'| < 0.1 |w|): there A v_j is mostly its component along v_j, which
// one pass removes accurately.
constexpr double kReorthAlways = 2.0;
constexpr double kReorthDR = 0.5;
constexpr double kReorthCycle = 0.01;
// MINRES-DR: kept-vector updates whose coefficients all lie below this
// fraction of |w| are skipped (they would move w below its rounding level)
constexpr double kKeptTau = 1e-14;

// Inner (FP32) solves of the refinement: at most this many GMRES(m-k)
// cycles per refinement step, and stop when a cycle reduces the residual
// by less than 10%.
constexpr int kInnerCycleCap = 20;
constexpr double kInnerStall = 0.9;
constexpr int kMaxRefinements = 60;

template <class R>
void arnoldi(lqcd_ctx *c, const Op<R> &A, void *W, size_t n, size_t Wrs, int j0, int m, int nb,
             Small &s, double eta2) {
  cx<R> *Wb = static_cast<cx<R> *>(W);
  for (int j = j0; j < m; ++j) {
    cx<R> *wj = Wb + size_t(j) * n, *wn = Wb + size_t(j + 1) * n;
    A.apply(wj, Wrs, wn, Wrs, nb);
    // classical Gram-Schmidt, second pass only where the DGKS test asks for it
    multi_dot<R>(c, Wb, n, Wrs, j + 1, wn, Wrs, n, nb, s.h1, m + 1);
    multi_axpy<R>(c, Wb, n, Wrs, j + 1, s.h1, m + 1, wn, Wrs, n, nb, s.nrm1);
    hipLaunchKernelGGL(k_dgks, dim3(nb), dim3(64), 0, c->stream,
                       reinterpret_cast<const cx<double> *>(s.h1), size_t(m + 1), j + 1, s.nrm1,
                       s.flag, s.reorth, eta2);
    LQCD_HIP(hipGetLastError());
    multi_dot<R>(c, Wb, n, Wrs, j + 1, wn, Wrs, n, nb, s.h2, m + 1, s.flag);
    multi_axpy<R>(c, Wb, n, Wrs, j + 1, s.h2, m + 1, wn, Wrs, n, nb, s.nrm2, s.flag);
    hipLaunchKernelGGL(k_finish_col, dim3(nb), dim3(64), 0, c->stream,
                       reinterpret_cast<cx<double> *>(s.Hd), s.Hrs, m + 1, j,
                       reinterpret_cast<cx<double> *>(s.h1), reinterpret_cast<cx<double> *>(s.h2),
                       size_t(m + 1), s.nrm1, s.nrm2, s.flag, s.inv);
    LQCD_HIP(hipGetLastError());
    scale_dev<R>(c, wn, Wrs, s.inv, wn, Wrs, n, nb);
  }
}

// Arnoldi steps with a 16-bit stored basis (kind BK, half.h): W holds
// the basis as stored vectors ldv words apart (bases Wrs words apart);
// A v_j is formed in FP32 in wt (vectors n apart).  The first
// Gram-Schmidt pass stores its result straight into slot j + 1 with
// per-site scales (not normalised: the scales take the norm afterwards,
// the stored digits do not depend on it); a second pass, where the DGKS
// test asks for one, works on that stored vector in place.  h_{j+1,j} is
// the norm of the stored vector.
template <int BK>
void arnoldi_h(lqcd_ctx *c, const Op<float> &A, void *W, size_t n, size_t ldv, size_t Wrs, int j0,
               int m, int nb, Small &s, double eta2, void *wt) {
  uint32_t *Wb = static_cast<uint32_t *>(W);
  for (int j = j0; j < m; ++j) {
    uint32_t *wn = Wb + size_t(j + 1) * ldv;
    A.template apply_h<BK>(Wb + size_t(j) * ldv, Wrs, wt, n, nb);
    hmulti_dot<BK>(c, Wb, ldv, Wrs, j + 1, wt, n, n, nb, s.h1, m + 1, nullptr);
    hmulti_axpy_q<BK>(c, Wb, ldv, Wrs, j + 1, s.h1, m + 1, wt, n, wn, Wrs, n, nb, s.nrm1, nullptr);
    hipLaunchKernelGGL(k_dgks, dim3(nb), dim3(64), 0, c->stream,
                       reinterpret_cast<const cx<double> *>(s.h1), size_t(m + 1), j + 1, s.nrm1,
                       s.flag, s.reorth, eta2);
    LQCD_HIP(hipGetLastError());
    hmulti_dot<BK>(c, Wb, ldv, Wrs, j + 1, wn, Wrs, n, nb, s.h2, m + 1, s.flag, true);
    hmulti_axpy_q<BK>(c, Wb, ldv, Wrs, j + 1, s.h2, m + 1, nullptr, 0, wn, Wrs, n, nb, s.nrm2, s.flag);
    hipLaunchKernelGGL(k_finish_col, dim3(nb), dim3(64), 0, c->stream,
                       reinterpret_cast<cx<double> *>(s.Hd), s.Hrs, m + 1, j,
                       reinterpret_cast<cx<double> *>(s.h1), reinterpret_cast<cx<double> *>(s.h2),
                       size_t(m + 1), s.nrm1, s.nrm2, s.flag, s.inv);
    LQCD_HIP(hipGetLastError());
    hscale_dev(c, wn, Wrs, n, nb, s.inv);
  }
}

// s-step form of arnoldi_h: Arnoldi steps j0 .. m - 1 in blocks of S
// (2..6).  For a block, z_1 = B v_j and z_k = B z_{k-1} with B = Mhat - 1
// (the shift centres the spectrum of Mhat, a disc about 1, on the origin,
// which keeps the power basis well conditioned; FP32, in the 16-byte pair
// layout) are projected on the basis together, in one dot pass and one
// update pass over it (the single-step form reads the basis twice per
// step), then orthonormalised among themselves by the Cholesky factor of
// their Gram matrix, in FP32, and stored (each stored value rounded once,
// after its whole orthogonalisation, as in the single-step form).  The dot
// pass also yields Z^H Z, so the Gram matrix of the projected block, Z^H Z
// - C^H C, and the Hessenberg columns (k_sstep_finish) are known before the
// update pass, which then stores the basis vectors directly (the direct
// path).  Where the DGKS test or the conditioning of the block asks
// (k_sstep_plan), the right-hand side takes the explicit path instead:
// update in place, a second block pass, the Gram matrix of the final
// vectors, store.  The Krylov space is the same: K(Mhat, v) = K(Mhat - 1,
// v).  A last block shorter than S runs with its own length, a single last
// step in the single-step form.
template <int BK, int S, bool W16>
void sstep_block(lqcd_ctx *c, const Op<float> &A, uint32_t *Wb, size_t n, size_t ldv, size_t Wrs, int j, int m,
                 int nb, Small &s, double eta2, void *wt) {
  constexpr double kSigma = 1.0;
  constexpr int NG = S * S;
  const size_t ldc = size_t(S) * (m + 1);
  const int nblk = int((n / 12 + kBlock - 1) / kBlock);
  const int J = j + 1;
  LQCD_CHECK(J <= kSstepMaxJ, LQCD_EINVAL, "s-step Arnoldi: basis of %d vectors exceeds %d", J, kSstepMaxJ);
  char *q = static_cast<char *>(c->sstep.ensure(2 * ldc * nb * sizeof(cdouble) + size_t(NG) * nb * sizeof(cdouble) +
                                                size_t(NG) * nb * sizeof(double) +
                                                2 * size_t(nb) * nblk * NG * sizeof(double)));
  cdouble *C1 = reinterpret_cast<cdouble *>(q), *C2 = C1 + ldc * nb, *f = C2 + ldc * nb;
  double *G = reinterpret_cast<double *>(f + size_t(NG) * nb), *part = G + size_t(NG) * nb;
  double *gpart = part + size_t(nb) * nblk * NG;
  // vector k of the block, right-hand side r at wt + k wvs + r wrs (complex
  // elements, FP32 pairs; or words, 16-bit stored)
  const size_t wrs = W16 ? ldv : n, wvs = size_t(nb) * wrs;
  auto wk = [&](int k) -> void * {
    return W16 ? static_cast<void *>(static_cast<uint32_t *>(wt) + k * wvs)
               : static_cast<void *>(static_cast<cx<float> *>(wt) + k * wvs);
  };
  uint32_t *out = Wb + size_t(J) * ldv;
  const cx<double> *C1d = reinterpret_cast<const cx<double> *>(C1), *C2d = reinterpret_cast<const cx<double> *>(C2);
  if constexpr (W16) {
    A.template apply_dd_hh<BK>(Wb + size_t(j) * ldv, Wrs, wk(0), wrs, nb);
    for (int k = 1; k < S; ++k) A.template apply_dd_hh<BK>(wk(k - 1), wrs, wk(k), wrs, nb);
  } else {
    A.template apply_dd_h<BK>(Wb + size_t(j) * ldv, Wrs, wk(0), wrs, nb);
    for (int k = 1; k < S; ++k) A.apply_dd(wk(k - 1), wrs, wk(k), wrs, nb);
  }
  hmulti_dots<BK, S, W16>(c, Wb, ldv, Wrs, J, wt, wvs, wrs, n, nb, C1, ldc, nullptr, gpart);
  hipLaunchKernelGGL(k_sstep_plan<S>, dim3(nb), dim3(64), 0, c->stream, gpart, nblk, C1d, ldc, J, G, s.flag,
                     s.reorth, eta2);
  LQCD_HIP(hipGetLastError());
  // direct path: Hessenberg columns and R^{-1} from the plan's Gram matrix,
  // then one update pass that stores the basis vectors
  hipLaunchKernelGGL((k_sstep_finish<S, false>), dim3(nb), dim3(64), 0, c->stream,
                     reinterpret_cast<cx<double> *>(s.Hd), s.Hrs, m + 1, j, C1d, C2d, ldc, part, nblk, G, s.flag,
                     kSigma, reinterpret_cast<cx<double> *>(f));
  LQCD_HIP(hipGetLastError());
  hmulti_axpys_store<BK, S, W16>(c, Wb, ldv, Wrs, J, C1, ldc, wt, wvs, wrs, n, nb, s.flag, f, out, ldv, Wrs);
  // explicit path (flagged right-hand sides): update in place, second block
  // pass, Gram matrix of the final vectors, store
  hmulti_axpys<BK, S, W16>(c, Wb, ldv, Wrs, J, C1, ldc, wt, wvs, wrs, n, nb, nullptr, s.flag);
  hmulti_dots<BK, S, W16>(c, Wb, ldv, Wrs, J, wt, wvs, wrs, n, nb, C2, ldc, s.flag, nullptr);
  hmulti_axpys<BK, S, W16>(c, Wb, ldv, Wrs, J, C2, ldc, wt, wvs, wrs, n, nb, part, s.flag);
  hipLaunchKernelGGL((k_sstep_finish<S, true>), dim3(nb), dim3(64), 0, c->stream,
                     reinterpret_cast<cx<double> *>(s.Hd), s.Hrs, m + 1, j, C1d, C2d, ldc, part, nblk, G, s.flag,
                     kSigma, reinterpret_cast<cx<double> *>(f));
  LQCD_HIP(hipGetLastError());
  hsstore<BK, S, W16>(c, wt, wvs, wrs, f, out, ldv, Wrs, n, nb, s.flag);
}

template <int BK, bool W16>
void arnoldi_hs_impl(lqcd_ctx *c, const Op<float> &A, void *W, size_t n, size_t ldv, size_t Wrs, int j0, int m,
                     int nb, Small &s, double eta2, void *wt, int steps) {
  uint32_t *Wb = static_cast<uint32_t *>(W);
  void *w = wt;
  int j = j0;
  while (j < m) {
    const int b = std::min(steps, m - j);
    if (b == 6)
      sstep_block<BK, 6, W16>(c, A, Wb, n, ldv, Wrs, j, m, nb, s, eta2, w);
    else if (b == 5)
      sstep_block<BK, 5, W16>(c, A, Wb, n, ldv, Wrs, j, m, nb, s, eta2, w);
    else if (b == 4)
      sstep_block<BK, 4, W16>(c, A, Wb, n, ldv, Wrs, j, m, nb, s, eta2, w);
    else if (b == 3)
      sstep_block<BK, 3, W16>(c, A, Wb, n, ldv, Wrs, j, m, nb, s, eta2, w);
    else if (b == 2)
      sstep_block<BK, 2, W16>(c, A, Wb, n, ldv, Wrs, j, m, nb, s, eta2, w);
    else
      arnoldi_h<BK>(c, A, W, n, ldv, Wrs, j, m, nb, s, eta2, wt);  // the one step left
    j += b;
  }
}

// The power vectors in FP32 (pair layout) or, with c->sstep_z16 and an
// FP16 basis, stored in its 16-bit form (the stencil then reads and writes
// them at 52 bytes per site; the Arnoldi relation carries their rounding,
// 2^-11 relative: BF16's 2^-8 costs cycles, so a BF16 basis keeps them in
// FP32).
template <int BK>
void arnoldi_hs(lqcd_ctx *c, const Op<float> &A, void *W, size_t n, size_t ldv, size_t Wrs, int j0, int m, int nb,
                Small &s, double eta2, void *wt, int steps) {
  if constexpr (BK == int(HKind::F16)) {
    if (c->sstep_z16) {
      arnoldi_hs_impl<BK, true>(c, A, W, n, ldv, Wrs, j0, m, nb, s, eta2, wt, steps);
      return;
    }
  }
  arnoldi_hs_impl<BK, false>(c, A, W, n, ldv, Wrs, j0, m, nb, s, eta2, wt, steps);
}

// MINRES-DR basis extension (one right-hand side, FP64; hermitian A):
// column j0 is orthogonalised twice against every vector before it (it
// couples to all kept vectors of the restart); each later column by the
// three-term recurrence against v_{j-1}, v_j, then once more against those
// two when the DGKS test asks for it, and on every other step (and the
// last) against the first `kept` vectors (the kept vectors of the last
// restart: selective reorthogonalisation against the approximate
// eigenvectors), whose update runs only when a coefficient exceeds
// kKeptTau |w|.  Both passes' coefficients add into column j of Hbar.
void lanczos_ext(lqcd_ctx *c, const Op<double> &A, void *V, size_t n, int j0, int m, int kept, Small &s) {
  cx<double> *Vb = static_cast<cx<double> *>(V);
  const size_t hb = size_t(m + 1) * sizeof(cdouble);
  for (int j = j0; j < m; ++j) {
    cx<double> *wj = Vb + size_t(j) * n, *wn = Vb + size_t(j + 1) * n;
    A.apply(wj, 0, wn, 0, 1);
    if (j == j0) {  // full classical Gram-Schmidt, twice
      multi_dot<double>(c, Vb, n, 0, j + 1, wn, 0, n, 1, s.h1, m + 1);
      multi_axpy<double>(c, Vb, n, 0, j + 1, s.h1, m + 1, wn, 0, n, 1, s.nrm1);
      hipLaunchKernelGGL(k_dgks, dim3(1), dim3(64), 0, c->stream,
                         reinterpret_cast<const cx<double> *>(s.h1), size_t(m + 1), j + 1, s.nrm1, s.flag,
                         s.reorth, kReorthAlways);
      LQCD_HIP(hipGetLastError());
      multi_dot<double>(c, Vb, n, 0, j + 1, wn, 0, n, 1, s.h2, m + 1);
      multi_axpy<double>(c, Vb, n, 0, j + 1, s.h2, m + 1, wn, 0, n, 1, s.nrm2);
      hipLaunchKernelGGL(k_finish_col, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<cx<double> *>(s.Hd),
                         s.Hrs, m + 1, j, reinterpret_cast<cx<double> *>(s.h1),
                         reinterpret_cast<cx<double> *>(s.h2), size_t(m + 1), s.nrm1, s.nrm2, s.flag, s.inv);
      LQCD_HIP(hipGetLastError());
      scale_dev<double>(c, wn, 0, s.inv, wn, 0, n, 1);
      continue;
    }
    cx<double> *wp = Vb + size_t(j - 1) * n;
    fill_zero(c, s.h1, hb);
    fill_zero(c, s.h2, hb);
    multi_dot<double>(c, wp, n, 0, 2, wn, 0, n, 1, s.h1 + (j - 1), m + 1);
    multi_axpy<double>(c, wp, n, 0, 2, s.h1 + (j - 1), m + 1, wn, 0, n, 1, s.nrm1);
    if (kept >= j - 1) {  // kept vectors and v_{j-1}, v_j are one range
      hipLaunchKernelGGL(k_dgks, dim3(1), dim3(64), 0, c->stream,
                         reinterpret_cast<const cx<double> *>(s.h1), size_t(m + 1), j + 1, s.nrm1, s.flag,
                         s.scratch_count, kReorthAlways);
      LQCD_HIP(hipGetLastError());
      multi_dot<double>(c, Vb, n, 0, j + 1, wn, 0, n, 1, s.h2, m + 1);
      multi_axpy<double>(c, Vb, n, 0, j + 1, s.h2, m + 1, wn, 0, n, 1, s.nrm2);
      hipLaunchKernelGGL(k_count1, dim3(1), dim3(1), 0, c->stream, s.reorth);
      LQCD_HIP(hipGetLastError());
    } else {
      // second pass against v_{j-1}, v_j by the DGKS test (its count is not
      // reported: MINRES-DR reports the kept-vector updates)
      hipLaunchKernelGGL(k_dgks, dim3(1), dim3(64), 0, c->stream,
                         reinterpret_cast<const cx<double> *>(s.h1), size_t(m + 1), j + 1, s.nrm1, s.flag,
                         s.scratch_count, kReorthDR);
      LQCD_HIP(hipGetLastError());
      multi_dot<double>(c, wp, n, 0, 2, wn, 0, n, 1, s.h2 + (j - 1), m + 1, s.flag);
      // the kept vectors are tested on every kept_period-th step (16 by
      // default) and on the last step of a cycle (their coefficients stay
      // zero otherwise)
      const bool test = kept > 0 && ((j - j0) % c->kept_period == c->kept_period - 1 || j == m - 1);
      if (test) {
        multi_dot<double>(c, Vb, n, 0, kept, wn, 0, n, 1, s.h2, m + 1);
        hipLaunchKernelGGL(k_kept_test, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<cx<double> *>(s.h2),
                           kept, s.nrm1, kKeptTau * kKeptTau, s.kflag, s.flag, s.reorth);
        LQCD_HIP(hipGetLastError());
        multi_axpy<double>(c, Vb, n, 0, kept, s.h2, m + 1, wn, 0, n, 1, nullptr, s.kflag);
      }
      // runs whenever either update is needed (with zero coefficients when
      // only the kept vectors' is), so that |w|^2 after the pass is formed
      multi_axpy<double>(c, wp, n, 0, 2, s.h2 + (j - 1), m + 1, wn, 0, n, 1, s.nrm2, s.flag);
    }
    hipLaunchKernelGGL(k_finish_col, dim3(1), dim3(64), 0, c->stream, reinterpret_cast<cx<double> *>(s.Hd),
                       s.Hrs, m + 1, j, reinterpret_cast<cx<double> *>(s.h1),
                       reinterpret_cast<cx<double> *>(s.h2), size_t(m + 1), s.nrm1, s.nrm2, s.flag, s.inv);
    LQCD_HIP(hipGetLastError());
    scale_dev<double>(c, wn, 0, s.inv, wn, 0, n, 1);
  }
}

// Add the per-slot second-pass counts to the host counters and reset them.
void harvest_reorth(lqcd_ctx *c, Small &s, int nb, const std::vector<int> &slot_to_rhs,
                    std::vector<int> &reorth) {
  std::vector<int> h(nb);
  d2h(c, h.data(), s.reorth, nb * sizeof(int));
  for (int r = 0; r < nb; ++r) reorth[slot_to_rhs[r]] += h[r];
  hipLaunchKernelGGL(k_izero, dim3(1), dim3(256), 0, c->stream, s.reorth, nb);
  LQCD_HIP(hipGetLastError());
}

bool finite_mat(const la::Mat &H) {
  for (auto &z : H.a)
    if (!std::isfinite(z.real()) || !std::isfinite(z.imag())) return false;
  return true;
}

// Harmonic Ritz restart data of an (m+1) x m Hessenberg-type matrix.
struct Restart {
  la::Mat P;                 // (m+1) x (k+1), orthonormal
  std::vector<cdouble> theta;
  std::vector<double> resid;
};

Restart harmonic_restart(const la::Mat &H, int m, int k) {
  la::Mat Hm(m, m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) Hm(i, j) = H(i, j);
  const cdouble h = H(m, m - 1);
  std::vector<cdouble> em(m, 0.0);
  em[m - 1] = 1.0;
  std::vector<cdouble> f = la::solve(la::adjoint(Hm), em);
  la::Mat G = Hm;
  const double h2 = std::norm(h);
  for (int i = 0; i < m; ++i) G(i, m - 1) += h2 * f[i];
  std::vector<cdouble> th;
  la::Mat g;
  LQCD_CHECK(la::eig(G, th, g), LQCD_ENOCONV, "harmonic Ritz eigenproblem did not converge");
  std::vector<int> ord(m);
  for (int i = 0; i < m; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int a, int b) { return std::abs(th[a]) < std::abs(th[b]); });
  la::Mat P(m + 1, k + 1);
  std::vector<cdouble> w(m + 1);
  double wn = 0;
  for (int i = 0; i < m; ++i) {
    w[i] = -h2 * f[i];
    wn += std::norm(w[i]);
  }
  w[m] = h;
  wn = std::sqrt(wn + h2);
  Restart R;
  for (int q = 0; q < k; ++q) {
    int col = ord[q];
    double gn = 0;
    for (int i = 0; i < m; ++i) {
      P(i, q) = g(i, col);
      gn += std::norm(g(i, col));
    }
    R.theta.push_back(th[col]);
    R.resid.push_back(std::abs(g(m - 1, col)) * wn / std::sqrt(gn));
  }
  for (int i = 0; i <= m; ++i) P(i, k) = w[i];
  la::QR qr;
  qr.factor(P);
  R.P = qr.thin_q();
  return R;
}

// MINRES-DR restart data: harmonic Ritz pairs of a hermitian operator from
// the pencil H_m^H g = mu Hbar^H Hbar g, theta = 1 / mu, which never solves
// with H_m (singular when a Ritz value of an indefinite operator crosses
// zero).  With L L^H = Hbar^H Hbar it is the eigenproblem of
// L^{-1} H_m^H L^{-H} (hermitian up to rounding), g = L^{-H} y.  H_m is
// used as computed: pairs of its hermitian part would not be exact for the
// computed Hbar, and the restart relation would decay from cycle to cycle.
// The residual direction is the unit vector orthogonal to range(Hbar),
// taken from the QR factorisation of [Hbar | e_m].
Restart harmonic_restart_herm(const la::Mat &H, int m, int k) {
  la::Mat Hm(m, m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) Hm(i, j) = H(i, j);
  la::Mat Li;
  LQCD_CHECK(la::cholesky_inv(la::matmul_hn(H, H), Li), LQCD_ENOCONV,
             "MINRES-DR: Hbar^H Hbar is not positive definite");
  la::Mat C = la::matmul(Li, la::matmul(la::adjoint(Hm), la::adjoint(Li)));
  std::vector<cdouble> mu;
  la::Mat Y;
  LQCD_CHECK(la::eig(C, mu, Y), LQCD_ENOCONV, "MINRES-DR: harmonic Ritz eigenproblem did not converge");
  la::Mat G = la::matmul_hn(Li, Y);  // g = L^{-H} y
  std::vector<int> ord(m);
  for (int i = 0; i < m; ++i) ord[i] = i;
  // smallest |theta| = largest |mu|; ties by index
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return std::abs(mu[a]) > std::abs(mu[b]); });
  la::Mat He(m + 1, m + 1);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i <= m; ++i) He(i, j) = H(i, j);
  He(m, m) = 1.0;
  la::QR qe;
  qe.factor(He);
  const la::Mat Qe = qe.thin_q();
  la::Mat P(m + 1, k + 1);
  Restart R;
  for (int q = 0; q < k; ++q) {
    const int col = ord[q];
    const cdouble th = mu[col] != cdouble(0, 0) ? 1.0 / mu[col]
                                                 : cdouble(std::numeric_limits<double>::infinity(), 0);
    double gn = 0, rn = 0;
    for (int i = 0; i < m; ++i) {
      P(i, q) = G(i, col);
      gn += std::norm(G(i, col));
    }
    for (int i = 0; i <= m; ++i) {  // |Hbar g - theta [g; 0]|
      cdouble v = 0;
      for (int j = 0; j < m; ++j) v += H(i, j) * G(j, col);
      if (i < m) v -= th * G(i, col);
      rn += std::norm(v);
    }
    R.theta.push_back(th);
    R.resid.push_back(std::sqrt(rn / gn));
  }
  for (int i = 0; i <= m; ++i) P(i, k) = Qe(i, m);
  la::QR qr;
  qr.factor(P);
  R.P = qr.thin_q();
  return R;
}

la::Mat sub(const la::Mat &A, int r, int c) {
  la::Mat B(r, c);
  for (int j = 0; j < c; ++j)
    for (int i = 0; i < r; ++i) B(i, j) = A(i, j);
  return B;
}

// ------------------------------------------------------------ GMRES-DR
// Solves A x = S (x starts at zero) for one right-hand side in FP64 and
// leaves the deflation data in d.  Returns true when it stopped on its
// targets (residual <= tol_super |S| and, with eig_tol, the n_eig smallest
// harmonic Ritz pairs converged), false when max_cycles ended it first.
bool gmres_dr(lqcd_ctx *c, const Op<double> &A, const void *S, void *X, const lqcd_solve_params &p,
              lqcd_defl *d, lqcd_solve_stats &st) {
  const int m = p.m, k = p.k;
  const size_t n = A.n;
  cx<double> *V = static_cast<cx<double> *>(d->V.ensure(size_t(m + 1) * n * sizeof(cx<double>)));
  Small s(c->small[0]);
  s.setup(m, 1, m);
  hipLaunchKernelGGL(k_izero, dim3(1), dim3(256), 0, c->stream, s.reorth, 1);
  std::vector<int> reorth1(1, 0);
  double *nrm_host = nullptr;
  double b2 = 0;
  norm2<double>(c, S, 0, n, 1, s.nrm2);
  d2h(c, &b2, s.nrm2, sizeof(double));
  (void)nrm_host;
  const double bnorm = std::sqrt(b2);
  LQCD_CHECK(std::isfinite(bnorm), LQCD_ENAN, "gmresdr_solve: right-hand side is not finite");
  fill_zero(c, X, n * sizeof(cx<double>));
  if (bnorm == 0.0) {
    LQCD_CHECK(false, LQCD_EINVAL, "gmresdr_solve: GMRES-DR needs a nonzero first right-hand side");
  }
  cdouble a(1.0 / bnorm, 0), zero(0, 0);
  axpby<double>(c, &a, S, 0, &zero, V, 0, n, 1, false);
  la::Mat H(m + 1, m);
  std::vector<cdouble> cv(m + 1, 0.0);
  cv[0] = bnorm;
  int j0 = 0;
  std::vector<cdouble> Hcols;
  int nev = p.n_eig > 0 ? std::min(p.n_eig, k) : k;
  const bool lz = p.method == LQCD_KRYLOV_MINRESDR;
  int kept = 0;  // MINRES-DR: vectors kept by the last restart
  bool converged = false;
  for (;;) {
    if (lz) lanczos_ext(c, A, V, n, j0, m, kept, s);
    else arnoldi<double>(c, A, V, n, 0, j0, m, 1, s, kReorthDR);
    st.matvecs += m - j0;
    harvest_reorth(c, s, 1, std::vector<int>{0}, reorth1);
    st.reorth = reorth1[0];
    Hcols.resize(size_t(m + 1) * m);
    d2h(c, Hcols.data(), s.Hd, Hcols.size() * sizeof(cdouble));
    // column j of the device matrix holds rows 0..j+1 only (the rest is stale)
    for (int j = j0; j < m; ++j)
      for (int i = 0; i <= m; ++i) H(i, j) = i <= j + 1 ? Hcols[size_t(j) * (m + 1) + i] : cdouble(0, 0);
    LQCD_CHECK(finite_mat(H), LQCD_ENAN, "gmresdr_solve: NaN/Inf in the Arnoldi process");
    for (int j = j0; j < m; ++j)
      LQCD_CHECK(std::abs(H(j + 1, j)) > 0, LQCD_EBREAKDOWN,
                 "gmresdr_solve: Arnoldi breakdown at column %d", j);
    std::vector<cdouble> dv = la::lstsq(H, cv);
    std::vector<cdouble> sv(cv);
    for (int j = 0; j < m; ++j)
      for (int i = 0; i <= m; ++i) sv[i] -= H(i, j) * dv[j];
    double res = 0;
    for (auto &z : sv) res += std::norm(z);
    res = std::sqrt(res);
    h2d(c, s.vec, dv.data(), size_t(m) * sizeof(cdouble));
    gemm_nn<double>(c, V, n, 0, m, s.vec, m, 0, X, n, 0, 1, n, 1, 1.0);
    st.cycles += 1;
    Restart R = lz ? harmonic_restart_herm(H, m, k) : harmonic_restart(H, m, k);
    bool done = res <= p.tol_super * bnorm;
    if (done && p.eig_tol > 0)
      for (int q = 0; q < nev; ++q)
        if (R.resid[q] > p.eig_tol * std::abs(R.theta[q])) done = false;
    // restart: V_{k+1} = V_{m+1} P_{k+1}, Hbar_k = P^H Hbar_m P_k, c = P^H s
    h2d(c, s.vec, R.P.a.data(), R.P.a.size() * sizeof(cdouble));
    recombine<double>(c, V, n, m + 1, s.vec, m + 1, k + 1, n);
    la::Mat Pk = sub(R.P, m, k);
    la::Mat Hk = la::matmul_hn(R.P, la::matmul(H, Pk));
    std::vector<cdouble> cn(k + 1, 0.0);
    for (int q = 0; q <= k; ++q)
      for (int i = 0; i <= m; ++i) cn[q] += std::conj(R.P(i, q)) * sv[i];
    d->H = Hk;
    d->theta = R.theta;
    d->theta_resid = R.resid;
    converged = done;
    if (done || st.cycles >= p.max_cycles) break;
    H = la::Mat(m + 1, m);
    for (int j = 0; j < k; ++j)
      for (int i = 0; i <= k; ++i) H(i, j) = Hk(i, j);
    std::fill(cv.begin(), cv.end(), cdouble(0, 0));
    for (int q = 0; q <= k; ++q) cv[q] = cn[q];
    j0 = k;
    kept = k + 1;
  }
  d->k = k;
  d->n = n;
  d->Hqr.factor(d->H);
  d->have_v32 = false;
  return converged;
}

// ---------------------------------------------------------- GMRES-Proj
// Batched solve of A X = S (nb right-hand sides, vectors n apart) with
// precision R, from X = 0, until |S - A X| <= tol * ref[r] or max_cycles.
// Vdef: V_{k+1} of precision R.  Works in place on X; S is not modified
// (its slots may be permuted internally and are restored on return).
// An inner solve of iterative refinement (cycle_cap > 0) also stops after
// cycle_cap cycles of this call, or when a cycle leaves the residual above
// `stall` times the previous one: it only has to shrink the residual.
// BK >= 0 (R = float only): the GMRES(p) basis W is stored in 16 bits
// (half.h kind BK) and wt is FP32 scratch of nb vectors.
template <class R, int BK = -1>
void proj_solve(lqcd_ctx *c, const Op<R> &A, const void *Vdef, const lqcd_defl *d, int p, void *S,
                void *X, void *Rr, void *W, int nb, std::vector<double> ref, double tol,
                int max_cycles, std::vector<int> &matvecs, std::vector<int> &cycles,
                std::vector<double> &resid, std::vector<int> &reorth, int cycle_cap = 0,
                double stall = 0.0, void *wt = nullptr) {
  static_assert(BK < 0 || std::is_same<R, float>::value, "16-bit bases hold FP32 solves");
  const size_t n = A.n;
  const int k = d->k;
  Small s(c->small[0]);
  s.setup(p, nb, k);
  hipLaunchKernelGGL(k_izero, dim3(1), dim3(256), 0, c->stream, s.reorth, nb);
  LQCD_HIP(hipGetLastError());
  const size_t vb = n * sizeof(cx<R>);
  cx<R> *Sb = static_cast<cx<R> *>(S), *Xb = static_cast<cx<R> *>(X), *Rb = static_cast<cx<R> *>(Rr);
  std::vector<int> slot_of(nb), perm(nb);  // perm[slot] = original rhs
  for (int r = 0; r < nb; ++r) perm[r] = r;
  std::vector<std::pair<int, int>> swaps;
  fill_zero(c, X, vb * nb);
  copy_dev(c, Rr, S, vb * nb);  // r = S - A 0
  int na = nb;
  std::vector<double> rn(nb), prev(nb, -1.0);
  std::vector<int> here(nb, 0);  // cycles of this call, per slot
  auto swap_slots = [&](int a, int b) {
    swap_vec<R>(c, Sb + a * n, Sb + b * n, n);
    swap_vec<R>(c, Xb + a * n, Xb + b * n, n);
    swap_vec<R>(c, Rb + a * n, Rb + b * n, n);
    std::swap(perm[a], perm[b]);
    std::swap(ref[a], ref[b]);
    std::swap(rn[a], rn[b]);
    std::swap(prev[a], prev[b]);
    std::swap(here[a], here[b]);
    swaps.emplace_back(a, b);
  };
  std::vector<cdouble> Ch, Dh, Eh, Hh;
  for (;;) {
    // residual norms and convergence; compact the active slots
    norm2<R>(c, Rb, n, n, na, s.nrm2);
    d2h(c, rn.data(), s.nrm2, size_t(na) * sizeof(double));
    for (int r = 0; r < na; ++r) {
      rn[r] = std::sqrt(rn[r]);
      LQCD_CHECK(std::isfinite(rn[r]), LQCD_ENAN, "gmresdr_solve: NaN/Inf residual");
      resid[perm[r]] = rn[r] / (ref[r] > 0 ? ref[r] : 1.0);
    }
    for (int r = 0; r < na;) {
      // ref <= 0 marks a right-hand side the caller does not want solved
      const bool capped = cycle_cap > 0 && here[r] >= cycle_cap;
      const bool stalled = stall > 0 && prev[r] > 0 && rn[r] > stall * prev[r];
      if (ref[r] <= 0 || rn[r] <= tol * ref[r] || cycles[perm[r]] >= max_cycles || capped || stalled) {
        if (r != na - 1) swap_slots(r, na - 1);
        --na;
      } else {
        ++r;
      }
    }
    if (na == 0) break;
    for (int r = 0; r < na; ++r) {
      prev[r] = rn[r];
      here[r] += 1;
    }
    // projection over the deflation space: c = V^H r, d = argmin |c - Hbar d|
    gemm_tn<R>(c, Vdef, n, k + 1, Rb, n, na, n, s.C, k + 1);
    Ch.resize(size_t(k + 1) * na);
    d2h(c, Ch.data(), s.C, Ch.size() * sizeof(cdouble));
    Dh.assign(size_t(k) * na, 0.0);
    Eh.assign(size_t(k + 1) * na, 0.0);
    for (int r = 0; r < na; ++r) {
      std::vector<cdouble> y(Ch.begin() + size_t(r) * (k + 1), Ch.begin() + size_t(r + 1) * (k + 1));
      d->Hqr.apply_qh(y.data());
      d->Hqr.solve_r(y.data());
      for (int j = 0; j < k; ++j) Dh[size_t(r) * k + j] = y[j];
      for (int j = 0; j < k; ++j)
        for (int i = 0; i <= k; ++i) Eh[size_t(r) * (k + 1) + i] += d->H(i, j) * y[j];
    }
    h2d(c, s.C, Dh.data(), Dh.size() * sizeof(cdouble));
    h2d(c, s.E, Eh.data(), Eh.size() * sizeof(cdouble));
    gemm_nn<R>(c, Vdef, n, 0, k, s.C, k, 0, Xb, n, 0, na, n, 1, 1.0);
    gemm_nn<R>(c, Vdef, n, 0, k + 1, s.E, k + 1, 0, Rb, n, 0, na, n, 1, -1.0);
    // one GMRES(p) cycle per active rhs
    norm2<R>(c, Rb, n, n, na, s.nrm2);
    d2h(c, rn.data(), s.nrm2, size_t(na) * sizeof(double));
    std::vector<cdouble> sc(na), zs(na, 0.0);
    for (int r = 0; r < na; ++r) {
      rn[r] = std::sqrt(rn[r]);
      sc[r] = rn[r] > 0 ? 1.0 / rn[r] : 0.0;
    }
    const size_t ldh = hvec_words(n / 12);
    const size_t Wrs = BK >= 0 ? size_t(p + 1) * ldh : size_t(p + 1) * n;
    if constexpr (BK >= 0) {
      norm2<R>(c, Rb, n, n, na, s.nrm2);
      inv_sqrt_dev(c, s.nrm2, s.inv, na);
      hquantize<BK>(c, Rb, n, s.inv, W, Wrs, n, na);
      const double eta2 = c->cycle_reorth ? kReorthAlways : kReorthCycle;
      if (c->arnoldi_steps > 1)
        arnoldi_hs<BK>(c, A, W, n, ldh, Wrs, 0, p, na, s, eta2, wt, c->arnoldi_steps);
      else
        arnoldi_h<BK>(c, A, W, n, ldh, Wrs, 0, p, na, s, eta2, wt);
    } else {
      axpby<R>(c, sc.data(), Rb, n, zs.data(), W, Wrs, n, na, true);
      arnoldi<R>(c, A, W, n, Wrs, 0, p, na, s, c->cycle_reorth ? kReorthAlways : kReorthCycle);
    }
    harvest_reorth(c, s, na, perm, reorth);
    Hh.resize(s.Hrs * na);
    d2h(c, Hh.data(), s.Hd, Hh.size() * sizeof(cdouble));
    std::vector<cdouble> dall(size_t(p) * na);
    for (int r = 0; r < na; ++r) {
      la::Mat H(p + 1, p);
      for (int j = 0; j < p; ++j)
        for (int i = 0; i <= j + 1; ++i) H(i, j) = Hh[r * s.Hrs + size_t(j) * (p + 1) + i];
      LQCD_CHECK(finite_mat(H), LQCD_ENAN, "gmresdr_solve: NaN/Inf in the Arnoldi process");
      std::vector<cdouble> cvec(p + 1, 0.0);
      cvec[0] = rn[r];
      std::vector<cdouble> dv = la::lstsq(H, cvec);
      std::copy(dv.begin(), dv.end(), dall.begin() + size_t(r) * p);
      matvecs[perm[r]] += p + 1;
      cycles[perm[r]] += 1;
    }
    h2d(c, s.vec, dall.data(), dall.size() * sizeof(cdouble));
    if constexpr (BK >= 0)
      hgemm_nn<BK>(c, W, ldh, Wrs, p, s.vec, p, p, Xb, n, n, 1, n, na, 1.0);
    else
      gemm_nn<R>(c, W, n, Wrs, p, s.vec, p, p, Xb, n, n, 1, n, na, 1.0);
    // true residual r = S - A X
    A.apply(Xb, n, Rb, n, na);
    cdouble one(1, 0), mone(-1, 0);
    axpby<R>(c, &one, Sb, n, &mone, Rb, n, n, na, false);
  }
  // restore the caller's slot order
  for (auto it = swaps.rbegin(); it != swaps.rend(); ++it) {
    swap_vec<R>(c, Sb + it->first * n, Sb + it->second * n, n);
    swap_vec<R>(c, Xb + it->first * n, Xb + it->second * n, n);
  }
}

// ------------------------------------------------------------- drivers
// Solver buffers live in the context so that repeated calls reuse them.
struct Work {
  DevBuf &Bp, &S, &X, &R, &W, &XF, &T, &S32, &X32, &R32, &W32, &tmp64, &tmp32, &red2, &WT;
  explicit Work(lqcd_ctx *c)
      : Bp(c->sw[0]), S(c->sw[1]), X(c->sw[2]), R(c->sw[3]), W(c->sw[4]), XF(c->sw[5]),
        T(c->sw[6]), S32(c->sw[7]), X32(c->sw[8]), R32(c->sw[9]), W32(c->sw[10]),
        tmp64(c->sw[11]), tmp32(c->sw[12]), red2(c->sw[13]), WT(c->sw[14]) {}
};

// Pack nb right-hand sides and build the system's source:
// SCHUR: S = eta_e + kappa D_eo eta_o (half vectors); MG5: S = b.
void make_source(lqcd_ctx *c, lqcd_op op, const void *b_lex, int nb, Work &w, size_t n) {
  const size_t hl = half_len(c->g), fl = full_len(c->g);
  cx<double> *Bp = static_cast<cx<double> *>(w.Bp.ensure(fl * nb * sizeof(cx<double>)));
  cx<double> *S = static_cast<cx<double> *>(w.S.ensure(n * nb * sizeof(cx<double>)));
  pack_eo<double>(c, b_lex, Bp, nb, fl);
  if (op == LQCD_OP_SCHUR)
    hop_half<double>(c, 0, Bp + hl, Bp, S, cdouble(1, 0), c->kappa, false, false, nb, fl, fl, n);
  else
    copy_dev(c, S, Bp, fl * nb * sizeof(cx<double>));
}

// x (lex) from the internal solution; true residual |b - A x| / |b| (full).
void finish(lqcd_ctx *c, lqcd_op op, const void *X, void *x_lex, int nb, Work &w, size_t n,
            std::vector<double> &true_resid) {
  const size_t hl = half_len(c->g), fl = full_len(c->g);
  cx<double> *Bp = w.Bp.as<cx<double>>();
  cx<double> *XF = static_cast<cx<double> *>(w.XF.ensure(fl * nb * sizeof(cx<double>)));
  cx<double> *T = static_cast<cx<double> *>(w.T.ensure(fl * nb * sizeof(cx<double>)));
  const cx<double> *Xs = static_cast<const cx<double> *>(X);
  if (op == LQCD_OP_SCHUR) {
    for (int r = 0; r < nb; ++r) copy_dev(c, XF + r * fl, Xs + r * n, hl * sizeof(cx<double>));
    // x_o = eta_o + kappa D_oe x_e
    hop_half<double>(c, 1, XF, Bp + hl, XF + hl, cdouble(1, 0), c->kappa, false, false, nb, fl, fl, fl);
  } else {
    copy_dev(c, XF, Xs, fl * nb * sizeof(cx<double>));
  }
  unpack_eo<double>(c, XF, x_lex, nb, fl);
  apply_full<double>(c, op == LQCD_OP_SCHUR ? LQCD_OP_M : LQCD_OP_MG5, XF, T, nb, fl, fl);
  cdouble one(1, 0), mone(-1, 0);
  axpby<double>(c, &one, Bp, fl, &mone, T, fl, fl, nb, false);
  double *d2 = static_cast<double *>(w.red2.ensure(2 * nb * sizeof(double)));
  norm2<double>(c, T, fl, fl, nb, d2);
  norm2<double>(c, Bp, fl, fl, nb, d2 + nb);
  std::vector<double> h(2 * nb);
  d2h(c, h.data(), d2, h.size() * sizeof(double));
  true_resid.resize(nb);
  for (int r = 0; r < nb; ++r) true_resid[r] = std::sqrt(h[r]) / std::max(std::sqrt(h[nb + r]), 1e-300);
}

void full_norms(lqcd_ctx *c, Work &w, int nb, std::vector<double> &out) {
  const size_t fl = full_len(c->g);
  double *d2 = static_cast<double *>(w.red2.ensure(2 * nb * sizeof(double)));
  norm2<double>(c, w.Bp.ptr, fl, fl, nb, d2);
  out.resize(nb);
  d2h(c, out.data(), d2, nb * sizeof(double));
  for (auto &v : out) v = std::sqrt(v);
}

}  // namespace

void defl_eigpairs(lqcd_ctx *c, lqcd_defl *d, int Q) {
  LQCD_CHECK(d->op == LQCD_OP_MG5, LQCD_EINVAL, "eigenpairs need a deflation space of M' (op MG5)");
  LQCD_CHECK(Q >= 1 && Q <= d->k, LQCD_EINVAL, "Q = %d outside 1..k = %d", Q, d->k);
  std::lock_guard<std::mutex> lk(d->fill_mu);
  if (d->Qe == Q && d->E.ptr) return;
  const int k = d->k;
  la::Mat T = sub(d->H, k, k);
  std::vector<double> lam;
  la::Mat Sv;
  la::eigh(T, lam, Sv);
  std::vector<int> ord(k);
  for (int i = 0; i < k; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (std::abs(lam[a]) != std::abs(lam[b])) return std::abs(lam[a]) < std::abs(lam[b]);
    return lam[a] < lam[b];
  });
  la::Mat S(k, Q);
  d->lam.resize(Q);
  d->lam_resid.resize(Q);
  for (int q = 0; q < Q; ++q) {
    d->lam[q] = lam[ord[q]];
    for (int i = 0; i < k; ++i) S(i, q) = Sv(i, ord[q]);
  }
  // residuals |Hbar_k s - lambda [s; 0]|
  la::Mat HS = la::matmul(d->H, S);
  for (int q = 0; q < Q; ++q) {
    double r = 0;
    for (int i = 0; i <= k; ++i) {
      cdouble v = HS(i, q) - (i < k ? d->lam[q] * S(i, q) : cdouble(0, 0));
      r += std::norm(v);
    }
    d->lam_resid[q] = std::sqrt(r);
  }
  // E = V_k S
  cx<double> *E = static_cast<cx<double> *>(d->E.ensure(size_t(Q) * d->n * sizeof(cx<double>)));
  DevBuf Sd;
  Sd.ensure(S.a.size() * sizeof(cdouble));
  h2d(c, Sd.ptr, S.a.data(), S.a.size() * sizeof(cdouble));
  fill_zero(c, E, size_t(Q) * d->n * sizeof(cx<double>));
  gemm_nn<double>(c, d->V.ptr, d->n, 0, k, Sd.as<cdouble>(), k, 0, E, d->n, 0, Q, d->n, 1, 1.0);
  LQCD_HIP(hipStreamSynchronize(c->stream));
  d->Qe = Q;
  d->bil.clear();
  d->xi_cache.clear();
  d->lex_Q = 0;
}

}  // namespace lqcd

using namespace lqcd;

extern "C" lqcd_status gmresdr_solve(lqcd_ctx *c, lqcd_op op, const lqcd_solve_params *pp,
                                     const void *b, void *x, int nrhs, lqcd_defl **defl_inout,
                                     lqcd_solve_stats *stats) {
  return guarded([&] {
    LQCD_CHECK(c && pp && defl_inout, LQCD_EINVAL, "gmresdr_solve: null argument");
    LQCD_CHECK(op == LQCD_OP_SCHUR || op == LQCD_OP_MG5, LQCD_EINVAL,
               "gmresdr_solve: op must be LQCD_OP_SCHUR or LQCD_OP_MG5");
    LQCD_CHECK(nrhs >= 0, LQCD_EINVAL, "gmresdr_solve: nrhs < 0");
    LQCD_CHECK(nrhs == 0 || (b && x), LQCD_EINVAL, "gmresdr_solve: null field");
    const lqcd_solve_params p = *pp;
    LQCD_CHECK(p.k >= 1 && p.m > p.k && p.m <= 250, LQCD_EINVAL,
               "gmresdr_solve: need 1 <= k < m <= 250 (m=%d, k=%d)", p.m, p.k);
    LQCD_CHECK(p.tol > 0 && p.max_cycles >= 1, LQCD_EINVAL, "gmresdr_solve: bad tol/max_cycles");
    LQCD_CHECK(p.inner >= LQCD_F64 && p.inner <= LQCD_BF16, LQCD_EINVAL,
               "gmresdr_solve: bad inner precision");
    LQCD_CHECK(op == LQCD_OP_SCHUR || p.inner == LQCD_F64 || p.inner == LQCD_F32, LQCD_EINVAL,
               "gmresdr_solve: 16-bit storage is available for LQCD_OP_SCHUR only");
    LQCD_CHECK(p.method == LQCD_KRYLOV_GMRESDR || p.method == LQCD_KRYLOV_MINRESDR, LQCD_EINVAL,
               "gmresdr_solve: unknown method %d", p.method);
    LQCD_CHECK(p.method != LQCD_KRYLOV_MINRESDR || op == LQCD_OP_MG5, LQCD_EINVAL,
               "gmresdr_solve: MINRES-DR needs the hermitian LQCD_OP_MG5");
    const size_t n = op == LQCD_OP_SCHUR ? half_len(c->g) : full_len(c->g);
    const size_t fl = full_len(c->g);
    if (stats)
      for (int r = 0; r < nrhs; ++r) stats[r] = lqcd_solve_stats{0, 0, 0, 0, 0.0};
    if (nrhs == 0) return;
    Work w(c);
    Op<double> A64{c, op, n, &w.tmp64};
    Op<float> A32{c, op, n, &w.tmp32};
    lqcd_defl *d = *defl_inout;
    int start = 0;
    std::vector<double> tr;
    bool nonconv = false;
    if (!d) {
      std::unique_ptr<lqcd_defl> nd(new lqcd_defl());
      nd->op = op;
      for (int i = 0; i < 4; ++i) nd->dims[i] = c->g.L[i];
      nd->kappa = c->kappa;
      make_source(c, op, b, 1, w, n);
      void *X = w.X.ensure(n * sizeof(cx<double>));
      lqcd_solve_stats st{0, 0, 0, 0, 0.0};
      lqcd_solve_params pd = p;
      pd.tol_super = std::max(0.0, std::min(p.tol_super > 0 ? p.tol_super : p.tol, p.tol));
      // a first right-hand side cut off by max_cycles has missed its residual
      // target, or left a deflation space short of eig_tol: ENOCONV, with
      // the iterate in x and the space still returned
      if (!gmres_dr(c, A64, w.S.ptr, X, pd, nd.get(), st)) nonconv = true;
      finish(c, op, X, x, 1, w, n, tr);
      st.true_resid = tr[0];
      if (stats) stats[0] = st;
      d = nd.release();
      *defl_inout = d;
      start = 1;
    } else {
      LQCD_CHECK(d->op == op, LQCD_EINVAL, "gmresdr_solve: deflation space built for another operator");
      for (int i = 0; i < 4; ++i)
        LQCD_CHECK(d->dims[i] == c->g.L[i], LQCD_EINVAL, "gmresdr_solve: deflation space of another lattice");
      LQCD_CHECK(d->kappa == c->kappa, LQCD_EINVAL, "gmresdr_solve: deflation space of another kappa");
    }
    LQCD_CHECK(p.proj_m >= 0 && p.proj_m <= 250, LQCD_EINVAL, "gmresdr_solve: proj_m outside 0..250");
    const int p_cyc = p.proj_m > 0 ? p.proj_m : p.m - p.k;
    const int blk = std::max(1, p.rhs_block);
    for (int r0 = start; r0 < nrhs; r0 += blk) {
      const int nb = std::min(blk, nrhs - r0);
      const cx<double> *bl = static_cast<const cx<double> *>(b) + size_t(r0) * fl;
      cx<double> *xl = static_cast<cx<double> *>(x) + size_t(r0) * fl;
      make_source(c, op, bl, nb, w, n);
      std::vector<double> ref;
      full_norms(c, w, nb, ref);
      std::vector<int> mv(nb, 0), cy(nb, 0), refn(nb, 0), ro(nb, 0);
      std::vector<double> res(nb, 0);
      void *X = w.X.ensure(n * nb * sizeof(cx<double>));
      void *Rr = w.R.ensure(n * nb * sizeof(cx<double>));
      if (p.inner == LQCD_F64) {
        void *W = w.W.ensure(size_t(p_cyc + 1) * n * nb * sizeof(cx<double>));
        proj_solve<double>(c, A64, d->V.ptr, d, p_cyc, w.S.ptr, X, Rr, W, nb, ref, p.tol,
                           p.max_cycles, mv, cy, res, ro);
      } else {
        // FP64 refinement around FP32 deflated inner solves
        {
          std::lock_guard<std::mutex> lk(d->fill_mu);
          if (!d->have_v32) {
            d->V32.ensure(size_t(d->k + 1) * n * sizeof(cx<float>));
            convert<double, float>(c, d->V.ptr, d->V32.ptr, size_t(d->k + 1) * n);
            LQCD_HIP(hipStreamSynchronize(c->stream));
            d->have_v32 = true;
          }
        }
        void *S32 = w.S32.ensure(n * nb * sizeof(cx<float>));
        void *X32 = w.X32.ensure(n * nb * sizeof(cx<float>));
        void *R32 = w.R32.ensure(n * nb * sizeof(cx<float>));
        const bool h16 = p.inner == LQCD_F16 || p.inner == LQCD_BF16;
        void *W32 = h16 ? w.W32.ensure(size_t(p_cyc + 1) * hvec_words(n / 12) * nb * sizeof(uint32_t))
                        : w.W32.ensure(size_t(p_cyc + 1) * n * nb * sizeof(cx<float>));
        // FP32 work vectors of the 16-bit Arnoldi steps (two per right-hand
        // side in the two-step form)
        void *WT = h16 ? w.WT.ensure(n * nb * sizeof(cx<float>) * size_t(c->arnoldi_steps)) : nullptr;
        void *T = w.T.ensure(n * nb * sizeof(cx<double>));
        fill_zero(c, X, n * nb * sizeof(cx<double>));
        copy_dev(c, Rr, w.S.ptr, n * nb * sizeof(cx<double>));
        Small s(c->small[1]);
        s.setup(1, nb, 1);
        std::vector<double> rn(nb);
        int outer_it = 0;
        for (;;) {
          norm2<double>(c, Rr, n, n, nb, s.nrm2);
          d2h(c, rn.data(), s.nrm2, nb * sizeof(double));
          bool all = true;
          int maxc = 0;
          for (int r = 0; r < nb; ++r) {
            rn[r] = std::sqrt(rn[r]);
            LQCD_CHECK(std::isfinite(rn[r]), LQCD_ENAN, "gmresdr_solve: NaN/Inf residual");
            res[r] = rn[r] / ref[r];
            if (rn[r] > p.tol * ref[r]) all = false;
            maxc = std::max(maxc, cy[r]);
          }
          if (all || maxc >= p.max_cycles) break;
          if (++outer_it > kMaxRefinements) break;
          // inner solve for the correction of every rhs not yet converged;
          // converged ones get a zero right-hand side (skipped at once).
          convert<double, float>(c, Rr, S32, n * nb);
          // an inner solve stops at itol times its residual, or as soon as
          // it is below a quarter of the outer target, whichever is larger:
          // the last refinement step then does not solve past tol
          const double itol = std::max(p.inner_tol, 1e-6);
          std::vector<double> iref(nb);
          for (int r = 0; r < nb; ++r)
            iref[r] = (rn[r] > p.tol * ref[r]) ? std::max(rn[r], 0.25 * p.tol * ref[r] / itol) : 0.0;
          std::vector<double> ires(nb);
          if (p.inner == LQCD_F16)
            proj_solve<float, 0>(c, A32, d->V32.ptr, d, p_cyc, S32, X32, R32, W32, nb, iref, itol,
                                 p.max_cycles, mv, cy, ires, ro, kInnerCycleCap, kInnerStall, WT);
          else if (p.inner == LQCD_BF16)
            proj_solve<float, 1>(c, A32, d->V32.ptr, d, p_cyc, S32, X32, R32, W32, nb, iref, itol,
                                 p.max_cycles, mv, cy, ires, ro, kInnerCycleCap, kInnerStall, WT);
          else
            proj_solve<float>(c, A32, d->V32.ptr, d, p_cyc, S32, X32, R32, W32, nb, iref, itol,
                              p.max_cycles, mv, cy, ires, ro, kInnerCycleCap, kInnerStall);
          hipLaunchKernelGGL(k_acc_widen, dim3(std::min<size_t>(nblocks(n * nb), 8192)), dim3(kBlock),
                             0, c->stream, static_cast<const cx<float> *>(X32), static_cast<cx<double> *>(X),
                             n * nb);
          LQCD_HIP(hipGetLastError());
          A64.apply(X, n, T, n, nb);
          cdouble one(1, 0), mone(-1, 0);
          copy_dev(c, Rr, w.S.ptr, n * nb * sizeof(cx<double>));
          axpby<double>(c, &mone, T, n, &one, Rr, n, n, nb, false);
          for (int r = 0; r < nb; ++r) {
            refn[r] += 1;
            mv[r] += 1;
          }
        }
      }
      finish(c, op, X, xl, nb, w, n, tr);
      for (int r = 0; r < nb; ++r) {
        if (stats) stats[r0 + r] = lqcd_solve_stats{mv[r], cy[r], refn[r], ro[r], tr[r]};
        if (res[r] > p.tol) nonconv = true;
      }
    }
    LQCD_CHECK(!nonconv, LQCD_ENOCONV, "gmresdr_solve: a right-hand side missed tol within max_cycles");
  });
}

extern "C" lqcd_status lqcd_defl_eigpairs(lqcd_ctx *c, lqcd_defl *d, int Q, double *lambda_host,
                                          double *resid_host) {
  return guarded([&] {
    LQCD_CHECK(c && d && lambda_host, LQCD_EINVAL, "lqcd_defl_eigpairs: null argument");
    defl_eigpairs(c, d, Q);
    for (int q = 0; q < Q; ++q) {
      lambda_host[q] = d->lam[q];
      if (resid_host) resid_host[q] = d->lam_resid[q];
    }
  });
}

extern "C" lqcd_status lqcd_defl_ritz(const lqcd_defl *d, double *theta_host, int *k_out) {
  return guarded([&] {
    LQCD_CHECK(d && theta_host && k_out, LQCD_EINVAL, "lqcd_defl_ritz: null argument");
    *k_out = int(d->theta.size());
    for (size_t i = 0; i < d->theta.size(); ++i) {
      theta_host[2 * i] = d->theta[i].real();
      theta_host[2 * i + 1] = d->theta[i].imag();
    }
  });
}

extern "C" void lqcd_defl_free(lqcd_defl *d) { delete d; }
