// Derivatives of the trace estimate in kappa and in the links.
//
// The stochastic estimate of Tr(Theta M^{-1}) with fixed noise is
// T = (1/N) sum_n eta_n^+ Theta M^{-1} eta_n, M = 1 - kappa P (Sec. 5.1
// Eqs. (24)-(25)).  With dM^{-1} = M^{-1} (dM) ... M^{-1} and the
// g5-hermiticity M^+ = g5 M g5 (Sec. 5.4), every derivative is a bilinear
// in x_n = M^{-1} eta_n and the adjoint vector
//   y_n = (M^{-1})^+ Theta^+ eta_n = g5 M^{-1} g5 Theta^+ eta_n:
//   dT/dkappa = (1/N) sum_n y_n^+ P x_n,
//   dT/dw^a(x, mu) = (kappa/N) sum_n i tr[T^a (U F1 - F2 U^+)]
// for the left rotation U_mu(x) -> exp(i w^a T^a) U_mu(x) (T^a = lambda^a/2),
// with colour outer products over spin
//   F1_ab = sum_s ((1 - g_mu) x(x+mu))_{s a} conj(y(x)_{s b}),
//   F2_ab = sum_s ((1 + g_mu) x(x))_{s a} conj(y(x+mu)_{s b}).
// Because (1 -+ g_mu) has rank 2 (the half-spinor form of the stencil),
// sum over four spins of ((1 - g_mu) a)_s conj(b_s) equals the sum over the
// two spins of the projected halves h(a)_s conj(h(b)_s), so each F is a sum
// of two 3x3 outer products.  The same traces give the kappa derivative:
// y^+ P x = sum over links of tr[U F1] + tr[U^+ F2].
//
// The force kernel reads LEX complex128 fields (site-major, 12 components
// per site), one thread per (site, direction) with the direction fastest,
// so the four threads of a site share its loads; it loops over the noise
// vectors in registers and writes each link's 8 generator components once.
#include <cmath>
#include <memory>

#include "cplx.h"
#include "gamma.h"
#include "fields.h"

namespace lqcd {
namespace {

struct Spin4 {
  double re[4][4], im[4][4];
};

// out_n(x) = A in_n(x) in spin space (A a 4x4 complex matrix per theta and
// timeslice: A[t]), colour untouched.  LEX fields.
__global__ void __launch_bounds__(kBlock)
    k_spin_mat(const cx<double> *__restrict__ in, cx<double> *__restrict__ out,
               const Spin4 *__restrict__ A, size_t V, int Vs, int nrhs) {
  const size_t s = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= V) return;
  const Spin4 &a = A[s / Vs];
  for (int r = 0; r < nrhs; ++r) {
    const size_t o = (size_t(r) * V + s) * 12;
    cx<double> v[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = ldc(in + o + k);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cx<double> acc = mk(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc = acc + mk(a.re[sp][t], a.im[sp][t]) * v[t * 3 + c];
        stc(out + o + sp * 3 + c, acc);
      }
  }
}

// Half spinor of (1 - g_mu) psi (FWD) or (1 + g_mu) psi (BWD), spins 0/1,
// for the chiral basis: h = u + i s_k l / u - i s_k l; t: h = u -+ l.
// G5 negates the lower spins of psi first (psi -> g5 psi).
template <bool FWD, bool G5>
__device__ inline void half_proj(int mu, const cx<double> p[12], cx<double> h[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<double> u0 = p[c], u1 = p[3 + c];
    cx<double> l0 = p[6 + c], l1 = p[9 + c];
    if (G5) {
      l0 = -l0;
      l1 = -l1;
    }
    cx<double> q0, q1;  // i s_mu l  (t: -l)
    if (mu == 0) {
      q0 = iz(l1);
      q1 = iz(l0);
    } else if (mu == 1) {
      q0 = l1;
      q1 = -l0;
    } else if (mu == 2) {
      q0 = iz(l0);
      q1 = miz(l1);
    } else {
      q0 = -l0;
      q1 = -l1;
    }
    h[0][c] = FWD ? u0 + q0 : u0 - q0;
    h[1][c] = FWD ? u1 + q1 : u1 - q1;
  }
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int kWaves = kBlock / 64;

// One thread per (site s, direction mu), mu = threadIdx.x % 4.
// x: solutions, xa: adjoint solutions x' (y = g5 x'), LEX [nrhs][V][12].
// dlinks: LEX [V][4][8] complex (may be null); part: per-block partial sums
// of sum_n (tr[U F1] + tr[U^+ F2]), 2 doubles per block.
__global__ void __launch_bounds__(kBlock)
    k_force(Geom g, const cx<double> *__restrict__ U, const cx<double> *__restrict__ x,
            const cx<double> *__restrict__ xa, int nrhs, double scale, cx<double> *__restrict__ dlinks,
            double *__restrict__ part) {
  __shared__ double sh[2][kWaves];
  const size_t V = size_t(g.V), Vh = size_t(g.Vh);
  const size_t s = size_t(blockIdx.x) * (kBlock / 4) + threadIdx.x / 4;
  const int mu = threadIdx.x % 4;
  double kre = 0, kim = 0;
  if (s < V) {
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    int c[4];
    c[0] = int(s % Lx);
    size_t r = s / Lx;
    c[1] = int(r % Ly);
    r /= Ly;
    c[2] = int(r % Lz);
    c[3] = int(r / Lz);
    const int Ls[4] = {Lx, Ly, Lz, Lt};
    const size_t stride[4] = {1, size_t(Lx), size_t(Lx) * Ly, size_t(Lx) * Ly * Lz};
    const size_t sp = c[mu] + 1 == Ls[mu] ? s - stride[mu] * (Ls[mu] - 1) : s + stride[mu];
    const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
    // link U_mu(s): even/odd layout [parity][mu][9][Vh], checkerboard index s / 2
    const cx<double> *ul = U + ((size_t(par) * 4 + mu) * 9) * Vh + s / 2;
    cx<double> u[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) u[a][b] = ldc(ul + (3 * a + b) * Vh);

    cx<double> F1[3][3], F2[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) F1[a][b] = F2[a][b] = mk(0.0, 0.0);
    for (int n = 0; n < nrhs; ++n) {
      const cx<double> *xn = x + size_t(n) * V * 12, *yn = xa + size_t(n) * V * 12;
      cx<double> p[12], hx[2][3], hy[2][3];
      // F1: (1 - g_mu) x(s + mu) against (1 - g_mu) y(s)
#pragma unroll
      for (int k = 0; k < 12; ++k) p[k] = ldc(xn + sp * 12 + k);
      half_proj<true, false>(mu, p, hx);
#pragma unroll
      for (int k = 0; k < 12; ++k) p[k] = ldc(yn + s * 12 + k);
      half_proj<true, true>(mu, p, hy);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          F1[a][b] = F1[a][b] + cmulc(hy[0][b], hx[0][a]) + cmulc(hy[1][b], hx[1][a]);
      // F2: (1 + g_mu) x(s) against (1 + g_mu) y(s + mu)
#pragma unroll
      for (int k = 0; k < 12; ++k) p[k] = ldc(xn + s * 12 + k);
      half_proj<false, false>(mu, p, hx);
#pragma unroll
      for (int k = 0; k < 12; ++k) p[k] = ldc(yn + sp * 12 + k);
      half_proj<false, true>(mu, p, hy);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          F2[a][b] = F2[a][b] + cmulc(hy[0][b], hx[0][a]) + cmulc(hy[1][b], hx[1][a]);
    }
    // G = U F1 - F2 U^+;  tr[U F1] + tr[U^+ F2] for the kappa derivative
    cx<double> G[3][3];
    cx<double> tk = mk(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        cx<double> v = mk(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          v = v + u[a][k] * F1[k][b];
          v = v - cmulc(u[b][k], F2[a][k]);  // F2_ak conj(U_bk) = (F2 U^+)_ab
        }
        G[a][b] = v;
        tk = tk + u[a][b] * F1[b][a] + cmulc(u[b][a], F2[b][a]);  // (U^+)_ab F2_ba
      }
    kre = tk.re;
    kim = tk.im;
    if (dlinks) {
      // i tr[T^a G] = (i/2) tr[lambda^a G]
      const double r3 = 0.57735026918962576451;  // 1/sqrt(3)
      cx<double> t[8];
      t[0] = G[1][0] + G[0][1];
      t[1] = iz(G[0][1] - G[1][0]);
      t[2] = G[0][0] - G[1][1];
      t[3] = G[2][0] + G[0][2];
      t[4] = iz(G[0][2] - G[2][0]);
      t[5] = G[2][1] + G[1][2];
      t[6] = iz(G[1][2] - G[2][1]);
      t[7] = r3 * (G[0][0] + G[1][1] - 2.0 * G[2][2]);
      cx<double> *o = dlinks + (s * 4 + mu) * 8;
#pragma unroll
      for (int a = 0; a < 8; ++a) stc(o + a, (0.5 * scale) * iz(t[a]));
    }
  }
  kre = wave_sum(kre);
  kim = wave_sum(kim);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wave] = kre;
    sh[1][wave] = kim;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double v = 0;
    for (int w = 0; w < kWaves; ++w) v += sh[threadIdx.x][w];
    part[2 * size_t(blockIdx.x) + threadIdx.x] = v;
  }
}

}  // namespace
}  // namespace lqcd

using namespace lqcd;

extern "C" lqcd_status loop_gradient(lqcd_ctx *c, const int *thetas, const double *weights,
                                     int nth, const lqcd_solve_params *params,
                                     lqcd_defl **defl_inout, const void *eta, const void *x,
                                     int nrhs, double *dkappa, void *dlinks,
                                     lqcd_solve_stats *stats) {
  return guarded([&] {
    LQCD_CHECK(c && thetas && params && defl_inout && eta && dkappa, LQCD_EINVAL,
               "loop_gradient: null argument");
    LQCD_CHECK(nrhs >= 1, LQCD_EINVAL, "loop_gradient: need at least one noise vector");
    LQCD_CHECK(nth >= 1, LQCD_EINVAL, "loop_gradient: no operator");
    for (int a = 0; a < nth; ++a)
      LQCD_CHECK(thetas[a] >= 0 && thetas[a] < kNumTheta, LQCD_EINVAL,
                 "loop_gradient: theta code %d outside 0..4", thetas[a]);
    const Geom &g = c->g;
    const int Lt = g.L[3], Vs = g.V / Lt;
    const size_t fl = full_len(g);
    // Adjoint source matrices per timeslice: g5 Theta_w^+ with
    // Theta_w = sum_a w[a][t] Theta_a (every Theta_a hermitian).
    std::vector<Spin4> A(Lt);
    for (int t = 0; t < Lt; ++t) {
      std::complex<double> m[4][4] = {};
      for (int a = 0; a < nth; ++a) {
        const cdouble w = weights ? cdouble(weights[2 * (a * Lt + t)], weights[2 * (a * Lt + t) + 1])
                                  : cdouble(1, 0);
        std::complex<double> th[4][4];
        gamma_dense(thetas[a], th);
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) m[i][j] += std::conj(w) * th[i][j];
      }
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          const double sg = i >= 2 ? -1.0 : 1.0;  // g5 on the left
          A[t].re[i][j] = sg * m[i][j].real();
          A[t].im[i][j] = sg * m[i][j].imag();
        }
    }
    // Right-hand sides: [eta (only when x is not given); g5 Theta_w^+ eta].
    const int nsolve = x ? nrhs : 2 * nrhs;
    // context workspaces, grown on first use and kept for later calls
    DevBuf &B = c->grad[0], &X = c->grad[1], &Am = c->grad[2];
    B.ensure(fl * nsolve * sizeof(cdouble));
    X.ensure(fl * nsolve * sizeof(cdouble));
    Am.ensure(Lt * sizeof(Spin4));
    LQCD_HIP(hipMemcpyAsync(Am.ptr, A.data(), Lt * sizeof(Spin4), hipMemcpyHostToDevice, c->stream));
    cx<double> *Bp = B.as<cx<double>>();
    const size_t off = x ? 0 : fl * nrhs;
    if (!x)
      LQCD_HIP(hipMemcpyAsync(Bp, eta, fl * nrhs * sizeof(cdouble), hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(k_spin_mat, dim3(nblocks(g.V)), dim3(kBlock), 0, c->stream,
                       static_cast<const cx<double> *>(eta), Bp + off, Am.as<Spin4>(), size_t(g.V), Vs,
                       nrhs);
    LQCD_HIP(hipGetLastError());
    std::vector<lqcd_solve_stats> st(nsolve);
    lqcd_status rc = gmresdr_solve(c, LQCD_OP_SCHUR, params, Bp, X.ptr, nsolve, defl_inout, st.data());
    if (rc != LQCD_OK) throw Error{rc};  // the solver's message stays in place
    if (stats)
      for (int r = 0; r < nrhs; ++r) stats[r] = st[(x ? 0 : nrhs) + r];
    const cx<double> *Xs = x ? static_cast<const cx<double> *>(x) : X.as<cx<double>>();
    const cx<double> *Xa = X.as<cx<double>>() + off;
    const unsigned nb = nblocks(size_t(g.V), kBlock / 4);
    double *part = static_cast<double *>(c->red.ensure(size_t(nb) * 2 * sizeof(double)));
    {
      // algorithmic bytes: x and x' read once per noise vector, the links
      // once, the force written once
      const double bytes = double(g.V) * (2.0 * nrhs * 192.0 + 4 * 9 * 16.0 + (dlinks ? 4 * 8 * 16.0 : 0.0));
      Timed tm(c, LQCD_KC_FORCE, bytes);
      LQCD_TLAUNCH(tm, true, true, k_force, dim3(nb), dim3(kBlock), 0, c->stream, g,
                         static_cast<const cx<double> *>(c->U64.ptr), Xs, Xa, nrhs,
                         c->kappa / nrhs, static_cast<cx<double> *>(dlinks), part);
      LQCD_HIP(hipGetLastError());
    }
    std::vector<double> h(size_t(nb) * 2);
    LQCD_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LQCD_HIP(hipStreamSynchronize(c->stream));
    double re = 0, im = 0;
    for (unsigned b = 0; b < nb; ++b) {
      re += h[2 * b];
      im += h[2 * b + 1];
    }
    dkappa[0] = re / nrhs;
    dkappa[1] = im / nrhs;
  });
}
