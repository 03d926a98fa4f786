// The subtracted trace estimator (Sec. 5 Eq. (23); Sec. 6):
//   t_n[Theta][t] = sum_{x in timeslice t} eta_n(x)^+ Theta (x_n - xt_n)(x)
//   est[Theta][t] = (1/N) sum_n t_n[Theta][t] + Tr_t(Theta tilde-M^{-1})
// One pass over eta, x and xt per (timeslice, right-hand side) block; the
// lexicographic layout keeps each timeslice contiguous.  Standard errors are
// s / sqrt(N) with the unbiased sample variance, for Re and Im separately.
#include <cmath>

#include "cplx.h"
#include "gamma.h"
#include "fields.h"
#include "pointsplit.h"

namespace lqcd {
namespace {

constexpr int kWaves = kBlock / 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(kBlock)
    k_estimate(const cx<double> *__restrict__ eta, const cx<double> *__restrict__ x,
               const cx<double> *__restrict__ xt, size_t V, int Vs, int Lt,
               double *__restrict__ out) {
  __shared__ double sh[2 * kNumTheta][kWaves];
  const int t = blockIdx.x, r = blockIdx.y;
  const size_t base = (size_t(r) * V + size_t(t) * Vs) * 12;
  double acc[2 * kNumTheta] = {};
  for (int i = threadIdx.x; i < Vs; i += kBlock) {
    const size_t o = base + size_t(i) * 12;
    cx<double> e[12], d[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      e[k] = ldc(eta + o + k);
      d[k] = ldc(x + o + k);
      if (xt) d[k] = d[k] - ldc(xt + o + k);
    }
#pragma unroll
    for (int th = 0; th < kNumTheta; ++th) {
      cx<double> s = mk(0.0, 0.0);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        const int col = kGamma[th].col[sp];
        const cx<double> v = mk(kGamma[th].re[sp], kGamma[th].im[sp]);
#pragma unroll
        for (int c = 0; c < 3; ++c) s = s + cmulc(e[sp * 3 + c], v * d[col * 3 + c]);
      }
      acc[2 * th] += s.re;
      acc[2 * th + 1] += s.im;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 2 * kNumTheta; ++k) acc[k] = wave_sum(acc[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 2 * kNumTheta; ++k) sh[k][wave] = acc[k];
  __syncthreads();
  if (threadIdx.x < 2 * kNumTheta) {
    double s = 0;
    for (int w = 0; w < kWaves; ++w) s += sh[threadIdx.x][w];
    const int th = threadIdx.x / 2, part = threadIdx.x % 2;
    out[((size_t(r) * kNumOps + th) * Lt + t) * 2 + part] = s;
  }
}

// Point-split operators (codes 5..8): t_n[mu][t] = sum_{x in t} eta_n(x)^+
// (Theta(mu) (x_n - xt_n))(x); one block per (timeslice, right-hand side).
__global__ void __launch_bounds__(kBlock)
    k_estimate_ps(Geom g, const cx<double> *__restrict__ U, double kappa,
                  const cx<double> *__restrict__ eta, const cx<double> *__restrict__ x,
                  const cx<double> *__restrict__ xt, double *__restrict__ out) {
  __shared__ double sh[2 * kNumPS][kWaves];
  const int t = blockIdx.x, r = blockIdx.y;
  const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
  const int Vs = Lx * Ly * Lz;
  const size_t V = size_t(g.V), Vh = size_t(g.Vh);
  const size_t base = size_t(r) * V * 12;
  double acc[2 * kNumPS] = {};
  for (int i = threadIdx.x; i < Vs; i += kBlock) {
    const int xx = i % Lx, yy = (i / Lx) % Ly, zz = i / (Lx * Ly);
    const size_t s = size_t(t) * Vs + i;
    cx<double> a[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = ldc(eta + base + s * 12 + k);
    const int c[4] = {xx, yy, zz, t};
    const int Ls[4] = {Lx, Ly, Lz, Lt};
    const size_t st[4] = {1, size_t(Lx), size_t(Lx) * Ly, size_t(Lx) * Ly * Lz};
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      const size_t sf = c[mu] + 1 == Ls[mu] ? s - st[mu] * (Ls[mu] - 1) : s + st[mu];
      const size_t sb = c[mu] == 0 ? s + st[mu] * (Ls[mu] - 1) : s - st[mu];
      int cb[4] = {c[0], c[1], c[2], c[3]};
      cb[mu] = c[mu] == 0 ? Ls[mu] - 1 : c[mu] - 1;
      cx<double> b[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        b[k] = ldc(x + base + sf * 12 + k);
        if (xt) b[k] = b[k] - ldc(xt + base + sf * 12 + k);
      }
      const cx<double> vf = ps_half<true>(a, b, ps_link(U, g, c[0], c[1], c[2], c[3], mu), Vh, mu);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        b[k] = ldc(x + base + sb * 12 + k);
        if (xt) b[k] = b[k] - ldc(xt + base + sb * 12 + k);
      }
      const cx<double> vb = ps_half<false>(a, b, ps_link(U, g, cb[0], cb[1], cb[2], cb[3], mu), Vh, mu);
      const cx<double> v = kappa * (vb - vf);
      // (mu is a runtime index: accumulate through a small switch-free select)
#pragma unroll
      for (int m = 0; m < 4; ++m)
        if (m == mu) {
          acc[2 * m] += v.re;
          acc[2 * m + 1] += v.im;
        }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 2 * kNumPS; ++k) acc[k] = wave_sum(acc[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 2 * kNumPS; ++k) sh[k][wave] = acc[k];
  __syncthreads();
  if (threadIdx.x < 2 * kNumPS) {
    double v = 0;
    for (int w = 0; w < kWaves; ++w) v += sh[threadIdx.x][w];
    const int mu = threadIdx.x / 2, part = threadIdx.x % 2;
    out[((size_t(r) * kNumOps + kNumTheta + mu) * Lt + t) * 2 + part] = v;
  }
}

}  // namespace
}  // namespace lqcd

using namespace lqcd;

extern "C" lqcd_status loop_estimate(lqcd_ctx *c, const int *thetas, int nth, const void *eta,
                                     const void *x, const void *xt, int nrhs, const double *corr,
                                     double *est, double *stderr_, double *samples) {
  return guarded([&] {
    LQCD_CHECK(c && eta && x && est && stderr_, LQCD_EINVAL, "loop_estimate: null argument");
    LQCD_CHECK(nrhs >= 1, LQCD_EINVAL, "loop_estimate: need at least one noise vector");
    LQCD_CHECK(nth >= 1 && thetas, LQCD_EINVAL, "loop_estimate: no operator");
    for (int a = 0; a < nth; ++a)
      LQCD_CHECK(thetas[a] >= 0 && thetas[a] < kNumOps, LQCD_EINVAL, "operator code %d outside 0..8",
                 thetas[a]);
    bool any_local = false, any_ps = false;
    for (int a = 0; a < nth; ++a) (thetas[a] < kNumTheta ? any_local : any_ps) = true;
    const Geom &g = c->g;
    const int Lt = g.L[3], Vs = g.V / Lt;
    double *d = static_cast<double *>(c->red.ensure(size_t(nrhs) * kNumOps * Lt * 2 * sizeof(double)));
    if (any_local) {
      hipLaunchKernelGGL(k_estimate, dim3(Lt, nrhs), dim3(kBlock), 0, c->stream,
                         static_cast<const cx<double> *>(eta), static_cast<const cx<double> *>(x),
                         static_cast<const cx<double> *>(xt), size_t(g.V), Vs, Lt, d);
      LQCD_HIP(hipGetLastError());
    }
    if (any_ps) {
      hipLaunchKernelGGL(k_estimate_ps, dim3(Lt, nrhs), dim3(kBlock), 0, c->stream, g,
                         static_cast<const cx<double> *>(c->U64.ptr), c->kappa,
                         static_cast<const cx<double> *>(eta), static_cast<const cx<double> *>(x),
                         static_cast<const cx<double> *>(xt), d);
      LQCD_HIP(hipGetLastError());
    }
    std::vector<double> h(size_t(nrhs) * kNumOps * Lt * 2);
    LQCD_HIP(hipMemcpyAsync(h.data(), d, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LQCD_HIP(hipStreamSynchronize(c->stream));
    const int W = Lt + 1;
    // samples [n][a][t], t = Lt the total
    std::vector<cdouble> smp(size_t(nrhs) * nth * W);
    for (int n = 0; n < nrhs; ++n)
      for (int a = 0; a < nth; ++a) {
        cdouble tot = 0;
        for (int t = 0; t < Lt; ++t) {
          size_t o = ((size_t(n) * kNumOps + thetas[a]) * Lt + t) * 2;
          cdouble v(h[o], h[o + 1]);
          smp[(size_t(n) * nth + a) * W + t] = v;
          tot += v;
        }
        smp[(size_t(n) * nth + a) * W + Lt] = tot;
      }
    for (int a = 0; a < nth; ++a)
      for (int t = 0; t < W; ++t) {
        cdouble mean = 0;
        for (int n = 0; n < nrhs; ++n) mean += smp[(size_t(n) * nth + a) * W + t];
        mean /= double(nrhs);
        double vr = 0, vi = 0;
        for (int n = 0; n < nrhs; ++n) {
          cdouble dv = smp[(size_t(n) * nth + a) * W + t] - mean;
          vr += dv.real() * dv.real();
          vi += dv.imag() * dv.imag();
        }
        double ser = 0, sei = 0;
        if (nrhs > 1) {
          ser = std::sqrt(vr / (nrhs - 1) / nrhs);
          sei = std::sqrt(vi / (nrhs - 1) / nrhs);
        }
        cdouble cr = 0;
        if (corr) {
          if (t < Lt) {
            cr = cdouble(corr[2 * (a * Lt + t)], corr[2 * (a * Lt + t) + 1]);
          } else {
            for (int s = 0; s < Lt; ++s) cr += cdouble(corr[2 * (a * Lt + s)], corr[2 * (a * Lt + s) + 1]);
          }
        }
        cdouble e = mean + cr;
        est[2 * (a * W + t)] = e.real();
        est[2 * (a * W + t) + 1] = e.imag();
        stderr_[2 * (a * W + t)] = ser;
        stderr_[2 * (a * W + t) + 1] = sei;
      }
    if (samples)
      for (size_t i = 0; i < smp.size(); ++i) {
        samples[2 * i] = smp[i].real();
        samples[2 * i + 1] = smp[i].imag();
      }
  });
}
