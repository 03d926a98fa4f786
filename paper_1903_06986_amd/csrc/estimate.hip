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
    out[((size_t(r) * kNumTheta + th) * Lt + t) * 2 + part] = s;
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
      LQCD_CHECK(thetas[a] >= 0 && thetas[a] < kNumTheta, LQCD_EINVAL, "theta code %d outside 0..4",
                 thetas[a]);
    const Geom &g = c->g;
    const int Lt = g.L[3], Vs = g.V / Lt;
    double *d = static_cast<double *>(c->red.ensure(size_t(nrhs) * kNumTheta * Lt * 2 * sizeof(double)));
    hipLaunchKernelGGL(k_estimate, dim3(Lt, nrhs), dim3(kBlock), 0, c->stream,
                       static_cast<const cx<double> *>(eta), static_cast<const cx<double> *>(x),
                       static_cast<const cx<double> *>(xt), size_t(g.V), Vs, Lt, d);
    LQCD_HIP(hipGetLastError());
    std::vector<double> h(size_t(nrhs) * kNumTheta * Lt * 2);
    LQCD_HIP(hipMemcpyAsync(h.data(), d, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LQCD_HIP(hipStreamSynchronize(c->stream));
    const int W = Lt + 1;
    // samples [n][a][t], t = Lt the total
    std::vector<cdouble> smp(size_t(nrhs) * nth * W);
    for (int n = 0; n < nrhs; ++n)
      for (int a = 0; a < nth; ++a) {
        cdouble tot = 0;
        for (int t = 0; t < Lt; ++t) {
          size_t o = ((size_t(n) * kNumTheta + thetas[a]) * Lt + t) * 2;
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
