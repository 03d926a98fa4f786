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

// Each timeslice is split over nch workgroups (blockIdx.x = t * nch + ch)
// so the launch fills the chip; partial sums go to
// out[((r * kNumOps + op) * Lt + t) * nch + ch] (re, im) and the host adds
// the chunks in a fixed order.
__global__ void __launch_bounds__(kBlock)
    k_estimate(const cx<double> *__restrict__ eta, const cx<double> *__restrict__ x,
               const cx<double> *__restrict__ xt, size_t V, int Vs, int Lt, int nch,
               double *__restrict__ out) {
  __shared__ double sh[2 * kNumTheta][kWaves];
  const int t = blockIdx.x / nch, ch = blockIdx.x % nch, r = blockIdx.y;
  const size_t base = (size_t(r) * V + size_t(t) * Vs) * 12;
  double acc[2 * kNumTheta] = {};
  // element-parallel: lane e handles component (spin sp, colour c) of one
  // site, so consecutive lanes read consecutive complex numbers; the spin
  // partners Theta needs (sp, 3 - sp, sp ^ 2 in this basis) lie in the same
  // 192-byte site block
  const size_t ne = size_t(Vs) * 12;
  for (size_t e = size_t(ch) * kBlock + threadIdx.x; e < ne; e += size_t(nch) * kBlock) {
    const size_t site0 = base + e / 12 * 12;
    const int k = int(e % 12), sp = k / 3, c = k % 3;
    const cx<double> a = ldc(eta + base + e);
    auto dval = [&](int col) {
      cx<double> v = ldc(x + site0 + col * 3 + c);
      if (xt) v = v - ldc(xt + site0 + col * 3 + c);
      return v;
    };
    const cx<double> d0 = dval(sp), d1 = dval(3 - sp), d2 = dval(sp ^ 2);
#pragma unroll
    for (int th = 0; th < kNumTheta; ++th) {
      const int col = kGamma[th].col[sp];
      const cx<double> dv = col == sp ? d0 : (col == 3 - sp ? d1 : d2);
      const cx<double> v = cmulc(a, mk(kGamma[th].re[sp], kGamma[th].im[sp]) * dv);
      acc[2 * th] += v.re;
      acc[2 * th + 1] += v.im;
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
    out[(((size_t(r) * kNumOps + th) * Lt + t) * nch + ch) * 2 + part] = s;
  }
}

// Point-split operators (codes 5..8): t_n[mu][t] = sum_{x in t} eta_n(x)^+
// (Theta(mu) (x_n - xt_n))(x).  One thread per (site, direction), the
// direction fastest, so the four threads of a site share its loads; each
// timeslice is split over nch workgroups as above.
__global__ void __launch_bounds__(kBlock)
    k_estimate_ps(Geom g, const cx<double> *__restrict__ U, double kappa,
                  const cx<double> *__restrict__ eta, const cx<double> *__restrict__ x,
                  const cx<double> *__restrict__ xt, int nch, double *__restrict__ out) {
  __shared__ double sh[2 * kNumPS][kWaves];
  const int t = blockIdx.x / nch, ch = blockIdx.x % nch, r = blockIdx.y;
  const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
  const int Vs = Lx * Ly * Lz;
  const size_t V = size_t(g.V), Vh = size_t(g.Vh);
  const size_t base = size_t(r) * V * 12;
  const int mu = threadIdx.x & 3;
  double are = 0, aim = 0;
  for (int i = ch * (kBlock / 4) + (threadIdx.x >> 2); i < Vs; i += nch * (kBlock / 4)) {
    const int xx = i % Lx, yy = (i / Lx) % Ly, zz = i / (Lx * Ly);
    const size_t s = size_t(t) * Vs + i;
    const int cm = mu == 0 ? xx : mu == 1 ? yy : mu == 2 ? zz : t;
    const int Lm = mu == 0 ? Lx : mu == 1 ? Ly : mu == 2 ? Lz : Lt;
    const size_t stm = mu == 0 ? 1 : mu == 1 ? size_t(Lx) : mu == 2 ? size_t(Lx) * Ly : size_t(Lx) * Ly * Lz;
    const size_t sf = cm + 1 == Lm ? s - stm * (Lm - 1) : s + stm;
    const size_t sb = cm == 0 ? s + stm * (Lm - 1) : s - stm;
    const int cb = cm == 0 ? Lm - 1 : cm - 1;
    cx<double> a[12], b[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = ldc(eta + base + s * 12 + k);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      b[k] = ldc(x + base + sf * 12 + k);
      if (xt) b[k] = b[k] - ldc(xt + base + sf * 12 + k);
    }
    const cx<double> vf = ps_half<true>(a, b, ps_link(U, g, xx, yy, zz, t, mu), Vh, mu);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      b[k] = ldc(x + base + sb * 12 + k);
      if (xt) b[k] = b[k] - ldc(xt + base + sb * 12 + k);
    }
    const cx<double> *ub = ps_link(U, g, mu == 0 ? cb : xx, mu == 1 ? cb : yy, mu == 2 ? cb : zz, mu == 3 ? cb : t, mu);
    const cx<double> vb = ps_half<false>(a, b, ub, Vh, mu);
    are += kappa * (vb.re - vf.re);
    aim += kappa * (vb.im - vf.im);
  }
  // reduce the four directions separately: lanes with the same mu
#pragma unroll
  for (int off = 32; off >= 4; off >>= 1) {
    are += __shfl_xor(are, off, 64);
    aim += __shfl_xor(aim, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane < 4) {
    sh[2 * lane][wave] = are;
    sh[2 * lane + 1][wave] = aim;
  }
  __syncthreads();
  if (threadIdx.x < 2 * kNumPS) {
    double v = 0;
    for (int w = 0; w < kWaves; ++w) v += sh[threadIdx.x][w];
    const int m = threadIdx.x / 2, part = threadIdx.x % 2;
    out[(((size_t(r) * kNumOps + kNumTheta + m) * Lt + t) * nch + ch) * 2 + part] = v;
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
    // chunks per timeslice: about 2048 workgroups in all, at least one site
    // block each
    const int nch = std::max(1, std::min((Vs + kBlock / 4 - 1) / (kBlock / 4), (2048 + Lt * nrhs - 1) / (Lt * nrhs)));
    double *d = static_cast<double *>(
        c->red.ensure(size_t(nrhs) * kNumOps * Lt * nch * 2 * sizeof(double)));
    if (any_local) {
      hipLaunchKernelGGL(k_estimate, dim3(Lt * nch, nrhs), dim3(kBlock), 0, c->stream,
                         static_cast<const cx<double> *>(eta), static_cast<const cx<double> *>(x),
                         static_cast<const cx<double> *>(xt), size_t(g.V), Vs, Lt, nch, d);
      LQCD_HIP(hipGetLastError());
    }
    if (any_ps) {
      hipLaunchKernelGGL(k_estimate_ps, dim3(Lt * nch, nrhs), dim3(kBlock), 0, c->stream, g,
                         static_cast<const cx<double> *>(c->U64.ptr), c->kappa,
                         static_cast<const cx<double> *>(eta), static_cast<const cx<double> *>(x),
                         static_cast<const cx<double> *>(xt), nch, d);
      LQCD_HIP(hipGetLastError());
    }
    std::vector<double> hc(size_t(nrhs) * kNumOps * Lt * nch * 2);
    LQCD_HIP(hipMemcpyAsync(hc.data(), d, hc.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LQCD_HIP(hipStreamSynchronize(c->stream));
    std::vector<double> h(size_t(nrhs) * kNumOps * Lt * 2, 0.0);
    for (size_t o = 0; o < h.size() / 2; ++o)
      for (int ch = 0; ch < nch; ++ch) {
        h[2 * o] += hc[(o * nch + ch) * 2];
        h[2 * o + 1] += hc[(o * nch + ch) * 2 + 1];
      }
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
