// The subtracted trace estimator (Sec. 5 Eq. (23); Sec. 6):
//   t_n[Theta][t] = sum_{x in timeslice t} eta_n(x)^+ Theta (x_n - xt_n)(x)
//   est[Theta][t] = (1/N) sum_n t_n[Theta][t] + Tr_t(Theta tilde-M^{-1})
// One pass over eta, x and xt per (timeslice, right-hand side) block; the
// lexicographic layout keeps each timeslice contiguous.  Standard errors are
// s / sqrt(N) with the unbiased sample variance, for Re and Im separately.
#include <cmath>
#include <mutex>

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
  // lane = (site, colour c): it loads the four spins of colour c of eta, x
  // and xt (12 loads of 16 bytes, three lanes cover a site's 192-byte block)
  // and forms every Theta's terms from registers, since each Theta only
  // permutes spins (with a phase) at fixed colour
  const size_t ne = size_t(Vs) * 3;
  for (size_t e = size_t(ch) * kBlock + threadIdx.x; e < ne; e += size_t(nch) * kBlock) {
    const size_t s0 = base + e / 3 * 12 + e % 3;  // (site, spin 0, colour c)
    cx<double> a[4], d[4];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
      a[sp] = ldc(eta + s0 + 3 * sp);
      d[sp] = ldc(x + s0 + 3 * sp);
    }
    if (xt)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) d[sp] = d[sp] - ldc(xt + s0 + 3 * sp);
#pragma unroll
    for (int th = 0; th < kNumTheta; ++th)
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        const cx<double> v = cmulc(a[sp], mk(kGamma[th].re[sp], kGamma[th].im[sp]) * d[kGamma[th].col[sp]]);
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
// (Theta(mu) (x_n - xt_n))(x), Theta(mu) = kappa [(1 + g_mu) U_mu(x - mu)^+
// S_- - (1 - g_mu) U_mu(x) S_+] with S_-+ the shifts to x -+ mu.
//
// (1 -+ g_mu) has rank 2 and squares to twice itself, and its lower half
// spinor is a unitary R times the upper one, so for any colour matrix W
//   a^+ (1 -+ g_mu) W b = sum_{s=0,1} at_s^+ W h_s,
// where at and h are the upper halves of (1 -+ g_mu) a and (1 -+ g_mu) b:
// at_s = a_s + alpha_s a_{p(s)} with a spin partner p(s) in {2, 3} and a
// phase alpha_s in {+-1, +-i}.  Each site gets 4 lanes: lane q < 2 takes the
// forward half spin s = q (W = U_mu(x), neighbour x + mu), lane q >= 2 the
// backward one s = q - 2 (W = U_mu(x - mu)^+, neighbour x - mu).  A lane
// loads two spins of eta(x), two spins of x and xt at its neighbour and one
// link, so 16 sites of a wave read contiguous 3 KiB runs.  The lanes' terms
// add up over the four lanes of a site; each timeslice is split over nch
// workgroups as in k_estimate.
template <int MU>
__device__ inline cx<double> ps_lane(const cx<double> *U, const Geom &g, double kappa,
                                     const cx<double> *eta, const cx<double> *x, const cx<double> *xt,
                                     const int c[4], size_t s, int q) {
  const int Lm = g.L[MU];
  const size_t stm = MU == 0 ? 1 : MU == 1 ? size_t(g.L[0]) : MU == 2 ? size_t(g.L[0]) * g.L[1]
                                                                        : size_t(g.L[0]) * g.L[1] * g.L[2];
  const bool fwd = q < 2;
  const int hs = q & 1;  // half spin
  const int cm = c[MU];
  const size_t nbr = fwd ? (cm + 1 == Lm ? s - stm * (Lm - 1) : s + stm) : (cm == 0 ? s + stm * (Lm - 1) : s - stm);
  int cl[4] = {c[0], c[1], c[2], c[3]};
  if (!fwd) cl[MU] = cm == 0 ? Lm - 1 : cm - 1;  // the backward link lives at x - mu
  const cx<double> *u = ps_link(U, g, cl[0], cl[1], cl[2], cl[3], MU);
  // partner spin and phase of the forward projector (negated backward)
  const int ps = MU < 2 ? 3 - hs : 2 + hs;
  double ar, ai;
  if (MU == 0) { ar = 0; ai = 1; }
  else if (MU == 1) { ar = hs ? -1 : 1; ai = 0; }
  else if (MU == 2) { ar = 0; ai = hs ? -1 : 1; }
  else { ar = -1; ai = 0; }
  if (!fwd) { ar = -ar; ai = -ai; }
  const cx<double> al = mk(ar, ai);
  cx<double> at[3], h[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    at[k] = ldc(eta + s * 12 + hs * 3 + k) + al * ldc(eta + s * 12 + ps * 3 + k);
    cx<double> bu = ldc(x + nbr * 12 + hs * 3 + k), bl = ldc(x + nbr * 12 + ps * 3 + k);
    if (xt) {
      bu = bu - ldc(xt + nbr * 12 + hs * 3 + k);
      bl = bl - ldc(xt + nbr * 12 + ps * 3 + k);
    }
    h[k] = bu + al * bl;
  }
  // the link loads go out after the projections (fewer registers live)
  asm volatile("" : "+v"(at[0].re), "+v"(at[0].im), "+v"(at[1].re), "+v"(at[1].im), "+v"(at[2].re),
               "+v"(at[2].im), "+v"(h[0].re), "+v"(h[0].im), "+v"(h[1].re), "+v"(h[1].im), "+v"(h[2].re),
               "+v"(h[2].im)::"memory");
  const size_t Vh = size_t(g.Vh);
  cx<double> acc = mk(0.0, 0.0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // row a of W: U_ab forward, conj(U_ba) backward
    cx<double> w[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const cx<double> e = ldc(u + (fwd ? 3 * a + b : 3 * b + a) * Vh);
      w[b] = fwd ? e : mk(e.re, -e.im);
    }
    acc = acc + cmulc(at[a], w[0] * h[0] + w[1] * h[1] + w[2] * h[2]);
  }
  return (fwd ? -kappa : kappa) * acc;
}

// Workgroup order: the right-hand side varies fastest within one XCD's
// contiguous range of logical workgroups (hardware workgroup h runs on XCD
// h % 8), so the nrhs workgroups of one chunk of sites run back to back on
// one XCD and read its links from that XCD's L2 (links are as many bytes as
// one right-hand side's three fields).
__global__ void __launch_bounds__(kBlock)
    k_estimate_ps(Geom g, const cx<double> *__restrict__ U, double kappa,
                  const cx<double> *__restrict__ eta, const cx<double> *__restrict__ x,
                  const cx<double> *__restrict__ xt, int nch, int nrhs, int xq, double *__restrict__ out) {
  __shared__ double sh[2 * kNumPS][kWaves];
  const int L = int(blockIdx.x % 8) * xq + int(blockIdx.x / 8);
  if (L >= g.L[3] * nch * nrhs) return;  // whole workgroup: padding of the grid
  const int r = L % nrhs, tch = L / nrhs;
  const int t = tch / nch, ch = tch % nch;
  const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
  const int Vs = Lx * Ly * Lz;
  const size_t base = size_t(r) * size_t(g.V) * 12;
  eta += base;
  x += base;
  if (xt) xt += base;
  const int q = threadIdx.x & 3;
  double acc[2 * kNumPS] = {};
  for (int i = ch * (kBlock / 4) + (threadIdx.x >> 2); i < Vs; i += nch * (kBlock / 4)) {
    const int c[4] = {i % Lx, (i / Lx) % Ly, i / (Lx * Ly), t};
    const size_t s = size_t(t) * Vs + i;
    // one direction at a time: the empty asm (with a memory clobber) keeps
    // the next direction's loads behind this direction's arithmetic, which
    // would otherwise all be issued at once and fill the register file
    cx<double> v;
    v = ps_lane<0>(U, g, kappa, eta, x, xt, c, s, q);
    acc[0] += v.re;
    acc[1] += v.im;
    asm volatile("" : "+v"(acc[0]), "+v"(acc[1])::"memory");
    v = ps_lane<1>(U, g, kappa, eta, x, xt, c, s, q);
    acc[2] += v.re;
    acc[3] += v.im;
    asm volatile("" : "+v"(acc[2]), "+v"(acc[3])::"memory");
    v = ps_lane<2>(U, g, kappa, eta, x, xt, c, s, q);
    acc[4] += v.re;
    acc[5] += v.im;
    asm volatile("" : "+v"(acc[4]), "+v"(acc[5])::"memory");
    v = ps_lane<3>(U, g, kappa, eta, x, xt, c, s, q);
    acc[6] += v.re;
    acc[7] += v.im;
    asm volatile("" : "+v"(acc[6]), "+v"(acc[7])::"memory");
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
    const int m = threadIdx.x / 2, part = threadIdx.x % 2;
    out[(((size_t(r) * kNumOps + kNumTheta + m) * Lt + t) * nch + ch) * 2 + part] = v;
  }
}

// Scratch of the allocation-free entry point loop_estimate_noalloc: the
// per-workgroup partial sums, in a fixed device array (one copy per GPU,
// held until the process ends).  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocDoubles = size_t(1) << 19;  // 4 MiB
static __device__ __align__(256) double scratch[kNoallocDoubles];

constexpr int kMaxDevices = 64;
std::mutex noalloc_mu;
double *noalloc_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device, looked up on
// the first call there.
double *noalloc_scratch() {
  int dev = 0;
  LQCD_HIP(hipGetDevice(&dev));
  LQCD_CHECK(dev >= 0 && dev < kMaxDevices, LQCD_EDEVICE, "loop_estimate_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void *p = nullptr;
    LQCD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    noalloc_ptr[dev] = static_cast<double *>(p);
  }
  return noalloc_ptr[dev];
}

// Chunks per timeslice: about 2048 workgroups in all, at least one site
// block each, and at most cap_doubles of partial sums (0: no cap).
int estimate_chunks(const Geom &g, int nrhs, size_t cap_doubles) {
  const int Lt = g.L[3], Vs = g.V / Lt;
  int nch = std::max(1, std::min((Vs + kBlock / 4 - 1) / (kBlock / 4), (2048 + Lt * nrhs - 1) / (Lt * nrhs)));
  if (cap_doubles)
    nch = std::max(1, std::min<int>(nch, int(cap_doubles / (size_t(nrhs) * kNumOps * Lt * 2))));
  return nch;
}

// The estimator with its partial sums in d (at least
// nrhs * kNumOps * Lt * nch * 2 doubles of device memory).
void estimate_with(lqcd_ctx *c, const int *thetas, int nth, const void *eta, const void *x, const void *xt,
                   int nrhs, const double *corr, double *est, double *stderr_, double *samples, double *d,
                   int nch) {
  {
    bool any_local = false, any_ps = false;
    for (int a = 0; a < nth; ++a) (thetas[a] < kNumTheta ? any_local : any_ps) = true;
    const Geom &g = c->g;
    const int Lt = g.L[3], Vs = g.V / Lt;
    if (any_local) {
      hipLaunchKernelGGL(k_estimate, dim3(Lt * nch, nrhs), dim3(kBlock), 0, c->stream,
                         static_cast<const cx<double> *>(eta), static_cast<const cx<double> *>(x),
                         static_cast<const cx<double> *>(xt), size_t(g.V), Vs, Lt, nch, d);
      LQCD_HIP(hipGetLastError());
    }
    if (any_ps) {
      const int xq = (Lt * nch * nrhs + 7) / 8;  // logical workgroups per XCD (grid padded to 8 xq)
      hipLaunchKernelGGL(k_estimate_ps, dim3(8 * xq), dim3(kBlock), 0, c->stream, g,
                         static_cast<const cx<double> *>(c->U64.ptr), c->kappa,
                         static_cast<const cx<double> *>(eta), static_cast<const cx<double> *>(x),
                         static_cast<const cx<double> *>(xt), nch, nrhs, xq, d);
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
  }
}

void check_args(lqcd_ctx *c, const int *thetas, int nth, const void *eta, const void *x, int nrhs,
                const double *est, const double *stderr_, const char *who) {
  LQCD_CHECK(c && eta && x && est && stderr_, LQCD_EINVAL, "%s: null argument", who);
  LQCD_CHECK(nrhs >= 1, LQCD_EINVAL, "%s: need at least one noise vector", who);
  LQCD_CHECK(nth >= 1 && thetas, LQCD_EINVAL, "%s: no operator", who);
  for (int a = 0; a < nth; ++a)
    LQCD_CHECK(thetas[a] >= 0 && thetas[a] < kNumOps, LQCD_EINVAL, "%s: operator code %d outside 0..8", who,
               thetas[a]);
}

}  // namespace
}  // namespace lqcd

using namespace lqcd;

extern "C" lqcd_status loop_estimate(lqcd_ctx *c, const int *thetas, int nth, const void *eta,
                                     const void *x, const void *xt, int nrhs, const double *corr,
                                     double *est, double *stderr_, double *samples) {
  return guarded([&] {
    check_args(c, thetas, nth, eta, x, nrhs, est, stderr_, "loop_estimate");
    const int nch = estimate_chunks(c->g, nrhs, 0);
    double *d = static_cast<double *>(
        c->red.ensure(size_t(nrhs) * kNumOps * c->g.L[3] * nch * 2 * sizeof(double)));
    estimate_with(c, thetas, nth, eta, x, xt, nrhs, corr, est, stderr_, samples, d, nch);
  });
}

extern "C" lqcd_status loop_estimate_noalloc(lqcd_ctx *c, const int *thetas, int nth, const void *eta,
                                             const void *x, const void *xt, int nrhs, const double *corr,
                                             double *est, double *stderr_, double *samples) {
  return guarded([&] {
    check_args(c, thetas, nth, eta, x, nrhs, est, stderr_, "loop_estimate_noalloc");
    const size_t one = size_t(nrhs) * kNumOps * c->g.L[3] * 2;
    LQCD_CHECK(one <= kNoallocDoubles, LQCD_EINVAL,
               "loop_estimate_noalloc: %d right-hand sides x %d timeslices need %zu partial sums, more than "
               "the fixed scratch of %zu (use loop_estimate)",
               nrhs, c->g.L[3], one, kNoallocDoubles);
    double *d = noalloc_scratch();
    const int nch = estimate_chunks(c->g, nrhs, kNoallocDoubles);
    estimate_with(c, thetas, nth, eta, x, xt, nrhs, corr, est, stderr_, samples, d, nch);
  });
}
