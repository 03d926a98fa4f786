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

// Up to kMaxVar subtracted vectors of one set of solutions are estimated
// together: variant v forms x - xt_v (xt_v null: x itself) with the same
// operations, in the same order, as a pass with that variant alone, so its
// sums equal that pass's bit for bit.  The local kernel reads eta and x once
// for a group of variants; the point-split kernel runs the variants'
// workgroups of one chunk side by side, so that they share eta, x and the
// links through the L2.
constexpr int kMaxVar = 6;
struct XtSet {
  const cx<double> *p[kMaxVar];
  int slot[kMaxVar];  // the point-split kernel: output slot of each variant
};

// Each timeslice is split over nch workgroups (blockIdx.x = t * nch + ch)
// so the launch fills the chip; partial sums of variant v0 + v go to
// out[(((v * nrhs + r) * kNumOps + op) * Lt + t) * nch + ch] (re, im) and
// the host adds the chunks in a fixed order.
template <int NV>
__global__ void __launch_bounds__(kBlock)
    k_estimate(const cx<double> *__restrict__ eta, const cx<double> *__restrict__ x, XtSet xts, int v0,
               size_t V, int Vs, int Lt, int nch, double *__restrict__ out) {
  __shared__ double sh[NV * 2 * kNumTheta][kWaves];
  const int t = blockIdx.x / nch, ch = blockIdx.x % nch, r = blockIdx.y, nrhs = gridDim.y;
  const size_t base = (size_t(r) * V + size_t(t) * Vs) * 12;
  double acc[NV][2 * kNumTheta] = {};
  // lane = (site, colour c): it loads the four spins of colour c of eta, x
  // and each xt_v (loads of 16 bytes, three lanes cover a site's 192-byte
  // block) and forms every Theta's terms from registers, since each Theta
  // only permutes spins (with a phase) at fixed colour
  const size_t ne = size_t(Vs) * 3;
  for (size_t e = size_t(ch) * kBlock + threadIdx.x; e < ne; e += size_t(nch) * kBlock) {
    const size_t s0 = base + e / 3 * 12 + e % 3;  // (site, spin 0, colour c)
    cx<double> a[4], xs[4];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
      a[sp] = ldc(eta + s0 + 3 * sp);
      xs[sp] = ldc(x + s0 + 3 * sp);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const cx<double> *xt = xts.p[v];
      cx<double> d[4];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) d[sp] = xs[sp];
      if (xt)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) d[sp] = d[sp] - ldc(xt + s0 + 3 * sp);
#pragma unroll
      for (int th = 0; th < kNumTheta; ++th)
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
          const cx<double> w = cmulc(a[sp], mk(kGamma[th].re[sp], kGamma[th].im[sp]) * d[kGamma[th].col[sp]]);
          acc[v][2 * th] += w.re;
          acc[v][2 * th + 1] += w.im;
        }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int k = 0; k < 2 * kNumTheta; ++k) acc[v][k] = wave_sum(acc[v][k]);
  if (lane == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int k = 0; k < 2 * kNumTheta; ++k) sh[v * 2 * kNumTheta + k][wave] = acc[v][k];
  __syncthreads();
  if (threadIdx.x < NV * 2 * kNumTheta) {
    double sum = 0;
    for (int w = 0; w < kWaves; ++w) sum += sh[threadIdx.x][w];
    const int v = threadIdx.x / (2 * kNumTheta), k = threadIdx.x % (2 * kNumTheta);
    const int th = k / 2, part = k % 2;
    out[((((size_t(v0 + v) * nrhs + r) * kNumOps + th) * Lt + t) * nch + ch) * 2 + part] = sum;
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
// phase alpha_s in {+-1, +-i}.
//
// A workgroup takes 64 consecutive sites of one timeslice at a time.  The
// fields are site-major (192 bytes per site), so it first stages them in
// LDS with coalesced 16-byte loads (consecutive lanes read consecutive
// pieces of consecutive sites): eta at its sites once, then for each
// direction d = x - xt at the sites' forward and backward neighbours
// (whose site runs are contiguous but for the wrap of the periodic
// boundary).  LDS holds them component-major, [12][64 sites] with a row
// stride of 65, so that a wave reading one component of 64 sites, and
// a wave writing 12 components of consecutive sites, touch distinct banks
// in every group of 8 lanes.  Then wave q of the workgroup takes one of the
// four halves for all 64 sites (lane = site): q < 2 the forward half spin
// s = q (W = U_mu(x)), q >= 2 the backward one s = q - 2 (W = U_mu(x -
// mu)^+); the branch is uniform per wave and the link loads are coalesced.
constexpr int kPsSites = 64;                // sites per chunk
constexpr int kPsRow = kPsSites + 1;        // LDS stride of one component
constexpr int kPsArr = 12 * kPsRow;         // one staged field

// Link U_mu at the site of full lexicographic index s and parity par, in
// the even/odd layout [parity][mu][9][Vh].
__device__ inline const cx<double> *ps_link_at(const cx<double> *U, size_t Vh, size_t s, int par, int mu) {
  return U + ((size_t(par) * 4 + mu) * 9) * Vh + (s >> 1);
}

// Half spin HS of the direction-mu term at a lane's site: FWD with U_mu(x)
// and d(x + mu), else U_mu(x - mu)^+ and d(x - mu).  ea and db point at the
// site's column of the staged eta and d (components kPsRow apart); u is
// the link (entries Vh apart).
template <int MU, bool FWD, int HS>
__device__ inline cx<double> ps_half_spin(const cx<double> *u, size_t Vh, const cx<double> *ea,
                                          const cx<double> *db) {
  // partner spin and phase of the forward projector (negated backward)
  constexpr int PS = MU < 2 ? 3 - HS : 2 + HS;
  constexpr double AR0 = MU == 1 ? (HS ? -1.0 : 1.0) : MU == 3 ? -1.0 : 0.0;
  constexpr double AI0 = MU == 0 ? 1.0 : MU == 2 ? (HS ? -1.0 : 1.0) : 0.0;
  constexpr double AR = FWD ? AR0 : -AR0, AI = FWD ? AI0 : -AI0;
  // at_k = a_HS,k + alpha a_PS,k with alpha in {+-1, +-i} (and likewise h)
  auto proj = [](cx<double> p, cx<double> q) {
    return AR != 0.0 ? mk(p.re + AR * q.re, p.im + AR * q.im) : mk(p.re - AI * q.im, p.im + AI * q.re);
  };
  cx<double> at[3], h[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    at[k] = proj(ea[(HS * 3 + k) * kPsRow], ea[(PS * 3 + k) * kPsRow]);
    h[k] = proj(db[(HS * 3 + k) * kPsRow], db[(PS * 3 + k) * kPsRow]);
  }
  // the link loads go out after the projections (fewer registers live)
  asm volatile("" : "+v"(at[0].re), "+v"(at[0].im), "+v"(at[1].re), "+v"(at[1].im), "+v"(at[2].re),
               "+v"(at[2].im), "+v"(h[0].re), "+v"(h[0].im), "+v"(h[1].re), "+v"(h[1].im), "+v"(h[2].re),
               "+v"(h[2].im)::"memory");
  cx<double> acc = mk(0.0, 0.0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<double> w[3];  // row a of W
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const cx<double> e = ldc(u + (FWD ? 3 * a + b : 3 * b + a) * Vh);
      w[b] = FWD ? e : mk(e.re, -e.im);
    }
    acc = acc + cmulc(at[a], w[0] * h[0] + w[1] * h[1] + w[2] * h[2]);
  }
  return acc;
}

// Stage 64 sites' worth of x - xt (XT) or of x into LDS: piece p = 12 site
// + k is complex k of the spinor at full site index idx[site] (-1: a site
// past the end, zero; it loads site 0 and drops it, so that the loads of
// all pieces go out together).
template <bool XT>
__device__ inline void ps_stage(cx<double> *sh, const cx<double> *x, const cx<double> *xt, const int *idx) {
  cx<double> v[3];
  bool ok[3];
  int at[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int p = threadIdx.x + u * kBlock;
    const int site = p / 12, k = p - 12 * site;
    const int s = idx[site];
    ok[u] = s >= 0;
    const size_t o = size_t(ok[u] ? s : 0) * 12 + k;
    v[u] = ldc(x + o);
    if (XT) v[u] = v[u] - ldc(xt + o);
    at[u] = k * kPsRow + site;
  }
#pragma unroll
  for (int u = 0; u < 3; ++u) sh[at[u]] = ok[u] ? v[u] : mk(0.0, 0.0);
}

template <int MU, bool XT>
__device__ inline void ps_dir(const cx<double> *U, size_t Vh, double kappa, const cx<double> *x,
                              const cx<double> *xt, const int (*nb)[kPsSites], const cx<double> *eS,
                              cx<double> *fS, cx<double> *bS, size_t s, int par, bool on, double &re,
                              double &im) {
  __syncthreads();  // the previous direction's reads of fS, bS are done
  ps_stage<XT>(fS, x, xt, nb[2 * MU]);
  asm volatile("" ::: "memory");  // the backward loads after the forward ones (fewer registers live)
  ps_stage<XT>(bS, x, xt, nb[2 * MU + 1]);
  __syncthreads();
  if (on) {
    const int site = threadIdx.x & 63;
    const int q = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const cx<double> *uf = ps_link_at(U, Vh, s, par, MU);
    const cx<double> *ub = ps_link_at(U, Vh, size_t(nb[2 * MU + 1][site]), par ^ 1, MU);
    cx<double> v;
    if (q == 0) v = -kappa * ps_half_spin<MU, true, 0>(uf, Vh, eS + site, fS + site);
    else if (q == 1) v = -kappa * ps_half_spin<MU, true, 1>(uf, Vh, eS + site, fS + site);
    else if (q == 2) v = kappa * ps_half_spin<MU, false, 0>(ub, Vh, eS + site, bS + site);
    else v = kappa * ps_half_spin<MU, false, 1>(ub, Vh, eS + site, bS + site);
    re += v.re;
    im += v.im;
  }
}

// Workgroup order: the variant varies fastest, then the right-hand side,
// within one XCD's contiguous range of logical workgroups (hardware
// workgroup h runs on XCD h % 8), so the nv workgroups of one chunk of one
// right-hand side run side by side on one XCD and read its eta and x from
// that XCD's L2, and the nv * nrhs workgroups of one chunk its links (links
// are as many bytes as one right-hand side's three fields).  Each workgroup
// is the estimator of its variant alone.
template <bool XT>
__global__ void __launch_bounds__(kBlock)
    k_estimate_ps(Geom g, const cx<double> *__restrict__ U, double kappa,
                  const cx<double> *__restrict__ eta, const cx<double> *__restrict__ x, XtSet xts, int nv,
                  int nch, int nrhs, int xq, double *__restrict__ out) {
  __shared__ double sh[2 * kNumPS][kWaves];
  __shared__ cx<double> eS[kPsArr], fS[kPsArr], bS[kPsArr];
  __shared__ int nb[2 * kNumPS + 1][kPsSites];  // neighbour site indices [2 mu + backward]; the sites
  const int L = int(blockIdx.x % 8) * xq + int(blockIdx.x / 8);
  if (L >= g.L[3] * nch * nrhs * nv) return;  // whole workgroup: padding of the grid
  const int var = L % nv, r = (L / nv) % nrhs, tch = L / (nv * nrhs);
  const cx<double> *__restrict__ xt = xts.p[var];
  const int t = tch / nch, ch = tch % nch;
  const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
  const int Vs = Lx * Ly * Lz;
  const size_t Vh = size_t(g.Vh);
  const size_t base = size_t(r) * size_t(g.V) * 12;
  eta += base;
  x += base;
  if (XT) xt += base;
  double acc[2 * kNumPS] = {};
  for (int i0 = ch * kPsSites; i0 < Vs; i0 += nch * kPsSites) {
    const int site = threadIdx.x & 63;
    const int i = i0 + site;
    const bool on = i < Vs;
    const int c[4] = {i % Lx, (i / Lx) % Ly, i / (Lx * Ly), t};
    const size_t s = size_t(t) * Vs + i;
    const int par = (c[0] + c[1] + c[2] + t) & 1;
    __syncthreads();  // the previous chunk's reads of eS and nb are done
    {
      // wave q: the forward and backward neighbours of the sites along mu = q
      const int q = threadIdx.x >> 6;
      const int st = q == 0 ? 1 : q == 1 ? Lx : q == 2 ? Lx * Ly : Vs;
      const int Lm = g.L[q], cm = c[q];
      nb[2 * q][site] = on ? int(cm + 1 == Lm ? s - size_t(st) * (Lm - 1) : s + st) : -1;
      nb[2 * q + 1][site] = on ? int(cm == 0 ? s + size_t(st) * (Lm - 1) : s - st) : -1;
      if (q == 0) nb[2 * kNumPS][site] = on ? int(s) : -1;
    }
    __syncthreads();
    ps_stage<false>(eS, eta, static_cast<const cx<double> *>(nullptr), nb[2 * kNumPS]);
    ps_dir<0, XT>(U, Vh, kappa, x, xt, nb, eS, fS, bS, s, par, on, acc[0], acc[1]);
    ps_dir<1, XT>(U, Vh, kappa, x, xt, nb, eS, fS, bS, s, par, on, acc[2], acc[3]);
    ps_dir<2, XT>(U, Vh, kappa, x, xt, nb, eS, fS, bS, s, par, on, acc[4], acc[5]);
    ps_dir<3, XT>(U, Vh, kappa, x, xt, nb, eS, fS, bS, s, par, on, acc[6], acc[7]);
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
    out[((((size_t(xts.slot[var]) * nrhs + r) * kNumOps + kNumTheta + m) * Lt + t) * nch + ch) * 2 + part] = v;
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

// Variants per launch of the local kernel (its per-lane sums grow by 10
// doubles per variant).
constexpr int kLocalGroup = 3;

template <int NV>
void launch_local(lqcd_ctx *c, const void *eta, const void *x, const XtSet &xts, int v0, int nrhs, double *d,
                  int nch) {
  const Geom &g = c->g;
  const int Lt = g.L[3], Vs = g.V / Lt;
  hipLaunchKernelGGL(k_estimate<NV>, dim3(Lt * nch, nrhs), dim3(kBlock), 0, c->stream,
                     static_cast<const cx<double> *>(eta), static_cast<const cx<double> *>(x), xts, v0, size_t(g.V),
                     Vs, Lt, nch, d);
  LQCD_HIP(hipGetLastError());
}

// The point-split kernel over the n variants of xts, all with (XT) or all
// without a subtracted vector.
template <bool XT>
void launch_ps(lqcd_ctx *c, const void *eta, const void *x, const XtSet &xts, int n, int nrhs, double *d,
               int nch) {
  const Geom &g = c->g;
  const int Lt = g.L[3];
  const int xq = (Lt * nch * nrhs * n + 7) / 8;  // logical workgroups per XCD (grid padded to 8 xq)
  hipLaunchKernelGGL(k_estimate_ps<XT>, dim3(8 * xq), dim3(kBlock), 0, c->stream, g,
                     static_cast<const cx<double> *>(c->U64.ptr), c->kappa, static_cast<const cx<double> *>(eta),
                     static_cast<const cx<double> *>(x), xts, n, nch, nrhs, xq, d);
  LQCD_HIP(hipGetLastError());
}

// Launch KERNEL<n> over the variants [v0, v0 + n) for n <= 6.
#define LQCD_EST_DISPATCH(KERNEL, n, ...)                  \
  switch (n) {                                             \
    case 1: KERNEL<1>(__VA_ARGS__); break;                 \
    case 2: KERNEL<2>(__VA_ARGS__); break;                 \
    case 3: KERNEL<3>(__VA_ARGS__); break;                 \
    case 4: KERNEL<4>(__VA_ARGS__); break;                 \
    case 5: KERNEL<5>(__VA_ARGS__); break;                 \
    default: KERNEL<6>(__VA_ARGS__); break;                \
  }

// The estimator of nvar variants (subtracted vectors xt[v], corrections
// corr[v]) with its partial sums in d (at least nvar * nrhs * kNumOps * Lt
// * nch * 2 doubles of device memory).  Variant v's outputs start at
// est + v * nth * (Lt + 1) * 2, stderr_ + (same), samples + v * nrhs * nth
// * (Lt + 1) * 2.
void estimate_with(lqcd_ctx *c, const int *thetas, int nth, const void *eta, const void *x,
                   const void *const *xt, int nvar, int nrhs, const double *const *corr, double *est,
                   double *stderr_, double *samples, double *d, int nch) {
  bool any_local = false, any_ps = false;
  for (int a = 0; a < nth; ++a) (thetas[a] < kNumTheta ? any_local : any_ps) = true;
  auto group = [&](int v0, int n) {
    XtSet xts{};
    for (int v = 0; v < n; ++v) xts.p[v] = static_cast<const cx<double> *>(xt[v0 + v]);
    return xts;
  };
  if (any_local)
    for (int v0 = 0; v0 < nvar; v0 += kLocalGroup) {
      const int n = std::min(kLocalGroup, nvar - v0);
      LQCD_EST_DISPATCH(launch_local, n, c, eta, x, group(v0, n), v0, nrhs, d, nch)
    }
  if (any_ps)
    // one launch over the variants with a subtracted vector, one over those
    // without
    for (int with = 0; with < 2; ++with) {
      int n = 0;
      XtSet xts{};
      for (int v = 0; v < nvar; ++v)
        if ((xt[v] != nullptr) == bool(with)) {
          xts.p[n] = static_cast<const cx<double> *>(xt[v]);
          xts.slot[n++] = v;
        }
      if (!n) continue;
      if (with) launch_ps<true>(c, eta, x, xts, n, nrhs, d, nch);
      else launch_ps<false>(c, eta, x, xts, n, nrhs, d, nch);
    }

  const int Lt = c->g.L[3];
  std::vector<double> hc(size_t(nvar) * nrhs * kNumOps * Lt * nch * 2);
  LQCD_HIP(hipMemcpyAsync(hc.data(), d, hc.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LQCD_HIP(hipStreamSynchronize(c->stream));
  const int W = Lt + 1;
  for (int var = 0; var < nvar; ++var) {
    const double *hv = hc.data() + size_t(var) * nrhs * kNumOps * Lt * nch * 2;
    const double *cv = corr ? corr[var] : nullptr;
    double *ev = est + size_t(var) * nth * W * 2, *sv = stderr_ + size_t(var) * nth * W * 2;
    std::vector<double> h(size_t(nrhs) * kNumOps * Lt * 2, 0.0);
    for (size_t o = 0; o < h.size() / 2; ++o)
      for (int ch = 0; ch < nch; ++ch) {
        h[2 * o] += hv[(o * nch + ch) * 2];
        h[2 * o + 1] += hv[(o * nch + ch) * 2 + 1];
      }
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
        if (cv) {
          if (t < Lt) {
            cr = cdouble(cv[2 * (a * Lt + t)], cv[2 * (a * Lt + t) + 1]);
          } else {
            for (int s = 0; s < Lt; ++s) cr += cdouble(cv[2 * (a * Lt + s)], cv[2 * (a * Lt + s) + 1]);
          }
        }
        cdouble e = mean + cr;
        ev[2 * (a * W + t)] = e.real();
        ev[2 * (a * W + t) + 1] = e.imag();
        sv[2 * (a * W + t)] = ser;
        sv[2 * (a * W + t) + 1] = sei;
      }
    if (samples) {
      double *pv = samples + size_t(var) * nrhs * nth * W * 2;
      for (size_t i = 0; i < smp.size(); ++i) {
        pv[2 * i] = smp[i].real();
        pv[2 * i + 1] = smp[i].imag();
      }
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
    estimate_with(c, thetas, nth, eta, x, &xt, 1, nrhs, &corr, est, stderr_, samples, d, nch);
  });
}

extern "C" lqcd_status loop_estimate_multi(lqcd_ctx *c, const int *thetas, int nth, const void *eta,
                                           const void *x, const void *const *xt_list, int nvar, int nrhs,
                                           const double *const *corr_list, double *est, double *stderr_,
                                           double *samples) {
  return guarded([&] {
    check_args(c, thetas, nth, eta, x, nrhs, est, stderr_, "loop_estimate_multi");
    LQCD_CHECK(xt_list && nvar >= 1 && nvar <= kMaxVar, LQCD_EINVAL,
               "loop_estimate_multi: %d variants (1..%d, with a list of subtracted vectors)", nvar, kMaxVar);
    const int nch = estimate_chunks(c->g, nrhs, 0);
    double *d = static_cast<double *>(
        c->red.ensure(size_t(nvar) * nrhs * kNumOps * c->g.L[3] * nch * 2 * sizeof(double)));
    estimate_with(c, thetas, nth, eta, x, xt_list, nvar, nrhs, corr_list, est, stderr_, samples, d, nch);
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
    estimate_with(c, thetas, nth, eta, x, &xt, 1, nrhs, &corr, est, stderr_, samples, d, nch);
  });
}
