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
// sums equal that pass's bit for bit.  Both kernels read eta and x once for
// a group of variants (the point-split kernel also its neighbours' eta and
// the links).
constexpr int kMaxVar = 6;
// Partial-sum slots per (variant, right-hand side, timeslice, chunk): the
// nine operator codes, with code 8 (point-split in t) in two slots, 8 and
// 9, for its terms whose row site lies one timeslice below and above the
// site the kernel works on.
constexpr int kOpSlots = kNumOps + 1;
struct XtSet {
  const cx<double> *p[kMaxVar];
};

// Each timeslice is split over nch workgroups (blockIdx.x = t * nch + ch)
// so the launch fills the chip; partial sums of variant v0 + v go to
// out[(((v * nrhs + r) * kOpSlots + op) * Lt + t) * nch + ch] (re, im) and
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
    out[((((size_t(v0 + v) * nrhs + r) * kOpSlots + th) * Lt + t) * nch + ch) * 2 + part] = sum;
  }
}

// Point-split operators (codes 5..8): t_n[mu][t] = sum_{x in t} eta_n(x)^+
// (Theta(mu) (x_n - xt_n))(x), Theta(mu) = kappa [(1 + g_mu) U_mu(x - mu)^+
// S_- - (1 - g_mu) U_mu(x) S_+] with S_-+ the shifts to x -+ mu.
//
// (1 -+ g_mu) has rank 2 and squares to twice itself, and its lower half
// spinor is a unitary R times the upper one, so for any colour matrix W
//   a^+ (1 -+ g_mu) W b = sum_{s=0,1} at_s^+ W h_s = sum_s (W^+ at_s)^+ h_s,
// where at and h are the upper halves of (1 -+ g_mu) a and (1 -+ g_mu) b:
// at_s = a_s + alpha_s a_{p(s)} with a spin partner p(s) in {2, 3} and a
// phase alpha_s in {+-1, +-i}.
//
// The sums are taken over the site y that d = x - xt is read at: the
// forward term of row x = y - mu is -kappa (U_mu(y - mu)^+ at)^+ h with at
// from eta(y - mu), the backward term of row x = y + mu is kappa (U_mu(y)
// at)^+ h with at from eta(y + mu), both with h from d(y).  So eta is read at
// the neighbours and d only at y: the colour vectors c = W^+ at of a site
// (one per direction and half spin) do not depend on d, and every variant
// adds a dot product of three per direction and half spin.  A term belongs
// to the timeslice of its row site, which for mu = t is the one below (the
// forward terms) or above (the backward terms) y's.
//
// A workgroup takes 64 consecutive sites of one timeslice at a time.  The
// fields are site-major (192 bytes per site), so it stages them in LDS with
// coalesced 16-byte loads (consecutive lanes read consecutive pieces of
// consecutive sites): for each direction eta at the sites' forward and
// backward neighbours (whose site runs are contiguous but for the wrap of
// the periodic boundary), then for each variant d at the sites.  LDS holds
// them component-major, [12][64 sites] with a row stride of 65, so that a
// wave reading one component of 64 sites, and a wave writing 12 components
// of consecutive sites, touch distinct banks in every group of 8 lanes.
// Wave q of the workgroup takes one of the four half spins for all 64 sites
// (lane = site): q < 2 the forward one s = q, q >= 2 the backward one s = q
// - 2; the branch is uniform per wave and the link loads are coalesced.
constexpr int kPsSites = 64;                // sites per chunk
constexpr int kPsRow = kPsSites + 1;        // LDS stride of one component
constexpr int kPsArr = 12 * kPsRow;         // one staged field

// Link U_mu at the site of full lexicographic index s and parity par, in
// the even/odd layout [parity][mu][9][Vh].
__device__ inline const cx<double> *ps_link_at(const cx<double> *U, size_t Vh, size_t s, int par, int mu) {
  return U + ((size_t(par) * 4 + mu) * 9) * Vh + (s >> 1);
}

// Half spin HS of direction MU, forward (FWD: projector 1 - g_mu) or
// backward (1 + g_mu).
template <int MU, bool FWD, int HS>
struct PsHalf {
  // partner spin and phase of the forward projector (negated backward)
  static constexpr int PS = MU < 2 ? 3 - HS : 2 + HS;
  static constexpr double AR0 = MU == 1 ? (HS ? -1.0 : 1.0) : MU == 3 ? -1.0 : 0.0;
  static constexpr double AI0 = MU == 0 ? 1.0 : MU == 2 ? (HS ? -1.0 : 1.0) : 0.0;
  static constexpr double AR = FWD ? AR0 : -AR0, AI = FWD ? AI0 : -AI0;
  // p + alpha q with alpha in {+-1, +-i}
  __device__ static cx<double> proj(cx<double> p, cx<double> q) {
    return AR != 0.0 ? mk(p.re + AR * q.re, p.im + AR * q.im) : mk(p.re - AI * q.im, p.im + AI * q.re);
  }
  // c = W^+ at for the staged eta column ea (components kPsRow apart) and
  // the link u (entries Vh apart): W = U_mu(y - mu) (FWD), U_mu(y)^+ (else)
  __device__ static void eta_side(const cx<double> *u, size_t Vh, const cx<double> *ea, cx<double> c[3]) {
    cx<double> at[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) at[k] = proj(ea[(HS * 3 + k) * kPsRow], ea[(PS * 3 + k) * kPsRow]);
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = mk(0.0, 0.0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<double> e[3];  // row a of U (one row in flight: fewer registers live)
#pragma unroll
      for (int b = 0; b < 3; ++b) e[b] = ldc(u + (3 * a + b) * Vh);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (FWD) c[b] = c[b] + cmulc(e[b], at[a]);  // (U^+ at)_b = sum_a conj(U_ab) at_a
        else c[a] = c[a] + e[b] * at[b];            // (U at)_a = sum_b U_ab at_b
      }
      asm volatile("" : "+v"(c[0].re), "+v"(c[0].im), "+v"(c[1].re), "+v"(c[1].im), "+v"(c[2].re),
                   "+v"(c[2].im)::"memory");
    }
  }
  // c^+ h for the staged d column db
  __device__ static cx<double> term(const cx<double> c[3], const cx<double> *db) {
    cx<double> acc = mk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) acc = acc + cmulc(c[k], proj(db[(HS * 3 + k) * kPsRow], db[(PS * 3 + k) * kPsRow]));
    return acc;
  }
};

// Stage 64 sites' worth of f - g (g null: f) into LDS: piece p = 12 site +
// k is complex k of the spinor at full site index idx[site] (-1: a site
// past the end, zero; it loads site 0 and drops it, so that the loads of
// all pieces go out together).
__device__ inline void ps_stage(cx<double> *sh, const cx<double> *f, const cx<double> *g, const int *idx) {
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
    v[u] = ldc(f + o);
    if (g) v[u] = v[u] - ldc(g + o);
    at[u] = k * kPsRow + site;
  }
#pragma unroll
  for (int u = 0; u < 3; ++u) sh[at[u]] = ok[u] ? v[u] : mk(0.0, 0.0);
}

// Wave q's colour vector of direction MU at its lane's site: eta at y + mu
// in fS, at y - mu in bS.
template <int MU>
__device__ inline void ps_eta_side(const cx<double> *U, size_t Vh, const int (*nb)[kPsSites],
                                   const cx<double> *fS, const cx<double> *bS, size_t s, int par, int q,
                                   cx<double> c[3]) {
  const int site = threadIdx.x & 63;
  if (q < 2) {
    const cx<double> *u = ps_link_at(U, Vh, size_t(nb[2 * MU + 1][site]), par ^ 1, MU);  // U_mu(y - mu)
    if (q == 0) PsHalf<MU, true, 0>::eta_side(u, Vh, bS + site, c);
    else PsHalf<MU, true, 1>::eta_side(u, Vh, bS + site, c);
  } else {
    const cx<double> *u = ps_link_at(U, Vh, s, par, MU);  // U_mu(y)
    if (q == 2) PsHalf<MU, false, 0>::eta_side(u, Vh, fS + site, c);
    else PsHalf<MU, false, 1>::eta_side(u, Vh, fS + site, c);
  }
}

template <int MU>
__device__ inline cx<double> ps_term(const cx<double> c[3], const cx<double> *dS, int q, double kappa) {
  const int site = threadIdx.x & 63;
  if (q == 0) return -kappa * PsHalf<MU, true, 0>::term(c, dS + site);
  if (q == 1) return -kappa * PsHalf<MU, true, 1>::term(c, dS + site);
  if (q == 2) return kappa * PsHalf<MU, false, 0>::term(c, dS + site);
  return kappa * PsHalf<MU, false, 1>::term(c, dS + site);
}

// Workgroup order: the right-hand side varies fastest within one XCD's
// contiguous range of logical workgroups (hardware workgroup h runs on XCD
// h % 8), so the nrhs workgroups of one chunk of sites run back to back on
// one XCD and read its links from that XCD's L2 (links are as many bytes as
// one right-hand side's three fields).  Variant v of the launch is variant
// v0 + v of the call.
template <int NV>
__global__ void __launch_bounds__(kBlock)
    k_estimate_ps(Geom g, const cx<double> *__restrict__ U, double kappa,
                  const cx<double> *__restrict__ eta, const cx<double> *__restrict__ x, XtSet xts, int v0,
                  int nch, int nrhs, int xq, double *__restrict__ out) {
  __shared__ double sh[NV * 2 * kNumPS][kWaves];
  __shared__ cx<double> fS[kPsArr], bS[kPsArr], dS[kPsArr];
  __shared__ int nb[2 * kNumPS + 1][kPsSites];  // neighbour site indices [2 mu + backward]; the sites
  const int L = int(blockIdx.x % 8) * xq + int(blockIdx.x / 8);
  if (L >= g.L[3] * nch * nrhs) return;  // whole workgroup: padding of the grid
  const int r = L % nrhs, tch = L / nrhs;
  const int t = tch / nch, ch = tch % nch;
  const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
  const int Vs = Lx * Ly * Lz;
  const size_t Vh = size_t(g.Vh);
  const size_t base = size_t(r) * size_t(g.V) * 12;
  eta += base;
  x += base;
#pragma unroll
  for (int v = 0; v < NV; ++v)
    if (xts.p[v]) xts.p[v] += base;
  const int q = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  double acc[NV][2 * kNumPS] = {};
  for (int i0 = ch * kPsSites; i0 < Vs; i0 += nch * kPsSites) {
    const int site = threadIdx.x & 63;
    const int i = i0 + site;
    const bool on = i < Vs;
    const int c4[4] = {i % Lx, (i / Lx) % Ly, i / (Lx * Ly), t};
    const size_t s = size_t(t) * Vs + i;
    const int par = (c4[0] + c4[1] + c4[2] + t) & 1;
    __syncthreads();  // the previous chunk's reads of nb and dS are done
    {
      // wave q: the forward and backward neighbours of the sites along mu = q
      const int st = q == 0 ? 1 : q == 1 ? Lx : q == 2 ? Lx * Ly : Vs;
      const int Lm = g.L[q], cm = c4[q];
      nb[2 * q][site] = on ? int(cm + 1 == Lm ? s - size_t(st) * (Lm - 1) : s + st) : -1;
      nb[2 * q + 1][site] = on ? int(cm == 0 ? s + size_t(st) * (Lm - 1) : s - st) : -1;
      if (q == 0) nb[2 * kNumPS][site] = on ? int(s) : -1;
    }
    // the colour vectors of the four directions
    cx<double> c[kNumPS][3];
#pragma unroll
    for (int mu = 0; mu < kNumPS; ++mu) {
      __syncthreads();  // nb written; the previous direction's reads of fS, bS done
      ps_stage(fS, eta, nullptr, nb[2 * mu]);
      asm volatile("" ::: "memory");  // the backward loads after the forward ones (fewer registers live)
      ps_stage(bS, eta, nullptr, nb[2 * mu + 1]);
      __syncthreads();
      if (on) {
        if (mu == 0) ps_eta_side<0>(U, Vh, nb, fS, bS, s, par, q, c[0]);
        else if (mu == 1) ps_eta_side<1>(U, Vh, nb, fS, bS, s, par, q, c[1]);
        else if (mu == 2) ps_eta_side<2>(U, Vh, nb, fS, bS, s, par, q, c[2]);
        else ps_eta_side<3>(U, Vh, nb, fS, bS, s, par, q, c[3]);
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (v > 0) __syncthreads();  // the previous variant's reads of dS are done
      ps_stage(dS, x, xts.p[v], nb[2 * kNumPS]);
      __syncthreads();
      if (on) {
        const cx<double> t0 = ps_term<0>(c[0], dS, q, kappa), t1 = ps_term<1>(c[1], dS, q, kappa);
        const cx<double> t2 = ps_term<2>(c[2], dS, q, kappa), t3 = ps_term<3>(c[3], dS, q, kappa);
        acc[v][0] += t0.re;
        acc[v][1] += t0.im;
        acc[v][2] += t1.re;
        acc[v][3] += t1.im;
        acc[v][4] += t2.re;
        acc[v][5] += t2.im;
        acc[v][6] += t3.re;
        acc[v][7] += t3.im;
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int k = 0; k < 2 * kNumPS; ++k) acc[v][k] = wave_sum(acc[v][k]);
  if (lane == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int k = 0; k < 2 * kNumPS; ++k) sh[v * 2 * kNumPS + k][wave] = acc[v][k];
  __syncthreads();
  // directions x, y, z: all four waves' sums at this timeslice; t: the
  // forward waves' (0, 1) at t - 1 in slot 8, the backward waves' (2, 3) at
  // t + 1 in slot 9
  if (threadIdx.x < NV * (2 * kNumPS + 2)) {
    const int v = threadIdx.x / (2 * kNumPS + 2), k = threadIdx.x % (2 * kNumPS + 2);
    const int m = k / 2, part = k % 2;  // m = 4: the backward t terms
    const double *row = sh[v * 2 * kNumPS + 2 * (m < kNumPS ? m : kNumPS - 1) + part];
    double sum;
    int slot, trow;
    if (m < kNumPS - 1) {
      sum = ((row[0] + row[1]) + row[2]) + row[3];
      slot = kNumTheta + m;
      trow = t;
    } else if (m == kNumPS - 1) {
      sum = row[0] + row[1];
      slot = kNumOps - 1;
      trow = t == 0 ? Lt - 1 : t - 1;
    } else {
      sum = row[2] + row[3];
      slot = kNumOps;
      trow = t + 1 == Lt ? 0 : t + 1;
    }
    out[((((size_t(v0 + v) * nrhs + r) * kOpSlots + slot) * Lt + trow) * nch + ch) * 2 + part] = sum;
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
    nch = std::max(1, std::min<int>(nch, int(cap_doubles / (size_t(nrhs) * kOpSlots * Lt * 2))));
  return nch;
}

// Variants per launch.  The local kernel's per-lane sums grow by 10 doubles
// per variant, and at 24^3 x 32 with 16 right-hand sides groups of three are
// fastest (2.2 ms for six variants, 2.6 in pairs, 2.4 all at once).  The
// point-split kernel's eta side (neighbour stagings and links, 2.5 ms) is
// shared by the variants of a launch, each adding 0.6 ms: all six in one
// launch (6.0 ms) beat three (8.9) or two (11.9) despite the occupancy its
// registers leave.
constexpr int kLocalGroup = 3, kPsGroup = 6;

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

template <int NV>
void launch_ps(lqcd_ctx *c, const void *eta, const void *x, const XtSet &xts, int v0, int nrhs, double *d,
               int nch) {
  const Geom &g = c->g;
  const int Lt = g.L[3];
  const int xq = (Lt * nch * nrhs + 7) / 8;  // logical workgroups per XCD (grid padded to 8 xq)
  hipLaunchKernelGGL(k_estimate_ps<NV>, dim3(8 * xq), dim3(kBlock), 0, c->stream, g,
                     static_cast<const cx<double> *>(c->U64.ptr), c->kappa, static_cast<const cx<double> *>(eta),
                     static_cast<const cx<double> *>(x), xts, v0, nch, nrhs, xq, d);
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
// corr[v]) with its partial sums in d (at least nvar * nrhs * kOpSlots * Lt
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
    for (int v0 = 0; v0 < nvar; v0 += kPsGroup) {
      const int n = std::min(kPsGroup, nvar - v0);
      LQCD_EST_DISPATCH(launch_ps, n, c, eta, x, group(v0, n), v0, nrhs, d, nch)
    }
#undef LQCD_EST_DISPATCH
  const int Lt = c->g.L[3];
  std::vector<double> hc(size_t(nvar) * nrhs * kOpSlots * Lt * nch * 2);
  LQCD_HIP(hipMemcpyAsync(hc.data(), d, hc.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LQCD_HIP(hipStreamSynchronize(c->stream));
  const int W = Lt + 1;
  for (int var = 0; var < nvar; ++var) {
    const double *hv = hc.data() + size_t(var) * nrhs * kOpSlots * Lt * nch * 2;
    const double *cv = corr ? corr[var] : nullptr;
    double *ev = est + size_t(var) * nth * W * 2, *sv = stderr_ + size_t(var) * nth * W * 2;
    std::vector<double> h(size_t(nrhs) * kOpSlots * Lt * 2, 0.0);
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
          size_t o = ((size_t(n) * kOpSlots + thetas[a]) * Lt + t) * 2;
          cdouble v(h[o], h[o + 1]);
          if (thetas[a] == kNumOps - 1) {  // point-split in t: its second slot
            const size_t o2 = ((size_t(n) * kOpSlots + kNumOps) * Lt + t) * 2;
            v += cdouble(h[o2], h[o2 + 1]);
          }
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
        c->red.ensure(size_t(nrhs) * kOpSlots * c->g.L[3] * nch * 2 * sizeof(double)));
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
        c->red.ensure(size_t(nvar) * nrhs * kOpSlots * c->g.L[3] * nch * 2 * sizeof(double)));
    estimate_with(c, thetas, nth, eta, x, xt_list, nvar, nrhs, corr_list, est, stderr_, samples, d, nch);
  });
}

extern "C" lqcd_status loop_estimate_noalloc(lqcd_ctx *c, const int *thetas, int nth, const void *eta,
                                             const void *x, const void *xt, int nrhs, const double *corr,
                                             double *est, double *stderr_, double *samples) {
  return guarded([&] {
    check_args(c, thetas, nth, eta, x, nrhs, est, stderr_, "loop_estimate_noalloc");
    const size_t one = size_t(nrhs) * kOpSlots * c->g.L[3] * 2;
    LQCD_CHECK(one <= kNoallocDoubles, LQCD_EINVAL,
               "loop_estimate_noalloc: %d right-hand sides x %d timeslices need %zu partial sums, more than "
               "the fixed scratch of %zu (use loop_estimate)",
               nrhs, c->g.L[3], one, kNoallocDoubles);
    double *d = noalloc_scratch();
    const int nch = estimate_chunks(c->g, nrhs, kNoallocDoubles);
    estimate_with(c, thetas, nth, eta, x, &xt, 1, nrhs, &corr, est, stderr_, samples, d, nch);
  });
}
