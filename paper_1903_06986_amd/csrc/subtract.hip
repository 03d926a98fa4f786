// Subtraction vectors and exact trace corrections (Sec. 5).
//
//  pert_subtract   PS:   xt = sum_{j=0}^{n} (kappa P)^j eta           (Eqs. (28), (31))
//  poly_subtract   POLY: xt = sum_j c_j (kappa P)^j eta, c from the Min-Res
//                  polynomial of one noise vector                    (Eqs. (40)-(50))
//  deflate_project HFES / hermitian-forced overlap removal:
//                  xt += g5 sum_q w_q e'_q (e'_q^+ eta)              (Eqs. (66)-(72))
//
// Polynomials are applied by Horner's rule, y <- c_j eta + kappa P y, one
// stencil pass (both parities) per degree.
//
// Trace corrections.  Tr_t(Theta p(kappa P)) = sum_j c_j kappa^j
// Tr_t(Theta P^j), and only closed paths contribute (Sec. 5.1): expanding
// P^j into sequences of hops, the diagonal element at site x is a sum over
// closed walks w of length j starting at x of (spin product S_w) x (link
// product W_w(x)), so Tr(Theta P^j)_xx = sum_w tr(Theta S_w) tr W_w(x).
// A hop followed by its reverse carries (1 - g)(1 + g) = 0, so only
// non-backtracking walks survive; on lattices with even extents every
// closed walk has even length.  The host enumerates the walks (closed
// modulo the periodic extents, so windings on short directions count) and
// their spin traces; the device forms the link products at every site.
// The paper obtains the same traces from unit-vector sources (Eqs.
// (32)-(35)); the walk sum is that computation with every source's
// non-returning paths dropped.
//
// Point-split operators (codes 5..8): Theta(mu) = kappa (backward minus
// forward hop along mu), so Tr(Theta(mu) P^j) is kappa times the sum over
// closed walks of length j + 1 whose first step runs along mu, each with
// tr(S_w) tr W_w(x) and the sign +1 for a backward, -1 for a forward first
// step.  Only odd j contribute (walks of even length), up to j = 7.
#include <algorithm>
#include <cmath>

#include "cplx.h"
#include "fields.h"
#include "gamma.h"
#include "pointsplit.h"
#include "smallla.h"
#include "solver.h"

namespace lqcd {

namespace {

// Right-hand sides per pass of the subtraction vectors: 16 fill the FP64
// link-tiled stencil and the 16-column matrix-core V C, at 3 x 16 full
// FP64 fields of workspace (4 GB on 24^3 x 32).
constexpr int kSubBlock = 16;

// ---------------------------------------------------------- walk tables
constexpr int kMaxWalkLen = 8;  // local: length <= 6 (orders <= 7); point-split: <= 8

struct Walk {
  int len;
  int dir[kMaxWalkLen];     // 2 * mu + (0: +mu, 1: -mu)
  double coef[kNumOps][2];  // tr(Theta S_w) for Theta = 1, g1..g4; point-split: +-tr(S_w)
};

using Spin = std::complex<double>[4][4];

void enumerate(int len, const int L[4], int depth, int last, int disp[4], const Spin &S,
               int dirs[kMaxWalkLen], std::vector<Walk> &out) {
  if (depth == len) {
    for (int mu = 0; mu < 4; ++mu)
      if (((disp[mu] % L[mu]) + L[mu]) % L[mu] != 0) return;
    Walk w;
    w.len = len;
    for (int i = 0; i < len; ++i) w.dir[i] = dirs[i];
    bool any = false;
    for (int th = 0; th < kNumTheta; ++th) {
      std::complex<double> G[4][4];
      gamma_dense(th, G);
      std::complex<double> t = 0;
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) t += G[a][b] * S[b][a];
      w.coef[th][0] = t.real();
      w.coef[th][1] = t.imag();
      if (std::abs(t) > 1e-12) any = true;
    }
    std::complex<double> trS = 0;
    for (int a = 0; a < 4; ++a) trS += S[a][a];
    for (int mu = 0; mu < kNumPS; ++mu) {
      const double sg = (dirs[0] >> 1) != mu ? 0.0 : ((dirs[0] & 1) ? 1.0 : -1.0);
      w.coef[kNumTheta + mu][0] = sg * trS.real();
      w.coef[kNumTheta + mu][1] = sg * trS.imag();
      if (sg != 0.0 && std::abs(trS) > 1e-12) any = true;
    }
    if (any) out.push_back(w);
    return;
  }
  for (int d = 0; d < 8; ++d) {
    if (depth > 0 && d == (last ^ 1)) continue;  // immediate reversal: zero spin factor
    const int mu = d >> 1, sgn = (d & 1) ? -1 : 1;
    disp[mu] += sgn;
    int dist = 0;
    for (int nu = 0; nu < 4; ++nu) {
      int a = ((disp[nu] % L[nu]) + L[nu]) % L[nu];
      dist += std::min(a, L[nu] - a);
    }
    if (dist <= len - depth - 1) {
      // S' = S (1 - g_mu) for a forward hop, S (1 + g_mu) backward
      std::complex<double> G[4][4], S2[4][4];
      gamma_dense(1 + mu, G);
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          std::complex<double> s = 0;
          for (int e = 0; e < 4; ++e) {
            std::complex<double> f = (e == b ? 1.0 : 0.0) - double(sgn) * G[e][b];
            s += S[a][e] * f;
          }
          S2[a][b] = s;
        }
      dirs[depth] = d;
      enumerate(len, L, depth + 1, d, disp, S2, dirs, out);
    }
    disp[mu] -= sgn;
  }
}

// Link U_mu at lexicographic coordinates (x, y, z, t) in the even/odd layout.
__device__ inline const cx<double> *link_at(const cx<double> *U, const Geom &g, int x, int y, int z,
                                            int t, int mu) {
  const int p = (x + y + z + t) & 1;
  const int s = x + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
  return U + ((size_t(p) * 4 + mu) * 9) * g.Vh + (s >> 1);
}

// One hop of a walk from coordinates c: the link of direction d (forward:
// U_mu(c), then c += mu; backward: c -= mu, then U_mu(c)^+) into Lk.
__device__ inline void walk_step(const cx<double> *U, const Geom &g, int c[4], int d, cx<double> Lk[3][3]) {
  const int mu = d >> 1;
  const size_t Vh = g.Vh;
  if ((d & 1) == 0) {
    const cx<double> *u = link_at(U, g, c[0], c[1], c[2], c[3], mu);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) Lk[a][b] = u[(3 * a + b) * Vh];
    c[mu] = (c[mu] + 1 == g.L[mu]) ? 0 : c[mu] + 1;
  } else {
    c[mu] = (c[mu] == 0) ? g.L[mu] - 1 : c[mu] - 1;
    const cx<double> *u = link_at(U, g, c[0], c[1], c[2], c[3], mu);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const cx<double> v = u[(3 * b + a) * Vh];
        Lk[a][b] = mk(v.re, -v.im);
      }
  }
}

// W <- W Lk
__device__ inline void su3_rmul(cx<double> W[3][3], const cx<double> Lk[3][3]) {
  cx<double> Nw[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Nw[a][b] = W[a][0] * Lk[0][b] + W[a][1] * Lk[1][b] + W[a][2] * Lk[2][b];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) W[a][b] = Nw[a][b];
}

// out[th][s] = sum_w coef_w[th] tr W_w(s) for every lexicographic site s.
// The walks come in depth-first order, cut into groups that share their
// first P steps (groups[i] = [first, end) walk indices): the prefix product
// A is formed once per group, each walk multiplies only its last len - P
// links into B, and tr W = tr(A B) = sum_ab A_ab B_ba.
__global__ void __launch_bounds__(kBlock)
    k_walk_trace(Geom g, const cx<double> *__restrict__ U, const Walk *__restrict__ walks,
                 const int2 *__restrict__ groups, int ngroup, int P, cx<double> *__restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int x0 = s % g.L[0], y0 = (s / g.L[0]) % g.L[1], z0 = (s / (g.L[0] * g.L[1])) % g.L[2],
            t0 = s / (g.L[0] * g.L[1] * g.L[2]);
  double acc[kNumOps][2] = {};
  for (int gi = 0; gi < ngroup; ++gi) {
    const int2 gr = groups[gi];
    int c[4] = {x0, y0, z0, t0};
    cx<double> A[3][3], Lk[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) A[a][b] = mk(a == b ? 1.0 : 0.0, 0.0);
    for (int i = 0; i < P; ++i) {
      walk_step(U, g, c, walks[gr.x].dir[i], Lk);
      su3_rmul(A, Lk);
    }
    for (int w = gr.x; w < gr.y; ++w) {
      const Walk &wk = walks[w];
      int cc[4] = {c[0], c[1], c[2], c[3]};
      cx<double> B[3][3];
      walk_step(U, g, cc, wk.dir[P], B);
      for (int i = P + 1; i < wk.len; ++i) {
        walk_step(U, g, cc, wk.dir[i], Lk);
        su3_rmul(B, Lk);
      }
      cx<double> tr = mk(0.0, 0.0);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) tr = tr + A[a][b] * B[b][a];
#pragma unroll
      for (int th = 0; th < kNumOps; ++th) {
        acc[th][0] += wk.coef[th][0] * tr.re - wk.coef[th][1] * tr.im;
        acc[th][1] += wk.coef[th][0] * tr.im + wk.coef[th][1] * tr.re;
      }
    }
  }
#pragma unroll
  for (int th = 0; th < kNumOps; ++th) out[size_t(th) * g.V + s] = mk(acc[th][0], acc[th][1]);
}

constexpr int kWaves = kBlock / 64;
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// out[row][t] = sum over the Vs sites of timeslice t of in[row][t * Vs + i]
__global__ void __launch_bounds__(kBlock)
    k_timeslice_sum(const cx<double> *__restrict__ in, int Vs, int Lt, cx<double> *__restrict__ out) {
  __shared__ double sh[2][kWaves];
  const int t = blockIdx.x, row = blockIdx.y;
  const cx<double> *p = in + (size_t(row) * Lt + t) * Vs;
  double a = 0, b = 0;
  for (int i = threadIdx.x; i < Vs; i += kBlock) {
    a += p[i].re;
    b += p[i].im;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wave] = a;
    sh[1][wave] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0, sb = 0;
    for (int w = 0; w < kWaves; ++w) {
      sa += sh[0][w];
      sb += sh[1][w];
    }
    out[size_t(row) * Lt + t] = mk(sa, sb);
  }
}

// Per-site bilinear for the hermitian-forced trace terms:
// out[th][s] = sum_q w_q e_q(s)^+ Theta g5 e_q(s), e_q in the even/odd
// layout (full fields n apart), s lexicographic.
__global__ void __launch_bounds__(kBlock)
    k_eig_bilinear(Geom g, const cx<double> *__restrict__ E, const cx<double> *__restrict__ F, size_t n,
                   int Q, const cx<double> *__restrict__ w, cx<double> *__restrict__ out, int g5) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int x = s % g.L[0], y = (s / g.L[0]) % g.L[1], z = (s / (g.L[0] * g.L[1])) % g.L[2],
            t = s / (g.L[0] * g.L[1] * g.L[2]);
  const int p = (x + y + z + t) & 1;
  const size_t Vh = g.Vh, off = size_t(p) * 12 * Vh + (s >> 1);
  double acc[kNumTheta][2] = {};
  for (int q = 0; q < Q; ++q) {
    cx<double> e[4][3], f[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        e[sp][c] = E[q * n + off + (sp * 3 + c) * Vh];
        f[sp][c] = F[q * n + off + (sp * 3 + c) * Vh];
      }
    const cx<double> wq = w[q];
#pragma unroll
    for (int th = 0; th < kNumTheta; ++th) {
      // (Theta [g5] f)_r = Theta_{r, col} [g5_{col}] f_col
      cx<double> sum = mk(0.0, 0.0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = kGamma[th].col[r];
        const double s5 = g5 ? kGamma[5].re[col] : 1.0;
        const cx<double> tv = mk(kGamma[th].re[r] * s5, kGamma[th].im[r] * s5);
#pragma unroll
        for (int c = 0; c < 3; ++c) sum = sum + cmulc(e[r][c], tv * f[col][c]);
      }
      cx<double> v = wq * sum;
      acc[th][0] += v.re;
      acc[th][1] += v.im;
    }
  }
#pragma unroll
  for (int th = 0; th < kNumTheta; ++th) out[size_t(th) * g.V + s] = mk(acc[th][0], acc[th][1]);
}

// Point-split bilinears of the subtraction trace terms:
// out[mu][s] = e(s)^+ (Theta(mu) [g5] f)(s) for one mode (e, f) in the
// even/odd layout (full fields), s lexicographic; g5 = 1 in the
// hermitian-forced terms (f = e), 0 in eigenvalue subtraction (e = left,
// f = right eigenvector).
__global__ void __launch_bounds__(kBlock)
    k_eig_bilinear_ps(Geom g, const cx<double> *__restrict__ U, double kappa,
                      const cx<double> *__restrict__ E, const cx<double> *__restrict__ F,
                      cx<double> *__restrict__ out, int g5) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int Ls[4] = {g.L[0], g.L[1], g.L[2], g.L[3]};
  const int c[4] = {s % Ls[0], (s / Ls[0]) % Ls[1], (s / (Ls[0] * Ls[1])) % Ls[2], s / (Ls[0] * Ls[1] * Ls[2])};
  const size_t Vh = g.Vh;
  auto load = [&](const cx<double> *src, const int cc[4], cx<double> v[12], bool gam5) {
    const int p = (cc[0] + cc[1] + cc[2] + cc[3]) & 1;
    const int sl = cc[0] + Ls[0] * (cc[1] + Ls[1] * (cc[2] + Ls[2] * cc[3]));
    const size_t off = size_t(p) * 12 * Vh + size_t(sl >> 1);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      v[k] = src[off + k * Vh];
      if (gam5 && k >= 6) v[k] = -v[k];
    }
  };
  cx<double> a[12];
  load(E, c, a, false);
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    int cf[4] = {c[0], c[1], c[2], c[3]}, cb[4] = {c[0], c[1], c[2], c[3]};
    cf[mu] = c[mu] + 1 == Ls[mu] ? 0 : c[mu] + 1;
    cb[mu] = c[mu] == 0 ? Ls[mu] - 1 : c[mu] - 1;
    cx<double> b[12];
    load(F, cf, b, g5 != 0);
    const cx<double> vf = ps_half<true>(a, b, ps_link(U, g, c[0], c[1], c[2], c[3], mu), Vh, mu);
    load(F, cb, b, g5 != 0);
    const cx<double> vb = ps_half<false>(a, b, ps_link(U, g, cb[0], cb[1], cb[2], cb[3], mu), Vh, mu);
    out[size_t(mu) * g.V + s] = kappa * (vb - vf);
  }
}

// In place g5 on full even/odd fields: negate spins 2, 3 (components 6..11).
__global__ void k_g5_eo(cx<double> *__restrict__ f, size_t Vh, size_t stride, int nf) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t per = 2 * 6 * Vh;  // per field: two parities x 6 lower components
  if (i >= per * nf) return;
  const size_t fidx = i / per, r = i % per;
  const size_t par = r / (6 * Vh), k = r % (6 * Vh);
  cx<double> *p = f + fidx * stride + par * 12 * Vh + 6 * Vh + k;
  *p = -*p;
}

// C[r][q] *= w[q] for nb columns of Q rows (w on the device).
__global__ void k_scale_rows(cx<double> *__restrict__ C, const cx<double> *__restrict__ w, int Q, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < Q * nb) C[i] = C[i] * w[i % Q];
}

void h2d(lqcd_ctx *c, void *dst, const void *src, size_t bytes) {
  LQCD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
  LQCD_HIP(hipStreamSynchronize(c->stream));
}
void d2h(lqcd_ctx *c, void *dst, const void *src, size_t bytes) {
  LQCD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream));
  LQCD_HIP(hipStreamSynchronize(c->stream));
}

// Per-timeslice sums of nrow site fields [row][V] (lexicographic).
std::vector<cdouble> timeslice_rows(lqcd_ctx *c, const void *site, int nrow, DevBuf &tmp) {
  const Geom &g = c->g;
  const int Lt = g.L[3], Vs = g.V / Lt;
  cdouble *d = static_cast<cdouble *>(tmp.ensure(size_t(nrow) * Lt * sizeof(cdouble)));
  hipLaunchKernelGGL(k_timeslice_sum, dim3(Lt, nrow), dim3(kBlock), 0, c->stream,
                     static_cast<const cx<double> *>(site), Vs, Lt, reinterpret_cast<cx<double> *>(d));
  LQCD_HIP(hipGetLastError());
  std::vector<cdouble> h(size_t(nrow) * Lt);
  d2h(c, h.data(), d, h.size() * sizeof(cdouble));
  return h;
}

// Tr_t(Theta P^j) for j = 0..kMaxOrder and every operator code, filled
// once per context (point-split rows without their factor kappa).
// The walks of length 8 (36k per site) serve only the point-split rows of
// order 7 and are enumerated when such a row is first asked for.
void ensure_walk_traces(lqcd_ctx *c, bool need_len8) {
  if (c->have_walk_traces && (!need_len8 || c->have_walk_len8)) return;
  const Geom &g = c->g;
  const int Lt = g.L[3], Vs = g.V / Lt;
  if (!c->have_walk_traces) {
    c->walk_traces.assign(size_t(kMaxOrder + 1) * kNumOps * Lt, 0.0);
    for (int t = 0; t < Lt; ++t) c->walk_traces[t] = 12.0 * Vs;  // Tr(1) per slice
  }
  std::vector<cdouble> &T = c->walk_traces;
  DevBuf site, walks, tmp;
  site.ensure(size_t(kNumOps) * g.V * sizeof(cdouble));
  // odd walks cannot close on even extents; a walk of length len gives the
  // local rows of order len and the point-split rows of order len - 1
  const int len0 = c->have_walk_traces ? kMaxWalkLen : 2;
  const int len1 = need_len8 ? kMaxWalkLen : kMaxWalkLen - 2;
  for (int len = len0; len <= len1; len += 2) {
    std::vector<Walk> ws;
    int disp[4] = {0, 0, 0, 0}, dirs[kMaxWalkLen];
    std::complex<double> I[4][4];
    gamma_dense(0, I);
    enumerate(len, g.L, 0, -1, disp, I, dirs, ws);
    if (ws.empty()) continue;
    // groups of consecutive walks with the same first P = len - 3 steps
    const int P = std::max(0, len - 3);
    std::vector<int2> gr;
    for (int w = 0; w < int(ws.size()); ++w) {
      const bool same = w > 0 && std::equal(ws[w].dir, ws[w].dir + P, ws[w - 1].dir);
      if (same)
        gr.back().y = w + 1;
      else
        gr.push_back(make_int2(w, w + 1));
    }
    walks.ensure(ws.size() * sizeof(Walk) + gr.size() * sizeof(int2));
    h2d(c, walks.ptr, ws.data(), ws.size() * sizeof(Walk));
    int2 *dgr = reinterpret_cast<int2 *>(static_cast<char *>(walks.ptr) + ws.size() * sizeof(Walk));
    h2d(c, dgr, gr.data(), gr.size() * sizeof(int2));
    hipLaunchKernelGGL(k_walk_trace, dim3(nblocks(g.V)), dim3(kBlock), 0, c->stream, g,
                       static_cast<const cx<double> *>(c->U64.ptr), walks.as<Walk>(), dgr, int(gr.size()), P,
                       site.as<cx<double>>());
    LQCD_HIP(hipGetLastError());
    std::vector<cdouble> ts = timeslice_rows(c, site.ptr, kNumOps, tmp);
    for (int th = 0; th < kNumOps; ++th) {
      const int j = th < kNumTheta ? len : len - 1;
      if (j > kMaxOrder) continue;
      for (int t = 0; t < Lt; ++t) T[(size_t(j) * kNumOps + th) * Lt + t] = ts[size_t(th) * Lt + t];
    }
  }
  c->have_walk_traces = true;
  if (need_len8) c->have_walk_len8 = true;
}

// corr[th][t] = sum_j coeffs[j] kappa^j Tr_t(Theta_th P^j)  (point-split:
// times the operator's own kappa)
void poly_trace(lqcd_ctx *c, const std::vector<cdouble> &coeffs, const int *thetas, int nth,
                double *corr_host) {
  bool ps = false;
  for (int a = 0; a < nth; ++a) ps = ps || thetas[a] >= kNumTheta;
  ensure_walk_traces(c, ps && coeffs.size() > size_t(kMaxWalkLen - 1));
  const int Lt = c->g.L[3];
  for (int a = 0; a < nth; ++a)
    for (int t = 0; t < Lt; ++t) {
      cdouble s = 0;
      double kj = 1;
      for (size_t j = 0; j < coeffs.size(); ++j, kj *= c->kappa)
        s += coeffs[j] * kj * c->walk_traces[(j * kNumOps + thetas[a]) * Lt + t];
      if (thetas[a] >= kNumTheta) s *= c->kappa;
      corr_host[2 * (a * Lt + t)] = s.real();
      corr_host[2 * (a * Lt + t) + 1] = s.imag();
    }
}

// y = sum_j coeffs[j] (kappa P)^j e on full even/odd FP64 fields (nf of
// them, fl apart).  Returns the buffer holding the result (a or b).
cx<double> *horner(lqcd_ctx *c, const std::vector<cdouble> &coeffs, const cx<double> *e,
                   cx<double> *a, cx<double> *b, int nf) {
  const size_t hl = half_len(c->g), fl = full_len(c->g);
  const int d = int(coeffs.size()) - 1;
  cdouble zero(0, 0);
  axpby<double>(c, &coeffs[d], e, fl, &zero, a, fl, fl, nf, false);
  cx<double> *y = a, *yn = b;
  for (int j = d - 1; j >= 0; --j) {
    for (int p = 0; p < 2; ++p)
      hop_half<double>(c, p, y + (1 - p) * hl, e + p * hl, yn + p * hl, coeffs[j], c->kappa, false,
                       false, nf, fl, fl, fl);
    std::swap(y, yn);
  }
  return y;
}

void check_thetas(const int *th, int nth) {
  LQCD_CHECK(nth >= 0 && (nth == 0 || th), LQCD_EINVAL, "thetas: null or negative count");
  for (int a = 0; a < nth; ++a)
    LQCD_CHECK(th[a] >= 0 && th[a] < kNumOps, LQCD_EINVAL, "operator code %d outside 0..8", th[a]);
}

// Several polynomials in kappa P applied to the same noise: the powers
// P_j = (kappa P)^j eta are formed once (one hopping step each) and kept,
// and one pass combines them into every polynomial's vector, written in the
// lexicographic layout.
constexpr int kMaxPolys = 4;
struct PolySet {
  cx<double> c[kMaxPolys][kMaxOrder + 1];
  cx<double> *out[kMaxPolys];
};

// out_a (lex) = sum_{j < d1} c[a][j] P_j for the powers P_j (even/odd, blk
// apart; right-hand side r at r fl) of one block.  A workgroup takes 64
// consecutive lex sites s0.. of right-hand side blockIdx.y: with Lx even,
// sites 2h and 2h + 1 are x neighbours of opposite parity, both at index h
// of their parity's half, so the 64 sites are 32 consecutive h in each
// half.  Thread element i = (component k, parity, h - s0/2) with h fastest
// loads coalesced runs of 32 complex of every power; each output goes
// through LDS in lex order and is stored contiguously (768 complex).
constexpr int kPolySites = 64;
template <int NP>
__global__ void __launch_bounds__(kBlock)
    k_poly_lex(Geom g, const cx<double> *__restrict__ P, size_t fl, size_t blk, int d1, PolySet ps) {
  __shared__ cx<double> sh[kPolySites * 12];
  constexpr int kPer = kPolySites * 12 / kBlock;  // elements per thread
  const int s0 = blockIdx.x * kPolySites;
  const size_t rhs = blockIdx.y;
  const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
  const size_t Vh = g.Vh;
  const cx<double> *src = P + rhs * fl;
  cx<double> acc[kPer][NP];
  int at[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = threadIdx.x + u * kBlock;
    const int hh = i % (kPolySites / 2), rest = i / (kPolySites / 2);
    const int par = rest & 1, k = rest >> 1;
    const int h = s0 / 2 + hh, e = 2 * h;  // the even-indexed site of the pair
    const bool ok = e < g.V;
    const int x = e % Lx, y = (e / Lx) % Ly, z = (e / (Lx * Ly)) % Lz, t = e / (Lx * Ly * Lz);
    const int s = ((x + y + z + t) & 1) == par ? e : e + 1;
    at[u] = ok ? (s - s0) * 12 + k : -1;
    const cx<double> *q = src + par * 12 * Vh + k * Vh + (ok ? h : 0);
    cx<double> v[kMaxOrder + 1];  // every power's element in flight together
#pragma unroll
    for (int j = 0; j <= kMaxOrder; ++j)
      if (j < d1) v[j] = ldc(q + j * blk);
#pragma unroll
    for (int a = 0; a < NP; ++a) {
      acc[u][a] = mk(0.0, 0.0);
#pragma unroll
      for (int j = 0; j <= kMaxOrder; ++j)
        if (j < d1) acc[u][a] = acc[u][a] + ps.c[a][j] * v[j];
    }
  }
  const size_t o = (rhs * size_t(g.V) + s0) * 12;
  const int nel = min(kPolySites, g.V - s0) * 12;
#pragma unroll
  for (int a = 0; a < NP; ++a) {
    if (a > 0) __syncthreads();  // the previous output's reads of sh are done
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (at[u] >= 0) sh[at[u]] = acc[u][a];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int i = threadIdx.x + u * kBlock;
      if (i < nel) stc(ps.out[a] + o + i, sh[i]);
    }
  }
}

// xt (lex) = p(kappa P) eta (lex) for nrhs fields, in blocks.
void apply_poly_lex(lqcd_ctx *c, const std::vector<cdouble> &coeffs, const void *eta, void *xt,
                    int nrhs) {
  const size_t fl = full_len(c->g);
  const int blk = kSubBlock;
  for (int r0 = 0; r0 < nrhs; r0 += blk) {
    const int nb = std::min(blk, nrhs - r0);
    cx<double> *E = static_cast<cx<double> *>(c->ws[0].ensure(fl * nb * sizeof(cx<double>)));
    cx<double> *A = static_cast<cx<double> *>(c->ws[1].ensure(fl * nb * sizeof(cx<double>)));
    cx<double> *B = static_cast<cx<double> *>(c->ws[2].ensure(fl * nb * sizeof(cx<double>)));
    pack_eo<double>(c, static_cast<const cdouble *>(eta) + r0 * fl, E, nb, fl);
    cx<double> *Y = horner(c, coeffs, E, A, B, nb);
    unpack_eo<double>(c, Y, static_cast<cdouble *>(xt) + r0 * fl, nb, fl);
  }
}

std::vector<cdouble> kp_to_m(const std::vector<cdouble> &cc) {
  // (kappa P)^j = (1 - M)^j = sum_k C(j,k) (-1)^k M^k
  const int d = int(cc.size()) - 1;
  std::vector<cdouble> a(d + 1, 0.0);
  for (int j = 0; j <= d; ++j) {
    double binom = 1;
    for (int k = 0; k <= j; ++k) {
      a[k] += cc[j] * binom * ((k % 2) ? -1.0 : 1.0);
      binom = binom * (j - k) / (k + 1);
    }
  }
  return a;
}

// Eigenvalue subtraction data (Sec. 5.3) from the even/odd deflation space
// A V_k = V_{k+1} Hbar_k of Mhat (op SCHUR): Ritz pairs H_k = S diag(lh) S^{-1}
// give right even vectors V_k S.  The Krylov space holds no left
// eigenvectors of the non-normal Mhat, so the left vector of lh is g5 times
// the right Ritz vector of its conjugate partner (Mhat^H = g5 Mhat g5),
// scaled so that lh_vec^H rh = 1.  The full eigenpairs of
// M = [[1, -kappa D_eo], [-kappa D_oe, 1]] follow from
// (1 - lambda)^2 = 1 - lh, small branch lambda = 1 - sqrt(1 - lh):
// r = (rh, kappa / (1 - lambda) D_oe rh),
// l = (lh_vec, kappa / (1 - conj lambda) g5 D_oe g5 lh_vec) / 2
// (D_eo^H = g5 D_oe g5; l^H r = 2 before the halving).  The Q pairs of
// smallest |lambda| are kept with the space.
void es_pairs(lqcd_ctx *c, lqcd_defl *d, int Q) {
  LQCD_CHECK(d->op == LQCD_OP_SCHUR, LQCD_EINVAL,
             "eigenvalue subtraction needs the even/odd deflation space (op LQCD_OP_SCHUR)");
  LQCD_CHECK(Q >= 1 && Q <= d->k, LQCD_EINVAL, "Q = %d outside 1..k = %d", Q, d->k);
  std::lock_guard<std::mutex> lk(d->fill_mu);
  if (d->Qes == Q && d->ER.ptr) return;
  const int k = d->k;
  la::Mat T(k, k);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i) T(i, j) = d->H(i, j);
  std::vector<cdouble> lh;
  la::Mat Sr;
  LQCD_CHECK(la::eig(T, lh, Sr), LQCD_ENOCONV, "eigenvalue subtraction: Ritz eigenproblem did not converge");
  std::vector<cdouble> lam(k);
  for (int i = 0; i < k; ++i) lam[i] = 1.0 - std::sqrt(1.0 - lh[i]);
  std::vector<int> ord(k);
  for (int i = 0; i < k; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return std::abs(lam[a]) < std::abs(lam[b]); });
  la::Mat SR(k, Q), SL(k, Q);  // SL: Ritz coefficients of each mode's conjugate partner
  d->es_lam.resize(Q);
  for (int q = 0; q < Q; ++q) {
    const int j = ord[q];
    int pj = 0;
    for (int i = 1; i < k; ++i)
      if (std::abs(lh[i] - std::conj(lh[j])) < std::abs(lh[pj] - std::conj(lh[j]))) pj = i;
    d->es_lam[q] = lam[j];
    for (int i = 0; i < k; ++i) {
      SR(i, q) = Sr(i, j);
      SL(i, q) = Sr(i, pj);
    }
  }
  const size_t hl = half_len(c->g), fl = full_len(c->g);
  cx<double> *R = static_cast<cx<double> *>(d->ER.ensure(size_t(Q) * fl * sizeof(cx<double>)));
  cx<double> *L = static_cast<cx<double> *>(d->EL.ensure(size_t(Q) * fl * sizeof(cx<double>)));
  fill_zero(c, R, size_t(Q) * fl * sizeof(cx<double>));
  fill_zero(c, L, size_t(Q) * fl * sizeof(cx<double>));
  DevBuf Sd;
  cdouble *sr = static_cast<cdouble *>(Sd.ensure(2 * size_t(k) * Q * sizeof(cdouble)));
  h2d(c, sr, SR.a.data(), SR.a.size() * sizeof(cdouble));
  h2d(c, sr + size_t(k) * Q, SL.a.data(), SL.a.size() * sizeof(cdouble));
  gemm_nn<double>(c, d->V.ptr, hl, 0, k, sr, k, 0, R, fl, 0, Q, hl, 1, 1.0);  // even halves
  gemm_nn<double>(c, d->V.ptr, hl, 0, k, sr + size_t(k) * Q, k, 0, L, fl, 0, Q, hl, 1, 1.0);
  // left even halves: g5 (partner), then scaled so that l^H r = 1
  {
    const size_t tot = 2 * 6 * size_t(c->g.Vh) * Q;  // the odd halves are still zero
    hipLaunchKernelGGL(k_g5_eo, dim3(nblocks(tot)), dim3(kBlock), 0, c->stream, L, size_t(c->g.Vh), fl, Q);
    LQCD_HIP(hipGetLastError());
    cdouble *Dd = static_cast<cdouble *>(c->ws[5].ensure(size_t(Q) * sizeof(cdouble)));
    multi_dot<double>(c, L, fl, fl, 1, R, fl, fl, Q, Dd, 1);  // l_q^H r_q
    std::vector<cdouble> D(Q), a(Q), z(Q, cdouble(0, 0));
    d2h(c, D.data(), Dd, Q * sizeof(cdouble));
    for (int q = 0; q < Q; ++q) {
      LQCD_CHECK(std::abs(D[q]) > 0, LQCD_ENOCONV, "eigenvalue subtraction: left/right pair %d orthogonal", q);
      a[q] = 1.0 / std::conj(D[q]);
    }
    axpby<double>(c, a.data(), L, fl, z.data(), L, fl, hl, Q, true);
  }
  // odd halves: D_oe r and g5 D_oe g5 l (parity 1 output from the even input)
  hop_half<double>(c, 1, R, nullptr, R + hl, cdouble(0, 0), 1.0, false, false, Q, fl, 0, fl);
  hop_half<double>(c, 1, L, nullptr, L + hl, cdouble(0, 0), 1.0, true, true, Q, fl, 0, fl);
  std::vector<cdouble> ar(Q), al(Q), ae(Q, cdouble(0.5, 0)), zero(Q, cdouble(0, 0));
  for (int q = 0; q < Q; ++q) {
    ar[q] = c->kappa / (1.0 - d->es_lam[q]);
    al[q] = 0.5 * c->kappa / (1.0 - std::conj(d->es_lam[q]));
  }
  axpby<double>(c, ar.data(), R + hl, fl, zero.data(), R + hl, fl, hl, Q, true);
  axpby<double>(c, ae.data(), L, fl, zero.data(), L, fl, hl, Q, true);
  axpby<double>(c, al.data(), L + hl, fl, zero.data(), L + hl, fl, hl, Q, true);
  LQCD_HIP(hipStreamSynchronize(c->stream));
  d->Qes = Q;
  d->es_bil.clear();
}

// Eigenvalue subtraction: xt += sum_q (1/lambda_q) r_q (l_q^H eta),
// corr += sum_q (1/lambda_q) sum_{x in t} l_q^H Theta r_q.
void es_project(lqcd_ctx *c, lqcd_defl *d, int Q, const int *thetas, int nth, const void *eta, void *xt,
                int nrhs, double *corr) {
  es_pairs(c, d, Q);
  const size_t fl = full_len(c->g);
  const int Lt = c->g.L[3];
  const cx<double> *R = d->ER.as<cx<double>>(), *L = d->EL.as<cx<double>>();
  std::vector<cdouble> w(Q);
  for (int q = 0; q < Q; ++q) w[q] = 1.0 / d->es_lam[q];
  if (corr && nth > 0) {
    std::lock_guard<std::mutex> lk(d->fill_mu);
    if (d->es_bil.empty()) {
      d->es_bil.assign(size_t(Q) * kNumOps * Lt, 0.0);
      cdouble one(1, 0);
      DevBuf wbuf, tmp;
      cdouble *wd = static_cast<cdouble *>(wbuf.ensure(sizeof(cdouble)));
      h2d(c, wd, &one, sizeof(cdouble));
      cx<double> *site = static_cast<cx<double> *>(c->ws[7].ensure(size_t(kNumOps) * c->g.V * sizeof(cdouble)));
      for (int q = 0; q < Q; ++q) {
        hipLaunchKernelGGL(k_eig_bilinear, dim3(nblocks(c->g.V)), dim3(kBlock), 0, c->stream, c->g,
                           L + size_t(q) * fl, R + size_t(q) * fl, fl, 1,
                           reinterpret_cast<const cx<double> *>(wd), site, 0);
        LQCD_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_eig_bilinear_ps, dim3(nblocks(c->g.V)), dim3(kBlock), 0, c->stream, c->g,
                           static_cast<const cx<double> *>(c->U64.ptr), c->kappa, L + size_t(q) * fl,
                           R + size_t(q) * fl, site + size_t(kNumTheta) * c->g.V, 0);
        LQCD_HIP(hipGetLastError());
        std::vector<cdouble> ts = timeslice_rows(c, site, kNumOps, tmp);
        std::copy(ts.begin(), ts.end(), d->es_bil.begin() + size_t(q) * kNumOps * Lt);
      }
    }
    for (int a = 0; a < nth; ++a)
      for (int t = 0; t < Lt; ++t) {
        cdouble v = 0;
        for (int q = 0; q < Q; ++q) v += w[q] * d->es_bil[(size_t(q) * kNumOps + thetas[a]) * Lt + t];
        corr[2 * (a * Lt + t)] += v.real();
        corr[2 * (a * Lt + t) + 1] += v.imag();
      }
  }
  const int blk = kSubBlock;
  for (int r0 = 0; r0 < nrhs; r0 += blk) {
    const int nb = std::min(blk, nrhs - r0);
    cx<double> *Et = static_cast<cx<double> *>(c->ws[0].ensure(fl * nb * sizeof(cx<double>)));
    cx<double> *Yt = static_cast<cx<double> *>(c->ws[3].ensure(fl * nb * sizeof(cx<double>)));
    cx<double> *Xl = static_cast<cx<double> *>(c->ws[4].ensure(fl * nb * sizeof(cx<double>)));
    pack_eo<double>(c, static_cast<const cdouble *>(eta) + r0 * fl, Et, nb, fl);
    cdouble *Cd = static_cast<cdouble *>(c->ws[5].ensure(size_t(Q) * nb * sizeof(cdouble)));
    gemm_tn<double>(c, L, fl, Q, Et, fl, nb, fl, Cd, Q);
    std::vector<cdouble> Ch(size_t(Q) * nb);
    d2h(c, Ch.data(), Cd, Ch.size() * sizeof(cdouble));
    for (int r = 0; r < nb; ++r)
      for (int q = 0; q < Q; ++q) Ch[size_t(r) * Q + q] *= w[q];
    h2d(c, Cd, Ch.data(), Ch.size() * sizeof(cdouble));
    fill_zero(c, Yt, fl * nb * sizeof(cx<double>));
    gemm_nn<double>(c, R, fl, 0, Q, Cd, Q, 0, Yt, fl, 0, nb, fl, 1, 1.0);
    unpack_eo<double>(c, Yt, Xl, nb, fl);
    cdouble one(1, 0);
    cx<double> *xo = reinterpret_cast<cx<double> *>(static_cast<cdouble *>(xt) + r0 * fl);
    axpby<double>(c, &one, Xl, fl, &one, xo, fl, fl, nb, false);
  }
}

// Hermitian-forced projections per deflate_project_multi call.
constexpr int kMaxHfVariants = 4;

// The weights w_q of a hermitian-forced projection (deflate_project, modes
// HFES and EIGPOLY) on the eigenpairs of d, with the trace correction added
// to corr (NULL: none) and 1/xi'_q written to xi_inv_host (NULL: not).
std::vector<cdouble> hf_weights(lqcd_ctx *c, lqcd_defl *d, int Q, lqcd_defl_mode mode, const double *coeffs_host,
                                int ncoeff, const int *thetas, int nth, double *corr, double *xi_inv_host) {
  const size_t fl = full_len(c->g);
  const cx<double> *E = d->E.as<cx<double>>();
  const int Lt = c->g.L[3];
  std::vector<cdouble> w(Q), xi(Q, 0.0);
  for (int q = 0; q < Q; ++q) w[q] = 1.0 / d->lam[q];
  if (mode == LQCD_DEFL_EIGPOLY) {
    // 1/xi'_q = e'^+ g5 p(kappa P) e'  (Eq. (69) with M'_poly^{-1} = g5 p),
    // computed once per polynomial and kept with the eigenpairs
    std::vector<cdouble> cc(ncoeff);
    for (int j = 0; j < ncoeff; ++j) cc[j] = cdouble(coeffs_host[2 * j], coeffs_host[2 * j + 1]);
    std::lock_guard<std::mutex> lk(d->fill_mu);
    bool found = false;
    for (auto &e : d->xi_cache)
      if (e.first == cc) {
        xi = e.second;
        found = true;
      }
    if (!found) {
      cx<double> *A = static_cast<cx<double> *>(c->ws[1].ensure(fl * Q * sizeof(cx<double>)));
      cx<double> *B = static_cast<cx<double> *>(c->ws[2].ensure(fl * Q * sizeof(cx<double>)));
      cx<double> *Y = horner(c, cc, E, A, B, Q);
      size_t tot = 2 * 6 * size_t(c->g.Vh) * Q;
      hipLaunchKernelGGL(k_g5_eo, dim3(nblocks(tot)), dim3(kBlock), 0, c->stream, Y, size_t(c->g.Vh), fl, Q);
      LQCD_HIP(hipGetLastError());
      cdouble *Cd = static_cast<cdouble *>(c->ws[5].ensure(size_t(Q) * sizeof(cdouble)));
      // xi_inv[q] = <E_q, Y_q>: a batched dot with each vector its own basis of one
      multi_dot<double>(c, E, fl, fl, 1, Y, fl, fl, Q, Cd, 1);
      d2h(c, xi.data(), Cd, Q * sizeof(cdouble));
      d->xi_cache.emplace_back(cc, xi);
    }
    for (int q = 0; q < Q; ++q) w[q] -= xi[q];
  }
  if (xi_inv_host)
    for (int q = 0; q < Q; ++q) {
      xi_inv_host[2 * q] = xi[q].real();
      xi_inv_host[2 * q + 1] = xi[q].imag();
    }
  // trace correction: sum_q w_q e_q^+ Theta g5 e_q per timeslice, from the
  // per-mode bilinears (computed once per set of eigenpairs)
  if (corr && nth > 0) {
    std::lock_guard<std::mutex> lk(d->fill_mu);
    if (d->bil.empty()) {
      d->bil.assign(size_t(Q) * kNumOps * Lt, 0.0);
      cdouble one(1, 0);
      cdouble *wd = static_cast<cdouble *>(c->ws[6].ensure(sizeof(cdouble)));
      h2d(c, wd, &one, sizeof(cdouble));
      cx<double> *site = static_cast<cx<double> *>(c->ws[7].ensure(size_t(kNumOps) * c->g.V * sizeof(cdouble)));
      DevBuf tmp;
      for (int q = 0; q < Q; ++q) {
        hipLaunchKernelGGL(k_eig_bilinear, dim3(nblocks(c->g.V)), dim3(kBlock), 0, c->stream, c->g,
                           E + size_t(q) * fl, E + size_t(q) * fl, fl, 1,
                           reinterpret_cast<const cx<double> *>(wd), site, 1);
        LQCD_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_eig_bilinear_ps, dim3(nblocks(c->g.V)), dim3(kBlock), 0, c->stream, c->g,
                           static_cast<const cx<double> *>(c->U64.ptr), c->kappa, E + size_t(q) * fl,
                           E + size_t(q) * fl, site + size_t(kNumTheta) * c->g.V, 1);
        LQCD_HIP(hipGetLastError());
        std::vector<cdouble> ts = timeslice_rows(c, site, kNumOps, tmp);
        std::copy(ts.begin(), ts.end(), d->bil.begin() + size_t(q) * kNumOps * Lt);
      }
    }
    for (int a = 0; a < nth; ++a)
      for (int t = 0; t < Lt; ++t) {
        cdouble v = 0;
        for (int q = 0; q < Q; ++q) v += w[q] * d->bil[(size_t(q) * kNumOps + thetas[a]) * Lt + t];
        corr[2 * (a * Lt + t)] += v.real();
        corr[2 * (a * Lt + t) + 1] += v.imag();
      }
  }
  return w;
}

// xt[v] += g5 E (w[v] .* (E^H eta)) for nvar weight sets, with E^H eta formed
// once per block of right-hand sides.
void hf_update(lqcd_ctx *c, lqcd_defl *d, int Q, const void *eta, int nvar, void *const *xt,
               const std::vector<cdouble> *w, int nrhs) {
  const size_t fl = full_len(c->g);
  const cx<double> *E = d->E.as<cx<double>>();
  // xt += g5 E (w .* (E^H eta)), on the lexicographic copies of E and g5 E
  // (made once per set of eigenpairs), so that eta is read and xt updated
  // in place: one pass over the modes for the dots, one for the update
  const size_t Vh = size_t(c->g.Vh);
  std::unique_lock<std::mutex> lk(d->fill_mu);
  if (d->lex_Q != Q) {
    cx<double> *El = static_cast<cx<double> *>(d->Elex.ensure(fl * Q * sizeof(cx<double>)));
    cx<double> *Gl = static_cast<cx<double> *>(d->G5Elex.ensure(fl * Q * sizeof(cx<double>)));
    cx<double> *T = static_cast<cx<double> *>(c->ws[1].ensure(fl * Q * sizeof(cx<double>)));
    unpack_eo<double>(c, E, El, Q, fl);
    LQCD_HIP(hipMemcpyAsync(T, E, fl * Q * sizeof(cx<double>), hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(k_g5_eo, dim3(nblocks(2 * 6 * Vh * Q)), dim3(kBlock), 0, c->stream, T, Vh, fl, Q);
    LQCD_HIP(hipGetLastError());
    unpack_eo<double>(c, T, Gl, Q, fl);
    LQCD_HIP(hipStreamSynchronize(c->stream));
    d->lex_Q = Q;
  }
  lk.unlock();
  const cx<double> *El = d->Elex.as<cx<double>>(), *Gl = d->G5Elex.as<cx<double>>();
  cdouble *wd = static_cast<cdouble *>(c->ws[6].ensure(size_t(Q) * nvar * sizeof(cdouble)));
  std::vector<cdouble> wh(size_t(Q) * nvar);
  for (int v = 0; v < nvar; ++v) std::copy(w[v].begin(), w[v].end(), wh.begin() + size_t(v) * Q);
  h2d(c, wd, wh.data(), wh.size() * sizeof(cdouble));
  const int blk = kSubBlock;
  for (int r0 = 0; r0 < nrhs; r0 += blk) {
    const int nb = std::min(blk, nrhs - r0);
    // [E^H eta | w[0] .* E^H eta | w[1] .* ...]: the overlaps, then one scaled copy per weight set
    cdouble *Cd = static_cast<cdouble *>(c->ws[5].ensure(size_t(Q) * nb * (nvar + 1) * sizeof(cdouble)));
    gemm_tn<double>(c, El, fl, Q, static_cast<const cdouble *>(eta) + r0 * fl, fl, nb, fl, Cd, Q);
    for (int v = 0; v < nvar; ++v) {
      cdouble *Cv = Cd + size_t(Q) * nb * (v + 1);
      LQCD_HIP(hipMemcpyAsync(Cv, Cd, size_t(Q) * nb * sizeof(cdouble), hipMemcpyDeviceToDevice, c->stream));
      hipLaunchKernelGGL(k_scale_rows, dim3(nblocks(size_t(Q) * nb)), dim3(kBlock), 0, c->stream,
                         reinterpret_cast<cx<double> *>(Cv), reinterpret_cast<const cx<double> *>(wd) + size_t(v) * Q,
                         Q, nb);
      LQCD_HIP(hipGetLastError());
      gemm_nn<double>(c, Gl, fl, 0, Q, Cv, Q, 0, static_cast<cdouble *>(xt[v]) + r0 * fl, fl, 0, nb, fl, 1, 1.0);
    }
  }
}

}  // namespace

}  // namespace lqcd

using namespace lqcd;

extern "C" lqcd_status pert_subtract(lqcd_ctx *c, int order, const int *thetas, int nth,
                                     const void *eta, void *xt, int nrhs, double *corr) {
  return guarded([&] {
    LQCD_CHECK(c, LQCD_EINVAL, "pert_subtract: null context");
    LQCD_CHECK(order >= 0 && order <= kMaxOrder, LQCD_EINVAL, "pert_subtract: order %d outside 0..%d",
               order, kMaxOrder);
    LQCD_CHECK(nrhs >= 0 && (nrhs == 0 || (eta && xt)), LQCD_EINVAL, "pert_subtract: null field");
    check_thetas(thetas, nth);
    std::vector<cdouble> coeffs(order + 1, cdouble(1, 0));
    apply_poly_lex(c, coeffs, eta, xt, nrhs);
    if (corr) poly_trace(c, coeffs, thetas, nth, corr);
  });
}

extern "C" lqcd_status poly_subtract(lqcd_ctx *c, int degree, const void *b, double *coeffs_host,
                                     double *a_host, const int *thetas, int nth, const void *eta,
                                     void *xt, int nrhs, double *corr) {
  return guarded([&] {
    LQCD_CHECK(c && coeffs_host, LQCD_EINVAL, "poly_subtract: null argument");
    LQCD_CHECK(degree >= 0 && degree <= kMaxOrder, LQCD_EINVAL, "poly_subtract: degree %d outside 0..%d",
               degree, kMaxOrder);
    LQCD_CHECK(nrhs >= 0 && (nrhs == 0 || (eta && xt)), LQCD_EINVAL, "poly_subtract: null field");
    check_thetas(thetas, nth);
    const int d1 = degree + 1;
    const size_t fl = full_len(c->g), hl = half_len(c->g);
    std::vector<cdouble> cc(d1);
    if (b) {
      // Columns w_j = M (kappa P)^j b = y_j - y_{j+1} with y_{j+1} = kappa P y_j.
      cx<double> *Y = static_cast<cx<double> *>(c->ws[3].ensure(fl * (d1 + 1) * sizeof(cx<double>)));
      cx<double> *Wc = static_cast<cx<double> *>(c->ws[4].ensure(fl * (d1 + 1) * sizeof(cx<double>)));
      pack_eo<double>(c, b, Y, 1, fl);
      for (int j = 0; j < d1; ++j)
        for (int p = 0; p < 2; ++p)
          hop_half<double>(c, p, Y + j * fl + (1 - p) * hl, nullptr, Y + (j + 1) * fl + p * hl,
                           cdouble(0, 0), c->kappa, false, false, 1, fl, 0, fl);
      cdouble one(1, 0), mone(-1, 0);
      for (int j = 0; j < d1; ++j) {  // W_j = y_j - y_{j+1}
        cdouble z(0, 0);
        axpby<double>(c, &one, Y + j * fl, 0, &z, Wc + j * fl, 0, fl, 1, false);
        axpby<double>(c, &mone, Y + (j + 1) * fl, 0, &one, Wc + j * fl, 0, fl, 1, false);
      }
      // b in the last slot of Wc (packed copy of y_0)
      cdouble z(0, 0);
      axpby<double>(c, &one, Y, 0, &z, Wc + d1 * fl, 0, fl, 1, false);
      // Gram matrix G = W^H W and g = W^H b, then FP64 normal equations with
      // one step of iterative refinement on the residual b - W c.
      cdouble *Gd = static_cast<cdouble *>(c->ws[5].ensure(size_t(d1 + 1) * d1 * sizeof(cdouble)));
      gemm_tn<double>(c, Wc, fl, d1, Wc, fl, d1 + 1, fl, Gd, d1);
      std::vector<cdouble> Gh(size_t(d1) * (d1 + 1));
      d2h(c, Gh.data(), Gd, Gh.size() * sizeof(cdouble));
      la::Mat G(d1, d1);
      std::vector<cdouble> g(d1);
      for (int j = 0; j < d1; ++j) {
        for (int i = 0; i < d1; ++i) G(i, j) = Gh[size_t(j) * d1 + i];
        g[j] = Gh[size_t(d1) * d1 + j];
      }
      cc = la::solve(G, g);
      // refinement: r = b - W c; c += G^{-1} W^H r
      cdouble *cd_dev = static_cast<cdouble *>(c->ws[6].ensure(size_t(d1) * sizeof(cdouble)));
      cx<double> *Rb = Y + d1 * fl;  // reuse y_{d+1} slot for the residual
      axpby<double>(c, &one, Y, 0, &z, Rb, 0, fl, 1, false);
      h2d(c, cd_dev, cc.data(), d1 * sizeof(cdouble));
      gemm_nn<double>(c, Wc, fl, 0, d1, cd_dev, d1, 0, Rb, fl, 0, 1, fl, 1, -1.0);
      gemm_tn<double>(c, Wc, fl, d1, Rb, fl, 1, fl, Gd, d1);
      std::vector<cdouble> gr(d1);
      d2h(c, gr.data(), Gd, d1 * sizeof(cdouble));
      std::vector<cdouble> dc = la::solve(G, gr);
      for (int j = 0; j < d1; ++j) cc[j] += dc[j];
      for (int j = 0; j < d1; ++j) {
        coeffs_host[2 * j] = cc[j].real();
        coeffs_host[2 * j + 1] = cc[j].imag();
      }
    } else {
      for (int j = 0; j < d1; ++j) cc[j] = cdouble(coeffs_host[2 * j], coeffs_host[2 * j + 1]);
    }
    if (a_host) {
      std::vector<cdouble> a = kp_to_m(cc);
      for (int j = 0; j < d1; ++j) {
        a_host[2 * j] = a[j].real();
        a_host[2 * j + 1] = a[j].imag();
      }
    }
    apply_poly_lex(c, cc, eta, xt, nrhs);
    if (corr) poly_trace(c, cc, thetas, nth, corr);
  });
}

extern "C" lqcd_status poly_subtract_multi(lqcd_ctx *c, int npoly, int degree, const double *coeffs_host,
                                           const void *eta, void *const *xt_list, int nrhs) {
  return guarded([&] {
    LQCD_CHECK(c && coeffs_host, LQCD_EINVAL, "poly_subtract_multi: null argument");
    LQCD_CHECK(npoly >= 1 && npoly <= kMaxPolys, LQCD_EINVAL, "poly_subtract_multi: %d polynomials (1..%d)",
               npoly, kMaxPolys);
    LQCD_CHECK(degree >= 0 && degree <= kMaxOrder, LQCD_EINVAL,
               "poly_subtract_multi: degree %d outside 0..%d", degree, kMaxOrder);
    LQCD_CHECK(nrhs >= 0, LQCD_EINVAL, "poly_subtract_multi: negative count");
    if (nrhs == 0) return;
    LQCD_CHECK(eta && xt_list, LQCD_EINVAL, "poly_subtract_multi: null field");
    for (int a = 0; a < npoly; ++a) LQCD_CHECK(xt_list[a], LQCD_EINVAL, "poly_subtract_multi: null field");
    const int d1 = degree + 1;
    PolySet ps{};
    for (int a = 0; a < npoly; ++a)
      for (int j = 0; j < d1; ++j)
        ps.c[a][j] = mk(coeffs_host[2 * (a * d1 + j)], coeffs_host[2 * (a * d1 + j) + 1]);
    LQCD_CHECK(c->g.L[0] % 2 == 0, LQCD_EINVAL, "poly_subtract_multi: odd x extent");
    const size_t fl = full_len(c->g), hl = half_len(c->g);
    for (int r0 = 0; r0 < nrhs; r0 += kSubBlock) {
      const int nb = std::min(kSubBlock, nrhs - r0);
      const size_t blk = fl * nb;
      cx<double> *W = static_cast<cx<double> *>(c->ws[0].ensure(blk * d1 * sizeof(cx<double>)));
      pack_eo<double>(c, static_cast<const cdouble *>(eta) + r0 * fl, W, nb, fl);
      for (int j = 0; j < degree; ++j)
        for (int p = 0; p < 2; ++p)
          hop_half<double>(c, p, W + j * blk + (1 - p) * hl, nullptr, W + (j + 1) * blk + p * hl, cdouble(0, 0),
                           c->kappa, false, false, nb, fl, 0, fl);
      for (int a = 0; a < npoly; ++a) ps.out[a] = static_cast<cx<double> *>(xt_list[a]) + r0 * fl;
      const dim3 grid((c->g.V + kPolySites - 1) / kPolySites, nb);
      switch (npoly) {
        case 1: hipLaunchKernelGGL(k_poly_lex<1>, grid, dim3(kBlock), 0, c->stream, c->g, W, fl, blk, d1, ps); break;
        case 2: hipLaunchKernelGGL(k_poly_lex<2>, grid, dim3(kBlock), 0, c->stream, c->g, W, fl, blk, d1, ps); break;
        case 3: hipLaunchKernelGGL(k_poly_lex<3>, grid, dim3(kBlock), 0, c->stream, c->g, W, fl, blk, d1, ps); break;
        default: hipLaunchKernelGGL(k_poly_lex<4>, grid, dim3(kBlock), 0, c->stream, c->g, W, fl, blk, d1, ps); break;
      }
      LQCD_HIP(hipGetLastError());
    }
  });
}

extern "C" lqcd_status deflate_project_multi(lqcd_ctx *c, lqcd_defl *d, int Q, int nvar, const int *modes,
                                             const double *const *coeffs_list, const int *ncoeffs,
                                             const int *thetas, int nth, const void *eta, void *const *xt_list,
                                             int nrhs, double *const *corr_list) {
  return guarded([&] {
    LQCD_CHECK(c && d && modes, LQCD_EINVAL, "deflate_project_multi: null argument");
    LQCD_CHECK(nvar >= 1 && nvar <= kMaxHfVariants, LQCD_EINVAL, "deflate_project_multi: %d variants (1..%d)",
               nvar, kMaxHfVariants);
    LQCD_CHECK(nrhs >= 0 && (nrhs == 0 || (eta && xt_list)), LQCD_EINVAL, "deflate_project_multi: null field");
    for (int v = 0; v < nvar; ++v) {
      LQCD_CHECK(modes[v] == LQCD_DEFL_HFES || modes[v] == LQCD_DEFL_EIGPOLY, LQCD_EINVAL,
                 "deflate_project_multi: variant %d: mode must be HFES or EIGPOLY", v);
      LQCD_CHECK(modes[v] != LQCD_DEFL_EIGPOLY || (coeffs_list && ncoeffs && coeffs_list[v] && ncoeffs[v] >= 1 &&
                                                   ncoeffs[v] <= kMaxOrder + 1),
                 LQCD_EINVAL, "deflate_project_multi: variant %d: EIGPOLY needs 1..%d coefficients", v,
                 kMaxOrder + 1);
      LQCD_CHECK(nrhs == 0 || xt_list[v], LQCD_EINVAL, "deflate_project_multi: variant %d: null field", v);
    }
    for (int i = 0; i < 4; ++i)
      LQCD_CHECK(d->dims[i] == c->g.L[i], LQCD_EINVAL, "deflate_project_multi: deflation space of another lattice");
    LQCD_CHECK(d->kappa == c->kappa, LQCD_EINVAL, "deflate_project_multi: deflation space of another kappa");
    check_thetas(thetas, nth);
    defl_eigpairs(c, d, Q);
    std::vector<std::vector<cdouble>> w(nvar);
    for (int v = 0; v < nvar; ++v) {
      const bool poly = modes[v] == LQCD_DEFL_EIGPOLY;
      w[v] = hf_weights(c, d, Q, lqcd_defl_mode(modes[v]), poly ? coeffs_list[v] : nullptr, poly ? ncoeffs[v] : 0,
                        thetas, nth, corr_list ? corr_list[v] : nullptr, nullptr);
    }
    hf_update(c, d, Q, eta, nvar, xt_list, w.data(), nrhs);
  });
}

extern "C" lqcd_status deflate_project(lqcd_ctx *c, lqcd_defl *d, int Q, lqcd_defl_mode mode,
                                       const double *coeffs_host, int ncoeff, const int *thetas,
                                       int nth, const void *eta, void *xt, int nrhs,
                                       double *corr, double *xi_inv_host) {
  return guarded([&] {
    LQCD_CHECK(c && d, LQCD_EINVAL, "deflate_project: null argument");
    LQCD_CHECK(mode == LQCD_DEFL_HFES || mode == LQCD_DEFL_EIGPOLY || mode == LQCD_DEFL_ES, LQCD_EINVAL,
               "deflate_project: bad mode");
    LQCD_CHECK(nrhs >= 0 && (nrhs == 0 || (eta && xt)), LQCD_EINVAL, "deflate_project: null field");
    LQCD_CHECK(mode != LQCD_DEFL_EIGPOLY || (coeffs_host && ncoeff >= 1 && ncoeff <= kMaxOrder + 1),
               LQCD_EINVAL, "deflate_project: EIGPOLY needs 1..%d polynomial coefficients", kMaxOrder + 1);
    for (int i = 0; i < 4; ++i)
      LQCD_CHECK(d->dims[i] == c->g.L[i], LQCD_EINVAL, "deflate_project: deflation space of another lattice");
    LQCD_CHECK(d->kappa == c->kappa, LQCD_EINVAL, "deflate_project: deflation space of another kappa");
    check_thetas(thetas, nth);
    if (mode == LQCD_DEFL_ES) {
      es_project(c, d, Q, thetas, nth, eta, xt, nrhs, corr);
      if (xi_inv_host)
        for (int q = 0; q < Q; ++q) {  // the eigenvalues of M used, in place of 1/xi'
          xi_inv_host[2 * q] = d->es_lam[q].real();
          xi_inv_host[2 * q + 1] = d->es_lam[q].imag();
        }
      return;
    }
    defl_eigpairs(c, d, Q);
    const std::vector<cdouble> w =
        hf_weights(c, d, Q, mode, coeffs_host, ncoeff, thetas, nth, corr, xi_inv_host);
    hf_update(c, d, Q, eta, 1, &xt, &w, nrhs);
  });
}
