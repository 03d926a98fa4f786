// Batched deflated solves over several lattices at once (the batching axis
// of the method's growth; the paper solves one configuration at a time).
//
// The right-hand sides of every lattice are flattened into one queue and
// taken rhs_block at a time into "slots": a slot is one right-hand side of
// one lattice, whatever the lattice's size.  A device table of slot
// descriptors (geometry, links, vector pointers, deflation basis) drives
// every kernel of the inner solve, so one launch serves all slots:
//   - the stencil is a persistent kernel over a flat work list of (slot,
//     256-site block) items, so lattices of different sizes and uneven
//     right-hand-side counts share the launch;
//   - Gram-Schmidt dots, updates, norms and basis products are batched over
//     slots with per-slot vector lengths.
// The FP32 GMRES(p) cycle of GMRES-Proj (start vector plus p Arnoldi steps,
// all decisions on the device) is captured once into a hipGraph and
// replayed every cycle; between cycles the host solves the small
// least-squares problems, applies the deflation projection (Sec. 7) and
// retires converged slots by clearing their active flag in the table.
// Around it, FP64 iterative refinement per slot as in the single-lattice
// mixed-precision solver.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>

#include "cplx.h"
#include "fields.h"
#include "solver.h"
#include "stencil.h"

namespace lqcd {
namespace {

using namespace st;

constexpr int kWaves = kBlock / 64;

struct BSlot {
  Geom g;
  const cx<float> *U;   // FP32 links of the slot's lattice, [parity][mu][9][Vh]
  float mk2;            // -kappa^2 of the lattice
  int active;           // 0: every kernel skips the slot
  int kd;               // deflation vectors (the basis holds kd + 1)
  size_t n;             // vector length 12 Vh
  cx<float> *W;         // GMRES basis, p + 1 vectors n apart
  cx<float> *T;         // odd-site temporary
  cx<float> *X, *R, *S; // inner correction, residual, right-hand side
  const cx<float> *Vd;  // deflation basis V_{kd+1} (FP32)
};

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------- stencil
// Modes: which operands of a slot the half hop reads and writes.
enum HopMode { HOP_W = 0, SCHUR_W = 1, HOP_X = 2, SCHUR_X = 3 };

// Work item = (256-site block, slot); every slot owns `per` site blocks
// (enough for the largest lattice), so the list does not depend on which
// lattice a slot holds and a captured launch stays valid when slots are
// refilled.  The slot index runs fastest and the list is cut into one
// contiguous range per XCD (workgroup h runs on XCD h % 8): the slots of a
// site block, mostly right-hand sides of one lattice, run back to back on
// one XCD and share that block's links in its L2.
template <int MODE>
__global__ void __launch_bounds__(kBlock)
    k_bhop(const BSlot *__restrict__ sl, unsigned nslot, unsigned nitems, int j) {
  const unsigned xq = (nitems + 7) / 8;
  for (unsigned h = blockIdx.x; h < 8 * xq; h += gridDim.x) {
    const unsigned item = (h % 8) * xq + h / 8;
    if (item >= nitems) continue;
    const unsigned s = item % nslot;
    const BSlot &d = sl[s];
    if (!d.active) continue;
    const int i = int(item / nslot) * kBlock + threadIdx.x;
    const Geom &g = d.g;
    if (i >= g.Vh) continue;
    const size_t Vh = size_t(g.Vh), n = d.n;
    // operands: out_p = alpha self + beta D_{p,1-p} in
    constexpr int p = (MODE == HOP_W || MODE == HOP_X) ? 1 : 0;
    const cx<float> *in;
    const cx<float> *self = nullptr;
    cx<float> *out;
    if (MODE == HOP_W) {
      in = d.W + size_t(j) * n;
      out = d.T;
    } else if (MODE == SCHUR_W) {
      in = d.T;
      self = d.W + size_t(j) * n;
      out = d.W + size_t(j + 1) * n;
    } else if (MODE == HOP_X) {
      in = d.X;
      out = d.T;
    } else {
      in = d.T;
      self = d.X;
      out = d.R;
    }
    const int Lxh = g.Lxh, Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const int xh = i % Lxh;
    int r = i / Lxh;
    const int y = r % Ly;
    r /= Ly;
    const int z = r % Lz;
    const int t = r / Lz;
    const int x = 2 * xh + ((p + y + z + t) & 1);
    const int rowb = i - xh;
    cx<float> acc[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[a][c] = mk(0.f, 0.f);
    const SrcPlain<float> src{in};
    {
      int xf = (x + 1 == Lx) ? 0 : x + 1, xb = (x == 0) ? Lx - 1 : x - 1;
      hop_dir<float, 0, false>(acc, d.U, src, p, i, rowb + (xf >> 1), rowb + (xb >> 1), Vh);
    }
    {
      const int st = Lxh;
      hop_dir<float, 1, false>(acc, d.U, src, p, i, (y == Ly - 1) ? i - st * (Ly - 1) : i + st,
                               (y == 0) ? i + st * (Ly - 1) : i - st, Vh);
    }
    {
      const int st = Lxh * Ly;
      hop_dir<float, 2, false>(acc, d.U, src, p, i, (z == Lz - 1) ? i - st * (Lz - 1) : i + st,
                               (z == 0) ? i + st * (Lz - 1) : i - st, Vh);
    }
    {
      const int st = Lxh * Ly * Lz;
      hop_dir<float, 3, false>(acc, d.U, src, p, i, (t == Lt - 1) ? i - st * (Lt - 1) : i + st,
                               (t == 0) ? i + st * (Lt - 1) : i - st, Vh);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cx<float> v = acc[a][c];
        if (self) {
          const cx<float> w = ldc(self + (a * 3 + c) * Vh + i);
          v = w + d.mk2 * v;
        }
        stc(out + (a * 3 + c) * Vh + i, v);
      }
  }
}

// ------------------------------------------------- batched reductions
// Basis selection: BAS_W = W_0 .. W_{J-1} against W_{j+1} (Arnoldi),
// BAS_V = Vd_0 .. Vd_{kd} against R (deflation projection).
enum BasisSel { BAS_W = 0, BAS_V = 1 };
constexpr int kEpt = 16;  // elements per lane
constexpr int kWch = 64 * kEpt;

// part[(s * nchunk + chunk) * Jmax + jj] (complex) = partial dot of
// wave chunk `chunk` of slot s.
template <int SEL>
__global__ void __launch_bounds__(kBlock)
    k_bdot_part(const BSlot *__restrict__ sl, int jnew, int Jw, int Jmax, size_t nchunk,
                cx<double> *__restrict__ part, const int *__restrict__ flag) {
  const int s = blockIdx.y;
  const BSlot &d = sl[s];
  const int lane = threadIdx.x & 63;
  const size_t chunk = size_t(blockIdx.x) * kWaves + (threadIdx.x >> 6);
  const int J = SEL == BAS_W ? Jw : d.kd + 1;
  cx<double> *po = part + (size_t(s) * nchunk + chunk) * Jmax;
  const bool on = d.active && (!flag || flag[s]) && chunk * kWch < d.n;
  if (!on) {
    if (lane == 0)
      for (int jj = 0; jj < Jmax; ++jj) po[jj] = mk(0.0, 0.0);
    return;
  }
  const size_t n = d.n;
  const cx<float> *w = SEL == BAS_W ? d.W + size_t(jnew) * n : d.R;
  const cx<float> *V = SEL == BAS_W ? d.W : d.Vd;
  const size_t base = chunk * kWch + lane;
  cx<double> wv[kEpt];
#pragma unroll
  for (int e = 0; e < kEpt; ++e) {
    const size_t idx = base + size_t(e) * 64;
    const cx<float> v = idx < n ? ldc(w + idx) : mk(0.f, 0.f);
    wv[e] = mk<double>(v.re, v.im);
  }
  int jj = 0;
  for (; jj + 2 <= J; jj += 2) {  // two basis vectors per pass
    double a0 = 0, b0 = 0, a1 = 0, b1 = 0;
    const cx<float> *v0 = V + size_t(jj) * n, *v1 = v0 + n;
#pragma unroll
    for (int e = 0; e < kEpt; ++e) {
      const size_t idx = base + size_t(e) * 64;
      if (idx < n) {
        const cx<float> q0 = ldc_nt(v0 + idx), q1 = ldc_nt(v1 + idx);  // streamed basis
        const cx<double> p0 = cmulc(mk<double>(q0.re, q0.im), wv[e]);
        const cx<double> p1 = cmulc(mk<double>(q1.re, q1.im), wv[e]);
        a0 += p0.re;
        b0 += p0.im;
        a1 += p1.re;
        b1 += p1.im;
      }
    }
    a0 = wave_sum(a0);
    b0 = wave_sum(b0);
    a1 = wave_sum(a1);
    b1 = wave_sum(b1);
    if (lane == 0) {
      po[jj] = mk(a0, b0);
      po[jj + 1] = mk(a1, b1);
    }
  }
  for (; jj < Jmax; ++jj) {
    double a = 0, b = 0;
    if (jj < J) {
      const cx<float> *v0 = V + size_t(jj) * n;
#pragma unroll
      for (int e = 0; e < kEpt; ++e) {
        const size_t idx = base + size_t(e) * 64;
        if (idx < n) {
          const cx<float> q = ldc_nt(v0 + idx);
          const cx<double> pr = cmulc(mk<double>(q.re, q.im), wv[e]);
          a += pr.re;
          b += pr.im;
        }
      }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) po[jj] = mk(a, b);
  }
}

// out[s * Jmax + jj] = sum over chunks; one block per (jj, s).
__global__ void __launch_bounds__(kBlock)
    k_bdot_final(const cx<double> *__restrict__ part, size_t nchunk, int Jmax,
                 cx<double> *__restrict__ out) {
  __shared__ double sh[2][kWaves];
  const int jj = blockIdx.x, s = blockIdx.y;
  double a = 0, b = 0;
  for (size_t c = threadIdx.x; c < nchunk; c += kBlock) {
    const cx<double> v = part[(size_t(s) * nchunk + c) * Jmax + jj];
    a += v.re;
    b += v.im;
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
    double ra = 0, rb = 0;
    for (int w = 0; w < kWaves; ++w) {
      ra += sh[0][w];
      rb += sh[1][w];
    }
    out[size_t(s) * Jmax + jj] = mk(ra, rb);
  }
}

// Vector updates with per-slot coefficients (coef[s * ldc + jj]):
//   UPD_ORTH:  W_{j+1} -= sum_{jj<J} W_jj c_jj        (+ |W_{j+1}|^2 partials)
//   UPD_XW:    X += sum_{jj<J} W_jj c_jj
//   UPD_XV:    X += sum_{jj<kd} Vd_jj c_jj
//   UPD_RV:    R -= sum_{jj<=kd} Vd_jj c_jj
enum UpdSel { UPD_ORTH = 0, UPD_XW = 1, UPD_XV = 2, UPD_RV = 3 };
constexpr int kAept = 4;
constexpr int kBatchMaxJ = 256;  // basis vectors of one update (p + 1 <= 251, kd + 1 <= 251)

template <int SEL>
__global__ void __launch_bounds__(kBlock)
    k_bupdate(const BSlot *__restrict__ sl, int jnew, int Jw, const cx<double> *__restrict__ coef,
              int ldcf, double *__restrict__ part, size_t nblk, const int *__restrict__ flag) {
  __shared__ double sh[kWaves];
  __shared__ cx<double> sc[kBatchMaxJ];
  const int s = blockIdx.y;
  const BSlot &d = sl[s];
  const size_t b = blockIdx.x;
  const bool on = d.active && (!flag || flag[s]) && b * kBlock * kAept < d.n;  // uniform per workgroup
  double nrm = 0;
  if (on) {
    const size_t n = d.n;
    cx<float> *w;
    const cx<float> *V;
    int J;
    double sign;
    if (SEL == UPD_ORTH) {
      w = d.W + size_t(jnew) * n;
      V = d.W;
      J = Jw;
      sign = -1;
    } else if (SEL == UPD_XW) {
      w = d.X;
      V = d.W;
      J = Jw;
      sign = 1;
    } else if (SEL == UPD_XV) {
      w = d.X;
      V = d.Vd;
      J = d.kd;
      sign = 1;
    } else {
      w = d.R;
      V = d.Vd;
      J = d.kd + 1;
      sign = -1;
    }
    // the coefficients (times the sign) from LDS, not one scalar load and
    // its wait per pass
    for (int t = threadIdx.x; t < J; t += kBlock) sc[t] = sign * coef[size_t(s) * ldcf + t];
    __syncthreads();
    const cx<double> *cf = sc;
    const size_t base = b * kBlock * kAept + threadIdx.x;
    cx<double> acc[kAept];
#pragma unroll
    for (int e = 0; e < kAept; ++e) {
      const size_t idx = base + size_t(e) * kBlock;
      const cx<float> v = idx < n ? ldc(w + idx) : mk(0.f, 0.f);
      acc[e] = mk<double>(v.re, v.im);
    }
    int jj = 0;
    for (; jj + 4 <= J; jj += 4) {  // four basis vectors per pass: 16 loads in flight per lane
      const cx<double> c0 = cf[jj], c1 = cf[jj + 1], c2 = cf[jj + 2], c3 = cf[jj + 3];
      const cx<float> *v0 = V + size_t(jj) * n;
#pragma unroll
      for (int e = 0; e < kAept; ++e) {
        const size_t idx = base + size_t(e) * kBlock;
        if (idx < n) {
          const cx<float> q0 = ldc_nt(v0 + idx), q1 = ldc_nt(v0 + n + idx), q2 = ldc_nt(v0 + 2 * n + idx),
                          q3 = ldc_nt(v0 + 3 * n + idx);  // streamed basis
          acc[e] = acc[e] + (mk<double>(q0.re, q0.im) * c0 + mk<double>(q1.re, q1.im) * c1) +
                   (mk<double>(q2.re, q2.im) * c2 + mk<double>(q3.re, q3.im) * c3);
        }
      }
    }
    for (; jj < J; ++jj) {
      const cx<double> c = cf[jj];
      const cx<float> *v0 = V + size_t(jj) * n;
#pragma unroll
      for (int e = 0; e < kAept; ++e) {
        const size_t idx = base + size_t(e) * kBlock;
        if (idx < n) {
          const cx<float> q = ldc_nt(v0 + idx);
          acc[e] = acc[e] + mk<double>(q.re, q.im) * c;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < kAept; ++e) {
      const size_t idx = base + size_t(e) * kBlock;
      if (idx < n) {
        const cx<float> st = mk(float(acc[e].re), float(acc[e].im));
        stc(w + idx, st);
        nrm += double(st.re) * st.re + double(st.im) * st.im;
      }
    }
  }
  if (SEL == UPD_ORTH && part) {
    nrm = wave_sum(nrm);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int w = 0; w < kWaves; ++w) t += sh[w];
      part[size_t(s) * nblk + b] = t;
    }
  }
}

// |v|^2 partials of R (SEL 0) per slot.
__global__ void __launch_bounds__(kBlock)
    k_bnorm_part(const BSlot *__restrict__ sl, double *__restrict__ part, size_t nblk) {
  __shared__ double sh[kWaves];
  const int s = blockIdx.y;
  const BSlot &d = sl[s];
  const size_t b = blockIdx.x;
  double nrm = 0;
  if (d.active) {
    const size_t base = b * kBlock * kAept + threadIdx.x;
#pragma unroll
    for (int e = 0; e < kAept; ++e) {
      const size_t idx = base + size_t(e) * kBlock;
      if (idx < d.n) {
        const cx<float> v = ldc(d.R + idx);
        nrm += double(v.re) * v.re + double(v.im) * v.im;
      }
    }
  }
  nrm = wave_sum(nrm);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < kWaves; ++w) t += sh[w];
    part[size_t(s) * nblk + b] = t;
  }
}

__global__ void __launch_bounds__(kBlock)
    k_bsum_final(const double *__restrict__ part, size_t nblk, double *__restrict__ out,
                 const int *__restrict__ flag) {
  __shared__ double sh[kWaves];
  const int s = blockIdx.x;
  if (flag && flag[s] == 0) return;
  double a = 0;
  for (size_t c = threadIdx.x; c < nblk; c += kBlock) a += part[size_t(s) * nblk + c];
  a = wave_sum(a);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < kWaves; ++w) t += sh[w];
    out[s] = t;
  }
}

// Second Gram-Schmidt pass test (DGKS, as the single-lattice solver).
__global__ void k_bdgks(const cx<double> *__restrict__ h1, int ldh, int J,
                        const double *__restrict__ nrm1, int *__restrict__ flag, double eta2) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= gridDim.x * blockDim.x) return;
  double hh = 0;
  for (int i = 0; i < J; ++i) {
    const cx<double> v = h1[size_t(s) * ldh + i];
    hh += v.re * v.re + v.im * v.im;
  }
  flag[s] = nrm1[s] < eta2 * (nrm1[s] + hh) ? 1 : 0;
}

// Column j of each slot's Hessenberg matrix (ldh = p + 1 rows, Hrs apart)
// and 1 / h_{j+1,j}.
__global__ void k_bfinish(cx<double> *__restrict__ H, size_t Hrs, int ldh, int j,
                          const cx<double> *__restrict__ h1, const cx<double> *__restrict__ h2,
                          int ldhh, const double *__restrict__ nrm1, const double *__restrict__ nrm2,
                          const int *__restrict__ flag, double *__restrict__ inv) {
  const int s = blockIdx.x;
  const bool two = flag[s] != 0;
  cx<double> *col = H + size_t(s) * Hrs + size_t(j) * ldh;
  for (int i = threadIdx.x; i <= j; i += blockDim.x)
    col[i] = two ? h1[size_t(s) * ldhh + i] + h2[size_t(s) * ldhh + i] : h1[size_t(s) * ldhh + i];
  if (threadIdx.x == 0) {
    const double nr = sqrt(two ? nrm2[s] : nrm1[s]);
    col[j + 1] = mk(nr, 0.0);
    inv[s] = (nr > 0 && isfinite(nr)) ? 1.0 / nr : 0.0;
  }
}

// W_{j} *= inv[s] (SEL 0) or W_0 = R / |R| (SEL 1, inv = 1 / sqrt(nrm)).
template <int SEL>
__global__ void __launch_bounds__(kBlock)
    k_bscale(const BSlot *__restrict__ sl, int j, const double *__restrict__ v) {
  const int s = blockIdx.y;
  const BSlot &d = sl[s];
  if (!d.active) return;
  double f = v[s];
  if (SEL == 1) f = (f > 0 && isfinite(f)) ? 1.0 / sqrt(f) : 0.0;
  const float ff = float(f);
  const cx<float> *src = SEL == 1 ? d.R : d.W + size_t(j) * d.n;
  cx<float> *dst = d.W + size_t(j) * d.n;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < d.n; i += size_t(gridDim.x) * kBlock) {
    const cx<float> q = ldc(src + i);
    stc(dst + i, mk(ff * q.re, ff * q.im));
  }
}

// R = S - R (after R = Mhat X)
__global__ void __launch_bounds__(kBlock) k_bresid(const BSlot *__restrict__ sl) {
  const int s = blockIdx.y;
  const BSlot &d = sl[s];
  if (!d.active) return;
  for (size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x; i < d.n; i += size_t(gridDim.x) * kBlock)
    stc(d.R + i, ldc(d.S + i) - ldc(d.R + i));
}

// y (FP64) += x (FP32); and the FP64 -> FP32 copy.
__global__ void k_widen_add(const cx<float> *__restrict__ x, cx<double> *__restrict__ y, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    const cx<float> v = x[i];
    const cx<double> w = y[i];
    y[i] = mk(w.re + double(v.re), w.im + double(v.im));
  }
}

__global__ void k_fill0(cx<float> *__restrict__ x, size_t n) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    x[i] = mk(0.f, 0.f);
}

}  // namespace
}  // namespace lqcd

using namespace lqcd;

// ------------------------------------------------------------- the batch
struct lqcd_batch {
  std::vector<lqcd_ctx *> ctx;
  hipStream_t stream = nullptr;
  // per-slot buffers, grown on demand
  DevBuf slots_dev, part, part2, hd, Hd, nrm1, nrm2, inv, flag, coef;
  DevBuf W, T, X, R, S, S64, X64, R64, Bp, XF, TF;
  // captured inner cycle
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int hop_grid = 8192;  // persistent stencil workgroups per launch (tunable)
  int tile = 0;         // 0: one persistent slot-table stencil launch; 16/32/64: link tiles per lattice group
  // Capture needs a stream other than the legacy null stream; the graph
  // is recorded on this private one (default priority) and launched on
  // the contexts' stream.
  hipStream_t capture = nullptr;
  ~lqcd_batch() {
    if (capture) (void)hipStreamDestroy(capture);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace lqcd {
namespace {

void d2h_b(lqcd_batch *b, void *dst, const void *src, size_t bytes) {
  LQCD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, b->stream));
  LQCD_HIP(hipStreamSynchronize(b->stream));
}
void h2d_b(lqcd_batch *b, void *dst, const void *src, size_t bytes) {
  LQCD_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->stream));
  LQCD_HIP(hipStreamSynchronize(b->stream));
}

inline unsigned grid_n(size_t n) { return unsigned(std::min<size_t>((n + kBlock - 1) / kBlock, 4096)); }

// A run of consecutive slots that hold right-hand sides of one lattice:
// their vectors lie at one stride from each other, so the single-lattice
// link-tiled stencil serves them in one launch (links staged once per tile
// for all of them).
struct Group {
  lqcd_ctx *c;
  int s0, G;
  size_t n;
};

// Runs of one lattice in a slot-to-lattice map (-1: empty slot).
std::vector<Group> lattice_groups(const std::vector<lqcd_ctx *> &ctx, const std::vector<int> &lat,
                                  const std::vector<size_t> &n) {
  std::vector<Group> g;
  for (int s = 0; s < int(lat.size()); ++s) {
    if (lat[s] < 0) continue;
    if (!g.empty() && lat[s - 1] == lat[s] && g.back().s0 + g.back().G == s)
      ++g.back().G;
    else
      g.push_back(Group{ctx[lat[s]], s, 1, n[s]});
  }
  return g;
}

// Launches of a context's stencil on the batch's current stream (the
// capture stream while a cycle is being recorded) with the batch's tile
// size and the context's event timer off; restored on exit.
struct OnBatchStream {
  lqcd_ctx *c;
  hipStream_t keep;
  int keep_ts;
  bool keep_timer;
  OnBatchStream(lqcd_ctx *cc, hipStream_t s, int ts)
      : c(cc), keep(cc->stream), keep_ts(cc->hop_tsites[1]), keep_timer(cc->timer.on) {
    c->stream = s;
    c->hop_tsites[1] = ts;
    c->timer.on = false;
  }
  ~OnBatchStream() {
    c->stream = keep;
    c->hop_tsites[1] = keep_ts;
    c->timer.on = keep_timer;
  }
};

// Device work of the batched inner solve, shared by the eager and the
// captured paths.  B slots, basis length p, longest vector nmax.  The
// stencil is one persistent launch over the slot table (tile == 0) or,
// with link tiles, one launch of the link-tiled stencil per lattice group
// (its groups are fixed while a block of slots is in flight; inactive
// slots of a group are computed and ignored).
struct Engine {
  lqcd_batch *b;
  int B, p;
  size_t nmax;
  unsigned per, items, hgrid;
  int kdmax;
  const BSlot *sl;
  int tile = 0;
  std::vector<Group> groups;
  cx<float> *W = nullptr, *T = nullptr, *X = nullptr, *R = nullptr;
  // longest vector of the block in flight (the grids of the batched
  // reductions and updates cover this much; slot buffers stay nmax apart)
  size_t nlen = 0;
  size_t nchunk() const { return (nlen + size_t(kWch) * kWaves - 1) / (size_t(kWch) * kWaves) * kWaves; }
  size_t nblk() const { return (nlen + size_t(kBlock) * kAept - 1) / (size_t(kBlock) * kAept); }
  unsigned hop_grid() const { return std::min<unsigned>((items + 7) / 8 * 8, hgrid); }

  void stencil_schur_w(int j) const {
    if (tile > 0) {
      const size_t ws = size_t(p + 1) * nmax;  // slot stride of the bases
      for (const Group &g : groups) {
        OnBatchStream on(g.c, b->stream, tile);
        cx<float> *w = W + size_t(g.s0) * ws;
        apply_schur<float>(g.c, w + size_t(j) * g.n, w + size_t(j + 1) * g.n, T + size_t(g.s0) * nmax, g.G, ws, ws,
                           nmax);
      }
      return;
    }
    hipLaunchKernelGGL(k_bhop<HOP_W>, dim3(hop_grid()), dim3(kBlock), 0, b->stream, sl, unsigned(B), items, j);
    hipLaunchKernelGGL(k_bhop<SCHUR_W>, dim3(hop_grid()), dim3(kBlock), 0, b->stream, sl, unsigned(B), items, j);
  }
  void stencil_schur_x() const {
    if (tile > 0) {
      for (const Group &g : groups) {
        OnBatchStream on(g.c, b->stream, tile);
        apply_schur<float>(g.c, X + size_t(g.s0) * nmax, R + size_t(g.s0) * nmax, T + size_t(g.s0) * nmax, g.G,
                           nmax, nmax, nmax);
      }
      return;
    }
    hipLaunchKernelGGL(k_bhop<HOP_X>, dim3(hop_grid()), dim3(kBlock), 0, b->stream, sl, unsigned(B), items, 0);
    hipLaunchKernelGGL(k_bhop<SCHUR_X>, dim3(hop_grid()), dim3(kBlock), 0, b->stream, sl, unsigned(B), items, 0);
  }
  // dots of the basis (W_0..W_{J-1} or Vd) against W_{jnew} or R into out [B][Jmax]
  template <int SEL>
  void dots(int jnew, int J, int Jmax, cx<double> *out, const int *flag) const {
    const size_t nc = nchunk();
    hipLaunchKernelGGL(k_bdot_part<SEL>, dim3(unsigned(nc / kWaves), B), dim3(kBlock), 0, b->stream, sl,
                       jnew, J, Jmax, nc, b->part.as<cx<double>>(), flag);
    hipLaunchKernelGGL(k_bdot_final, dim3(Jmax, B), dim3(kBlock), 0, b->stream, b->part.as<cx<double>>(), nc,
                       Jmax, out);
  }
  template <int SEL>
  void update(int jnew, int J, const cx<double> *coef, int ldcf, double *nrm_out, const int *flag) const {
    const size_t nb = nblk();
    hipLaunchKernelGGL(k_bupdate<SEL>, dim3(unsigned(nb), B), dim3(kBlock), 0, b->stream, sl, jnew, J, coef,
                       ldcf, nrm_out ? b->part2.as<double>() : nullptr, nb, flag);
    if (nrm_out)
      hipLaunchKernelGGL(k_bsum_final, dim3(B), dim3(kBlock), 0, b->stream, b->part2.as<double>(), nb, nrm_out,
                         flag);
  }
  void norm_r(double *out) const {
    const size_t nb = nblk();
    hipLaunchKernelGGL(k_bnorm_part, dim3(unsigned(nb), B), dim3(kBlock), 0, b->stream, sl,
                       b->part2.as<double>(), nb);
    hipLaunchKernelGGL(k_bsum_final, dim3(B), dim3(kBlock), 0, b->stream, b->part2.as<double>(), nb, out,
                       static_cast<const int *>(nullptr));
  }
  // One GMRES(p) cycle on every active slot: W_0 = R / |R|, then p Arnoldi
  // steps with DGKS-conditional second pass; column j of each slot's Hbar
  // in Hd, the starting norm^2 in nrm2[B + s].
  void cycle() const {
    cx<double> *Hd = b->Hd.as<cx<double>>();
    cx<double> *h1 = b->hd.as<cx<double>>(), *h2 = h1 + size_t(B) * (p + 1);
    double *n1 = b->nrm1.as<double>(), *n2 = b->nrm2.as<double>(), *iv = b->inv.as<double>();
    int *fl = b->flag.as<int>();
    const size_t Hrs = size_t(p + 1) * p;
    norm_r(n2 + B);
    hipLaunchKernelGGL(k_bscale<1>, dim3(grid_n(nlen), B), dim3(kBlock), 0, b->stream, sl, 0, n2 + B);
    for (int j = 0; j < p; ++j) {
      stencil_schur_w(j);
      dots<BAS_W>(j + 1, j + 1, p + 1, h1, nullptr);
      update<UPD_ORTH>(j + 1, j + 1, h1, p + 1, n1, nullptr);
      hipLaunchKernelGGL(k_bdgks, dim3(B), dim3(1), 0, b->stream, h1, p + 1, j + 1, n1, fl, 0.01);
      dots<BAS_W>(j + 1, j + 1, p + 1, h2, fl);
      update<UPD_ORTH>(j + 1, j + 1, h2, p + 1, n2, fl);
      hipLaunchKernelGGL(k_bfinish, dim3(B), dim3(64), 0, b->stream, Hd, Hrs, p + 1, j, h1, h2, p + 1, n1, n2,
                         fl, iv);
      hipLaunchKernelGGL(k_bscale<0>, dim3(grid_n(nlen), B), dim3(kBlock), 0, b->stream, sl, j + 1, iv);
    }
  }
};

}  // namespace
}  // namespace lqcd

namespace lqcd {
namespace {

constexpr int kBatchCycleCap = 20;   // GMRES(p) cycles per inner solve
constexpr int kTuneBlocks = 4, kTuneTiles = 4;  // autotuner trials: rhs_block x stencil form
constexpr double kBatchStall = 0.9;  // stop an inner solve when a cycle gains < 10%
constexpr int kBatchMaxRefine = 60;

struct SlotState {
  int lat = -1, rhs = -1;   // which right-hand side the slot holds
  bool done = true;         // FP64-converged (or empty)
  double ref = 0;           // |b| on the full lattice
  double rn = 0;            // current FP64 residual of the even/odd system
  lqcd_solve_stats st{0, 0, 0, 0, 0.0};
};

void run_batch(lqcd_batch *b, const lqcd_solve_params &prm, const void *const *bvec,
               void *const *xvec, const int *nrhs, lqcd_defl *const *defl, bool use_graph,
               lqcd_solve_stats *stats, int *nonconv) {
  const int nl = int(b->ctx.size());
  const int p = prm.proj_m > 0 ? prm.proj_m : prm.m - prm.k;
  const int B = std::max(1, std::min(prm.rhs_block, 64));
  // queue of (lattice, rhs); first stats index of each lattice
  std::vector<std::pair<int, int>> q;
  std::vector<size_t> first(nl, 0);
  for (int l = 0; l < nl; ++l) {
    first[l] = q.size();
    for (int r = 0; r < nrhs[l]; ++r) q.emplace_back(l, r);
  }
  if (q.empty()) return;
  size_t nmax = 0, flmax = 0;
  int Vhmax = 0, kdmax = 0;
  for (int l = 0; l < nl; ++l) {
    nmax = std::max(nmax, half_len(b->ctx[l]->g));
    flmax = std::max(flmax, full_len(b->ctx[l]->g));
    Vhmax = std::max(Vhmax, b->ctx[l]->g.Vh);
    kdmax = std::max(kdmax, defl[l]->k);
  }
  const unsigned per = unsigned((Vhmax + kBlock - 1) / kBlock);
  // buffers (grown, never shrunk)
  cx<float> *W = static_cast<cx<float> *>(b->W.ensure(size_t(B) * (p + 1) * nmax * sizeof(cx<float>)));
  cx<float> *T = static_cast<cx<float> *>(b->T.ensure(size_t(B) * nmax * sizeof(cx<float>)));
  cx<float> *X = static_cast<cx<float> *>(b->X.ensure(size_t(B) * nmax * sizeof(cx<float>)));
  cx<float> *R = static_cast<cx<float> *>(b->R.ensure(size_t(B) * nmax * sizeof(cx<float>)));
  cx<float> *S = static_cast<cx<float> *>(b->S.ensure(size_t(B) * nmax * sizeof(cx<float>)));
  cx<double> *S64 = static_cast<cx<double> *>(b->S64.ensure(size_t(B) * nmax * sizeof(cx<double>)));
  cx<double> *X64 = static_cast<cx<double> *>(b->X64.ensure(size_t(B) * nmax * sizeof(cx<double>)));
  cx<double> *R64 = static_cast<cx<double> *>(b->R64.ensure(size_t(B) * nmax * sizeof(cx<double>)));
  cx<double> *Bp = static_cast<cx<double> *>(b->Bp.ensure(size_t(B) * flmax * sizeof(cx<double>)));
  cx<double> *XF = static_cast<cx<double> *>(b->XF.ensure(size_t(B) * flmax * sizeof(cx<double>)));
  cx<double> *TF = static_cast<cx<double> *>(b->TF.ensure(size_t(B) * flmax * sizeof(cx<double>)));
  BSlot *sld = static_cast<BSlot *>(b->slots_dev.ensure(size_t(B) * sizeof(BSlot)));
  Engine e{b, B, p, nmax, per, unsigned(B) * per, unsigned(b->hop_grid), kdmax, sld};
  e.nlen = nmax;
  e.tile = b->tile;
  e.W = W;
  e.T = T;
  e.X = X;
  e.R = R;
  const size_t Jpart = size_t(std::max(p + 1, kdmax + 1));
  b->part.ensure(size_t(B) * e.nchunk() * Jpart * sizeof(cx<double>));
  b->part2.ensure(size_t(B) * e.nblk() * sizeof(double));
  b->hd.ensure(2 * size_t(B) * (p + 1) * sizeof(cx<double>));
  b->Hd.ensure(size_t(B) * (p + 1) * p * sizeof(cx<double>));
  b->nrm1.ensure(size_t(B) * sizeof(double));
  b->nrm2.ensure(2 * size_t(B) * sizeof(double));
  b->inv.ensure(size_t(B) * sizeof(double));
  b->flag.ensure(size_t(B) * sizeof(int));
  b->coef.ensure(size_t(B) * (Jpart + 1) * sizeof(cx<double>));
  // deflation bases in FP32
  for (int l = 0; l < nl; ++l) {
    lqcd_defl *d = defl[l];
    if (!d->have_v32) {
      d->V32.ensure(size_t(d->k + 1) * d->n * sizeof(cx<float>));
      convert<double, float>(b->ctx[l], d->V.ptr, d->V32.ptr, size_t(d->k + 1) * d->n);
      d->have_v32 = true;
    }
  }
  // the captured inner cycle (kernel arguments are the fixed buffers
  // above; with link tiles also the lattice groups of the block in flight,
  // so it is recorded again whenever a refill changes them)
  struct GraphGuard {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    void reset() {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
      x = nullptr;
      g = nullptr;
    }
    ~GraphGuard() { reset(); }
  } guard;
  hipGraphExec_t exec = nullptr;
  auto record = [&]() {
    guard.reset();
    exec = nullptr;
    if (!b->capture) LQCD_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    LQCD_HIP(hipStreamSynchronize(b->stream));
    // the engine launches on b->stream: point it at the capture stream.
    // The guard ends a capture that an error left open (discarding its
    // graph) and restores the stream on every exit path.
    struct CaptureGuard {
      lqcd_batch *b;
      hipStream_t keep;
      bool open;
      ~CaptureGuard() {
        if (open) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(b->capture, &g);
          if (g) (void)hipGraphDestroy(g);
        }
        b->stream = keep;
      }
    } cg{b, b->stream, false};
    b->stream = b->capture;
    LQCD_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    cg.open = true;
    e.cycle();
    cg.open = false;
    const hipError_t ce = hipStreamEndCapture(b->capture, &guard.g);
    b->stream = cg.keep;
    LQCD_HIP(ce);
    LQCD_HIP(hipGetLastError());
    LQCD_HIP(hipGraphInstantiate(&guard.x, guard.g, nullptr, nullptr, 0));
    exec = guard.x;
  };
  if (use_graph && e.tile == 0) record();

  std::vector<BSlot> slh(B);
  std::vector<SlotState> ss(B);
  const double itol = std::max(prm.inner_tol, 1e-6);
  size_t next = 0;
  while (next < q.size()) {
    // fill the slots
    for (int s = 0; s < B; ++s) {
      BSlot &d = slh[s];
      d = BSlot{};
      ss[s] = SlotState{};
      if (next >= q.size()) continue;
      const int l = q[next].first, r = q[next].second;
      ++next;
      lqcd_ctx *c = b->ctx[l];
      const size_t n = half_len(c->g), fl = full_len(c->g);
      d.g = c->g;
      d.U = static_cast<const cx<float> *>(c->U32.ptr);
      d.mk2 = float(-c->kappa * c->kappa);
      d.active = 0;
      d.kd = defl[l]->k;
      d.n = n;
      d.W = W + size_t(s) * (p + 1) * nmax;
      d.T = T + size_t(s) * nmax;
      d.X = X + size_t(s) * nmax;
      d.R = R + size_t(s) * nmax;
      d.S = S + size_t(s) * nmax;
      d.Vd = static_cast<const cx<float> *>(defl[l]->V32.ptr);
      ss[s].lat = l;
      ss[s].rhs = r;
      ss[s].done = false;
      // FP64 source of the even/odd system: S = eta_e + kappa D_eo eta_o
      const cx<double> *bl = static_cast<const cx<double> *>(bvec[l]) + size_t(r) * fl;
      cx<double> *bp = Bp + size_t(s) * flmax;
      pack_eo<double>(c, bl, bp, 1, fl);
      hop_half<double>(c, 0, bp + n, bp, S64 + size_t(s) * nmax, cdouble(1, 0), c->kappa, false, false, 1,
                       fl, fl, n);
      norm2<double>(c, bp, fl, fl, 1, b->nrm1.as<double>() + s);
      fill_zero(c, X64 + size_t(s) * nmax, n * sizeof(cx<double>));
      LQCD_HIP(hipMemcpyAsync(R64 + size_t(s) * nmax, S64 + size_t(s) * nmax, n * sizeof(cx<double>),
                              hipMemcpyDeviceToDevice, b->stream));
    }
    if (e.tile > 0) {
      std::vector<int> lat(B);
      std::vector<size_t> nn(B);
      for (int s = 0; s < B; ++s) {
        lat[s] = ss[s].lat;
        nn[s] = slh[s].n;
      }
      std::vector<Group> g = lattice_groups(b->ctx, lat, nn);
      const bool same = g.size() == e.groups.size() &&
                        std::equal(g.begin(), g.end(), e.groups.begin(), [](const Group &u, const Group &v) {
                          return u.c == v.c && u.s0 == v.s0 && u.G == v.G;
                        });
      e.groups = g;
      // the block's longest vector bounds the batched grids (it changes
      // only with the lattice runs, so the recorded cycle stays valid)
      e.nlen = 0;
      for (const Group &gr : g) e.nlen = std::max(e.nlen, gr.n);
      if (use_graph && (!same || !exec)) record();
    }
    {
      // |b| of every filled slot, one copy
      std::vector<double> h(B, 0.0);
      d2h_b(b, h.data(), b->nrm1.ptr, size_t(B) * sizeof(double));
      for (int s = 0; s < B; ++s) {
        if (ss[s].lat < 0) continue;
        ss[s].ref = std::sqrt(h[s]);
        LQCD_CHECK(std::isfinite(ss[s].ref), LQCD_ENAN, "batch_solve: right-hand side is not finite");
        if (ss[s].ref == 0) ss[s].ref = 1;  // zero right-hand side: x = 0 converges at once
      }
    }
    // FP64 refinement around batched FP32 inner solves
    for (int outer = 0;; ++outer) {
      bool any = false;
      for (int s = 0; s < B; ++s) {
        if (ss[s].lat < 0 || ss[s].done) continue;
        norm2<double>(b->ctx[ss[s].lat], R64 + size_t(s) * nmax, 0, slh[s].n, 1, b->nrm1.as<double>() + s);
      }
      std::vector<double> hr(B, 0.0);
      d2h_b(b, hr.data(), b->nrm1.ptr, size_t(B) * sizeof(double));
      for (int s = 0; s < B; ++s) {
        if (ss[s].lat < 0 || ss[s].done) continue;
        const double h = hr[s];
        ss[s].rn = std::sqrt(h);
        LQCD_CHECK(std::isfinite(ss[s].rn), LQCD_ENAN, "batch_solve: NaN/Inf residual");
        if (ss[s].rn <= prm.tol * ss[s].ref || ss[s].st.cycles >= prm.max_cycles || outer > kBatchMaxRefine)
          ss[s].done = true;
        else
          any = true;
      }
      if (!any) break;
      // inner right-hand sides (FP32) and the active set
      std::vector<double> iref(B, 0), prev(B, -1), rn32(B, 0);
      std::vector<int> here(B, 0);
      for (int s = 0; s < B; ++s) {
        slh[s].active = (ss[s].lat >= 0 && !ss[s].done) ? 1 : 0;
        if (!slh[s].active) continue;
        convert<double, float>(b->ctx[ss[s].lat], R64 + size_t(s) * nmax, slh[s].S, slh[s].n);
        iref[s] = ss[s].rn;
      }
      hipLaunchKernelGGL(k_fill0, dim3(grid_n(size_t(B) * nmax)), dim3(kBlock), 0, b->stream, X,
                         size_t(B) * nmax);
      LQCD_HIP(hipMemcpyAsync(R, S, size_t(B) * nmax * sizeof(cx<float>), hipMemcpyDeviceToDevice, b->stream));
      for (;;) {
        h2d_b(b, sld, slh.data(), size_t(B) * sizeof(BSlot));
        e.norm_r(b->nrm1.as<double>());
        d2h_b(b, rn32.data(), b->nrm1.ptr, size_t(B) * sizeof(double));
        bool act = false;
        for (int s = 0; s < B; ++s) {
          if (!slh[s].active) continue;
          rn32[s] = std::sqrt(rn32[s]);
          LQCD_CHECK(std::isfinite(rn32[s]), LQCD_ENAN, "batch_solve: NaN/Inf inner residual");
          const bool stalled = prev[s] > 0 && rn32[s] > kBatchStall * prev[s];
          if (rn32[s] <= itol * iref[s] || here[s] >= kBatchCycleCap || stalled ||
              ss[s].st.cycles >= prm.max_cycles)
            slh[s].active = 0;
          else
            act = true;
        }
        if (!act) break;
        h2d_b(b, sld, slh.data(), size_t(B) * sizeof(BSlot));
        // deflation projection: c = V^H r, d = argmin |c - Hbar d|, x += V d, r -= V Hbar d
        const int Jv = kdmax + 1;
        cx<double> *cd = b->coef.as<cx<double>>();
        e.dots<BAS_V>(0, 0, Jv, cd, nullptr);
        std::vector<cdouble> C(size_t(B) * Jv), D(size_t(B) * Jv, 0.0), E(size_t(B) * Jv, 0.0);
        d2h_b(b, C.data(), cd, C.size() * sizeof(cdouble));
        for (int s = 0; s < B; ++s) {
          if (!slh[s].active) continue;
          const lqcd_defl *d = defl[ss[s].lat];
          const int k = d->k;
          std::vector<cdouble> y(C.begin() + size_t(s) * Jv, C.begin() + size_t(s) * Jv + k + 1);
          d->Hqr.apply_qh(y.data());
          d->Hqr.solve_r(y.data());
          for (int j = 0; j < k; ++j) D[size_t(s) * Jv + j] = y[j];
          for (int j = 0; j < k; ++j)
            for (int i = 0; i <= k; ++i) E[size_t(s) * Jv + i] += d->H(i, j) * y[j];
        }
        h2d_b(b, cd, D.data(), D.size() * sizeof(cdouble));
        e.update<UPD_XV>(0, 0, cd, Jv, nullptr, nullptr);
        h2d_b(b, cd, E.data(), E.size() * sizeof(cdouble));
        e.update<UPD_RV>(0, 0, cd, Jv, nullptr, nullptr);
        // one GMRES(p) cycle on every active slot
        if (exec) LQCD_HIP(hipGraphLaunch(exec, b->stream));
        else e.cycle();
        LQCD_HIP(hipGetLastError());
        std::vector<cdouble> Hh(size_t(B) * (p + 1) * p);
        std::vector<double> n0(B);
        d2h_b(b, Hh.data(), b->Hd.ptr, Hh.size() * sizeof(cdouble));
        d2h_b(b, n0.data(), b->nrm2.as<double>() + B, size_t(B) * sizeof(double));
        std::vector<cdouble> Y(size_t(B) * p, 0.0);
        for (int s = 0; s < B; ++s) {
          if (!slh[s].active) continue;
          la::Mat H(p + 1, p);
          const cdouble *hs = Hh.data() + size_t(s) * (p + 1) * p;
          for (int j = 0; j < p; ++j)
            for (int i = 0; i <= j + 1; ++i) H(i, j) = hs[size_t(j) * (p + 1) + i];
          for (auto &z : H.a)
            LQCD_CHECK(std::isfinite(z.real()) && std::isfinite(z.imag()), LQCD_ENAN,
                       "batch_solve: NaN/Inf in the Arnoldi process");
          std::vector<cdouble> cv(p + 1, 0.0);
          cv[0] = std::sqrt(n0[s]);
          std::vector<cdouble> y = la::lstsq(H, cv);
          std::copy(y.begin(), y.end(), Y.begin() + size_t(s) * p);
          ss[s].st.matvecs += p + 1;
          ss[s].st.cycles += 1;
          prev[s] = rn32[s];
          here[s] += 1;
        }
        h2d_b(b, cd, Y.data(), Y.size() * sizeof(cdouble));
        e.update<UPD_XW>(0, p, cd, p, nullptr, nullptr);
        // true inner residual r = s - Mhat x
        e.stencil_schur_x();
        hipLaunchKernelGGL(k_bresid, dim3(grid_n(e.nlen), B), dim3(kBlock), 0, b->stream, sld);
        LQCD_HIP(hipGetLastError());
      }
      // x += e (FP64), r = S - Mhat x (FP64)
      for (int s = 0; s < B; ++s) {
        if (ss[s].lat < 0 || ss[s].done) continue;
        lqcd_ctx *c = b->ctx[ss[s].lat];
        const size_t n = slh[s].n;
        hipLaunchKernelGGL(k_widen_add, dim3(grid_n(n)), dim3(kBlock), 0, b->stream, X + size_t(s) * nmax,
                           X64 + size_t(s) * nmax, n);
        apply_schur<double>(c, X64 + size_t(s) * nmax, R64 + size_t(s) * nmax, TF + size_t(s) * flmax, 1, n, n,
                            n);
        cdouble one(1, 0), mone(-1, 0);
        axpby<double>(c, &one, S64 + size_t(s) * nmax, n, &mone, R64 + size_t(s) * nmax, n, n, 1, false);
        ss[s].st.matvecs += 1;
        ss[s].st.refinements += 1;
      }
    }
    // odd sites, LEX solution, FP64 true residual on the full lattice
    for (int s = 0; s < B; ++s) {
      if (ss[s].lat < 0) continue;
      const int l = ss[s].lat;
      lqcd_ctx *c = b->ctx[l];
      const size_t n = slh[s].n, fl = full_len(c->g);
      cx<double> *xf = XF + size_t(s) * flmax, *tf = TF + size_t(s) * flmax, *bp = Bp + size_t(s) * flmax;
      LQCD_HIP(hipMemcpyAsync(xf, X64 + size_t(s) * nmax, n * sizeof(cx<double>), hipMemcpyDeviceToDevice,
                              b->stream));
      hop_half<double>(c, 1, xf, bp + n, xf + n, cdouble(1, 0), c->kappa, false, false, 1, fl, fl, fl);
      cx<double> *xl = static_cast<cx<double> *>(xvec[l]) + size_t(ss[s].rhs) * fl;
      unpack_eo<double>(c, xf, xl, 1, fl);
      apply_full<double>(c, LQCD_OP_M, xf, tf, 1, fl, fl);
      cdouble one(1, 0), mone(-1, 0);
      axpby<double>(c, &one, bp, fl, &mone, tf, fl, fl, 1, false);
      norm2<double>(c, tf, fl, fl, 1, b->nrm1.as<double>() + s);
    }
    {
      std::vector<double> h(B, 0.0);
      d2h_b(b, h.data(), b->nrm1.ptr, size_t(B) * sizeof(double));
      for (int s = 0; s < B; ++s) {
        if (ss[s].lat < 0) continue;
        ss[s].st.true_resid = std::sqrt(h[s]) / ss[s].ref;
        if (ss[s].rn > prm.tol * ss[s].ref) *nonconv = 1;
        if (stats) stats[first[ss[s].lat] + ss[s].rhs] = ss[s].st;
      }
    }
  }
}

void check_batch_args(lqcd_batch *b, const lqcd_solve_params *pp, const void *const *bvec,
                      const int *nrhs, lqcd_defl *const *defl) {
  LQCD_CHECK(b && pp && bvec && nrhs && defl, LQCD_EINVAL, "batch_solve: null argument");
  const lqcd_solve_params &p = *pp;
  LQCD_CHECK(p.k >= 1 && p.m > p.k && p.m <= 250, LQCD_EINVAL, "batch_solve: need 1 <= k < m <= 250");
  LQCD_CHECK(p.proj_m >= 0 && p.proj_m <= 250, LQCD_EINVAL, "batch_solve: proj_m outside 0..250");
  LQCD_CHECK(p.tol > 0 && p.max_cycles >= 1, LQCD_EINVAL, "batch_solve: bad tol/max_cycles");
  LQCD_CHECK(p.inner == LQCD_F32, LQCD_EINVAL, "batch_solve: the batched inner solver is FP32 (inner = LQCD_F32)");
  LQCD_CHECK(p.rhs_block >= 1 && p.rhs_block <= 64, LQCD_EINVAL, "batch_solve: rhs_block outside 1..64");
  for (size_t l = 0; l < b->ctx.size(); ++l) {
    LQCD_CHECK(nrhs[l] >= 0, LQCD_EINVAL, "batch_solve: nrhs < 0");
    LQCD_CHECK(nrhs[l] == 0 || bvec[l], LQCD_EINVAL, "batch_solve: null field");
    const lqcd_defl *d = defl[l];
    LQCD_CHECK(d && d->op == LQCD_OP_SCHUR, LQCD_EINVAL,
               "batch_solve: lattice %zu needs a deflation space of the even/odd system", l);
    for (int i = 0; i < 4; ++i)
      LQCD_CHECK(d->dims[i] == b->ctx[l]->g.L[i], LQCD_EINVAL, "batch_solve: deflation space of another lattice");
    LQCD_CHECK(d->kappa == b->ctx[l]->kappa, LQCD_EINVAL, "batch_solve: deflation space of another kappa");
  }
}

}  // namespace
}  // namespace lqcd

extern "C" lqcd_status lqcd_batch_create(lqcd_ctx *const *ctxs, int nlat, lqcd_batch **out) {
  return guarded([&] {
    LQCD_CHECK(ctxs && out && nlat >= 1, LQCD_EINVAL, "lqcd_batch_create: bad argument");
    std::unique_ptr<lqcd_batch> b(new lqcd_batch());
    for (int l = 0; l < nlat; ++l) {
      LQCD_CHECK(ctxs[l], LQCD_EINVAL, "lqcd_batch_create: null context %d", l);
      LQCD_CHECK(ctxs[l]->stream == ctxs[0]->stream && ctxs[l]->device == ctxs[0]->device, LQCD_EINVAL,
                 "lqcd_batch_create: contexts must share one device and one stream");
      b->ctx.push_back(ctxs[l]);
    }
    b->stream = ctxs[0]->stream;
    *out = b.release();
  });
}

extern "C" lqcd_status lqcd_batch_destroy(lqcd_batch *b) {
  return guarded([&] {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    delete b;
  });
}

extern "C" lqcd_status lqcd_batch_set_grid(lqcd_batch *b, int workgroups) {
  return guarded([&] {
    LQCD_CHECK(b && workgroups >= 1 && workgroups <= 65536, LQCD_EINVAL, "lqcd_batch_set_grid: bad argument");
    b->hop_grid = workgroups;
  });
}

extern "C" lqcd_status lqcd_batch_set_tile(lqcd_batch *b, int tile_sites) {
  return guarded([&] {
    LQCD_CHECK(b && (tile_sites == 0 || tile_sites == 16 || tile_sites == 32 || tile_sites == 64), LQCD_EINVAL,
               "lqcd_batch_set_tile: tile of 0, 16, 32 or 64 sites");
    b->tile = tile_sites;
  });
}

extern "C" lqcd_status batch_solve(lqcd_batch *b, const lqcd_solve_params *params, const void *const *bvec,
                                   void *const *xvec, const int *nrhs, lqcd_defl *const *defl, int use_graph,
                                   lqcd_solve_stats *stats) {
  return guarded([&] {
    check_batch_args(b, params, bvec, nrhs, defl);
    LQCD_CHECK(xvec, LQCD_EINVAL, "batch_solve: null solution array");
    for (size_t l = 0; l < b->ctx.size(); ++l)
      LQCD_CHECK(nrhs[l] == 0 || xvec[l], LQCD_EINVAL, "batch_solve: null solution field");
    int nonconv = 0;
    run_batch(b, *params, bvec, xvec, nrhs, defl, use_graph != 0, stats, &nonconv);
    LQCD_CHECK(!nonconv, LQCD_ENOCONV, "batch_solve: a right-hand side missed tol within max_cycles");
  });
}

extern "C" lqcd_status batch_autotune(lqcd_batch *b, const lqcd_solve_params *params, const void *const *bvec,
                                      const int *nrhs, lqcd_defl *const *defl, int *best_rhs_block,
                                      int *best_tile, double *rate_host) {
  return guarded([&] {
    check_batch_args(b, params, bvec, nrhs, defl);
    LQCD_CHECK(best_rhs_block && best_tile, LQCD_EINVAL, "batch_autotune: null output");
    const int nl = int(b->ctx.size());
    int total = 0;
    for (int l = 0; l < nl; ++l) total += nrhs[l];
    LQCD_CHECK(total >= 1, LQCD_EINVAL, "batch_autotune: no right-hand sides");
    // scratch solutions for the trial solves
    std::vector<DevBuf> xs(nl);
    std::vector<void *> xp(nl, nullptr);
    for (int l = 0; l < nl; ++l)
      if (nrhs[l] > 0) xp[l] = xs[l].ensure(size_t(nrhs[l]) * full_len(b->ctx[l]->g) * sizeof(cdouble));
    const int blocks[kTuneBlocks] = {4, 8, 16, 32};
    const int tiles[kTuneTiles] = {0, 16, 32, 64};
    const int keep_tile = b->tile;
    struct Restore {
      lqcd_batch *b;
      int t;
      ~Restore() { b->tile = t; }
    } restore{b, keep_tile};
    double best = -1;
    int bi = 0;
    for (int ib = 0; ib < kTuneBlocks; ++ib)
      for (int it = 0; it < kTuneTiles; ++it) {
        double rate = 0;
        if (blocks[ib] <= std::max(4, total)) {
          // a trial solves one block of right-hand sides, taken evenly from the lattices
          std::vector<int> nt(nl, 0);
          int left = std::min(blocks[ib], total);
          while (left > 0)
            for (int l = 0; l < nl && left > 0; ++l)
              if (nt[l] < nrhs[l]) {
                ++nt[l];
                --left;
              }
          lqcd_solve_params pr = *params;
          pr.rhs_block = blocks[ib];
          b->tile = tiles[it];
          int nonconv = 0;
          LQCD_HIP(hipStreamSynchronize(b->stream));
          const auto t0 = std::chrono::steady_clock::now();
          run_batch(b, pr, bvec, xp.data(), nt.data(), defl, true, nullptr, &nonconv);
          LQCD_HIP(hipStreamSynchronize(b->stream));
          const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
          int ns = 0;
          for (int v : nt) ns += v;
          rate = ns / dt;
        }
        if (rate_host) rate_host[bi] = rate;
        ++bi;
        if (rate > best) {
          best = rate;
          *best_rhs_block = blocks[ib];
          *best_tile = tiles[it];
        }
      }
  });
}

extern "C" lqcd_status batch_wilson_apply(lqcd_batch *b, const void *const *in, void *const *out,
                                          const int *nrhs) {
  return guarded([&] {
    LQCD_CHECK(b && in && out && nrhs, LQCD_EINVAL, "batch_wilson_apply: null argument");
    const int nl = int(b->ctx.size());
    std::vector<std::pair<int, int>> q;
    for (int l = 0; l < nl; ++l) {
      LQCD_CHECK(nrhs[l] >= 0 && (nrhs[l] == 0 || (in[l] && out[l])), LQCD_EINVAL,
                 "batch_wilson_apply: bad field");
      for (int r = 0; r < nrhs[l]; ++r) q.emplace_back(l, r);
    }
    if (q.empty()) return;
    const int B = int(q.size());
    size_t nmax = 0, flmax = 0;
    int Vhmax = 0;
    for (int l = 0; l < nl; ++l) {
      nmax = std::max(nmax, half_len(b->ctx[l]->g));
      flmax = std::max(flmax, full_len(b->ctx[l]->g));
      Vhmax = std::max(Vhmax, b->ctx[l]->g.Vh);
    }
    const unsigned per = unsigned((Vhmax + kBlock - 1) / kBlock);
    cx<float> *X = static_cast<cx<float> *>(b->X.ensure(size_t(B) * nmax * sizeof(cx<float>)));
    cx<float> *R = static_cast<cx<float> *>(b->R.ensure(size_t(B) * nmax * sizeof(cx<float>)));
    cx<float> *T = static_cast<cx<float> *>(b->T.ensure(size_t(B) * nmax * sizeof(cx<float>)));
    cx<float> *E = static_cast<cx<float> *>(b->W.ensure(size_t(B) * 2 * flmax * sizeof(cx<float>)));
    BSlot *sld = static_cast<BSlot *>(b->slots_dev.ensure(size_t(B) * sizeof(BSlot)));
    std::vector<BSlot> slh(B);
    for (int s = 0; s < B; ++s) {
      const int l = q[s].first, r = q[s].second;
      lqcd_ctx *c = b->ctx[l];
      const size_t n = half_len(c->g), fl = full_len(c->g);
      BSlot &d = slh[s];
      d = BSlot{};
      d.g = c->g;
      d.U = static_cast<const cx<float> *>(c->U32.ptr);
      d.mk2 = float(-c->kappa * c->kappa);
      d.active = 1;
      d.n = n;
      d.X = X + size_t(s) * nmax;
      d.R = R + size_t(s) * nmax;
      d.T = T + size_t(s) * nmax;
      cx<float> *ef = E + size_t(s) * flmax;
      pack_eo<float>(c, static_cast<const cdouble *>(in[l]) + size_t(r) * fl, ef, 1, fl);
      LQCD_HIP(hipMemcpyAsync(d.X, ef, n * sizeof(cx<float>), hipMemcpyDeviceToDevice, b->stream));
    }
    h2d_b(b, sld, slh.data(), size_t(B) * sizeof(BSlot));
    Engine e{b, B, 1, nmax, per, unsigned(B) * per, unsigned(b->hop_grid), 0, sld};
    e.nlen = nmax;
    e.tile = b->tile;
    e.X = X;
    e.R = R;
    e.T = T;
    if (e.tile > 0) {
      std::vector<int> lat(B);
      std::vector<size_t> nn(B);
      for (int s = 0; s < B; ++s) {
        lat[s] = q[s].first;
        nn[s] = slh[s].n;
      }
      e.groups = lattice_groups(b->ctx, lat, nn);
    }
    e.stencil_schur_x();
    LQCD_HIP(hipGetLastError());
    for (int s = 0; s < B; ++s) {
      const int l = q[s].first, r = q[s].second;
      lqcd_ctx *c = b->ctx[l];
      const size_t n = half_len(c->g), fl = full_len(c->g);
      cx<float> *ef = E + size_t(s) * flmax;
      LQCD_HIP(hipMemcpyAsync(ef, slh[s].R, n * sizeof(cx<float>), hipMemcpyDeviceToDevice, b->stream));
      fill_zero(c, ef + n, n * sizeof(cx<float>));
      unpack_eo<float>(c, ef, static_cast<cdouble *>(out[l]) + size_t(r) * fl, 1, fl);
    }
  });
}
