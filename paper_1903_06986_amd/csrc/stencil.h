// Device building blocks of the Wilson hopping stencil (Sec. 5.1 Eqs.
// (24)-(25)) on even/odd fields, shared by the single-lattice and the
// batched kernels.
//
//   (P psi)(x) = sum_mu [ (1 - g_mu) U_mu(x) psi(x + mu)
//                       + (1 + g_mu) U_mu(x - mu)^+ psi(x - mu) ]
//
// In the chiral basis (g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0,1],[1,0]])
// every (1 -+ g_mu) has rank 2: with psi = (u, l) in upper/lower spin
// pairs, (1 - g_mu) psi = (h, R h) where h = u + i s_k l (h = u - l for
// mu = t) and R = -i s_k (R = -1 for t); (1 + g_mu) psi = (h', R' h') with
// h' = u - i s_k l (u + l), R' = +i s_k (+1).  The link therefore acts on a
// two-spin "half spinor" only (6 complex), and the lower spins are rebuilt
// from the product.
//
// Data layouts (per right-hand side, per parity), component c = spin * 3 +
// colour.  Every layout stores a site's spinor as 16-byte granules, granule
// g of all sites contiguous ([granules][Vh][16 bytes]), so that one lane
// gathers a neighbour with 16-byte loads and a wavefront's load of one
// granule of 64 consecutive sites is one contiguous 1 KiB run:
//   FP64 plain:  [12][Vh] complex (one component per granule);
//   FP32 pairs:  [6][Vh] x (c = 2g, 2g + 1) -- the stencil's internal
//                odd-site temporary of the even/odd operator;
//   16-bit:      [3][Vh] x (c = 4g .. 4g + 3), then the per-site scales
//                (half.h).
// FP32 fields the solvers hold are component-major [12][Vh] (8-byte
// granules), the layout their Gram-Schmidt kernels share with FP64.
// Links: [parity][mu][9][Vh].
#pragma once

#include "common.h"
#include "cplx.h"
#include "half.h"

namespace lqcd {
namespace st {

// Field sources of the stencil: plain complex fields of precision R, or
// 16-bit fields with per-site scales (half.h), decoded to FP32.  at(r)
// moves to right-hand side r (stride in elements of the storage); site(i)
// fetches what every component load of site i shares.
//
// The *_at forms address a site by a 32-bit byte offset o = oslot + i *
// kSiteBytes from the base p (kSiteBytes: bytes of one granule of one
// site; oslot: the lane's right-hand side, counted from the wave's): with p
// the same for the whole wave, p + granule offset stays in scalar
// registers and every load is "scalar base + one 32-bit lane offset", one
// VGPR per neighbour instead of a 64-bit address per component.
// kElemBytes: bytes of one storage element (the unit of right-hand-side
// strides and of at()).
template <class R>
struct SrcPlain {
  const cx<R> *p;
  using Ctx = int;
  static constexpr uint32_t kElemBytes = sizeof(cx<R>), kSiteBytes = sizeof(cx<R>);
  __device__ SrcPlain at(size_t off) const { return SrcPlain{p + off}; }
  __device__ Ctx site(size_t) const { return 0; }
  __device__ cx<R> ld(Ctx, size_t i, int comp, size_t Vh) const { return ldc(p + comp * Vh + i); }
  __device__ Ctx site_at(uint32_t, uint32_t) const { return 0; }
  __device__ cx<R> ld_at(Ctx, uint32_t o, int comp, size_t Vh) const {
    return ldc(reinterpret_cast<const cx<R> *>(reinterpret_cast<const char *>(p + comp * Vh) + o));
  }
};

// FP32 in component pairs: granule g of site i (components 2g, 2g + 1) at
// complex elements 2 (g Vh + i) and 2 (g Vh + i) + 1.
struct SrcPair {
  const cx<float> *p;
  using Ctx = int;
  static constexpr uint32_t kElemBytes = 8, kSiteBytes = 16;
  __device__ SrcPair at(size_t off) const { return SrcPair{p + off}; }
  __device__ Ctx site(size_t) const { return 0; }
  __device__ cx<float> ld(Ctx, size_t i, int comp, size_t Vh) const {
    return ldc(p + 2 * ((comp >> 1) * Vh + i) + (comp & 1));
  }
  __device__ Ctx site_at(uint32_t, uint32_t) const { return 0; }
  __device__ cx<float> ld_at(Ctx, uint32_t o, int comp, size_t Vh) const {
    return ldc(reinterpret_cast<const cx<float> *>(reinterpret_cast<const char *>(p + 2 * (comp >> 1) * Vh) + o) +
               (comp & 1));
  }
};

template <HKind K>
struct SrcHalf {
  const uint32_t *p;
  size_t n;  // payload words (12 Vh); the scales follow
  using Ctx = float;
  static constexpr uint32_t kElemBytes = 4, kSiteBytes = 16;
  __device__ SrcHalf at(size_t off) const { return SrcHalf{p + off, n}; }
  __device__ Ctx site(size_t i) const { return __uint_as_float(p[n + i]); }
  __device__ cx<float> ld(Ctx sc, size_t i, int comp, size_t Vh) const {
    const cx<float> v = Codec<K>::unpack(p[hword(comp, i, Vh)]);
    return mk(sc * v.re, sc * v.im);
  }
  // o = oslot + 16 i (oslot: the right-hand side's byte offset from p);
  // the scale of site i sits at byte oslot + 4 i after the payload
  __device__ Ctx site_at(uint32_t o, uint32_t oslot) const {
    return __uint_as_float(*reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(p + n) + oslot +
                                                               ((o - oslot) >> 2)));
  }
  __device__ cx<float> ld_at(Ctx sc, uint32_t o, int comp, size_t Vh) const {
    const cx<float> v = Codec<K>::unpack(*reinterpret_cast<const uint32_t *>(
        reinterpret_cast<const char *>(p + 4 * (comp >> 2) * Vh) + o + 4 * (comp & 3)));
    return mk(sc * v.re, sc * v.im);
  }
};

// Output layouts of the stencil (plain component-major, FP32 pairs, or
// 16-bit with a per-site scale): store12 writes a site's 12 components,
// streamed past the caches when NT.  o + oo is the site's first element;
// ob (bytes) locates the right-hand side's field within o (o + ob its start;
// oo - ob = i kSiteBytes for site i).
template <class R>
struct OutPlain {
  static constexpr uint32_t kElemBytes = sizeof(cx<R>), kSiteBytes = sizeof(cx<R>);
  static constexpr double kFieldBytes = 12.0 * sizeof(cx<R>);  // per site
  template <bool NT>
  __device__ static void store12(char *o, uint32_t oo, uint32_t, size_t Vh, const cx<R> (&v)[12]) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      cx<R> *q = reinterpret_cast<cx<R> *>(o + k * Vh * sizeof(cx<R>) + oo);
      if (NT) stc_nt(q, v[k]);
      else stc(q, v[k]);
    }
  }
};
struct OutPair {
  static constexpr uint32_t kElemBytes = 8, kSiteBytes = 16;
  static constexpr double kFieldBytes = 96.0;
  template <bool NT>
  __device__ static void store12(char *o, uint32_t oo, uint32_t, size_t Vh, const cx<float> (&v)[12]) {
    typedef float f4v __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int g = 0; g < 6; ++g) {
      f4v w;
      w.x = v[2 * g].re;
      w.y = v[2 * g].im;
      w.z = v[2 * g + 1].re;
      w.w = v[2 * g + 1].im;
      f4v *q = reinterpret_cast<f4v *>(o + g * Vh * 16 + oo);
      if (NT) __builtin_nontemporal_store(w, q);
      else *q = w;
    }
  }
};

// The stored 16-bit form of SrcHalf (kind K): component c of site i in word
// hword(c, i, Vh) as the pair v / m rounded (m = the site's largest |re|,
// |im|; 0 for a zero site), the scale m in word 12 Vh + i (strides in words).
template <HKind K>
struct OutHalf {
  static constexpr uint32_t kElemBytes = 4, kSiteBytes = 16;
  static constexpr double kFieldBytes = 52.0;
  template <bool NT>
  __device__ static void store12(char *o, uint32_t oo, uint32_t ob, size_t Vh, const cx<float> (&v)[12]) {
    typedef unsigned u4v __attribute__((ext_vector_type(4)));
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
      u4v q;
#pragma unroll
      for (int k = 0; k < 4; ++k) q[k] = Codec<K>::pack(inv * v[4 * g + k].re, inv * v[4 * g + k].im);
      u4v *d = reinterpret_cast<u4v *>(o + g * Vh * 16 + oo);
      if (NT) __builtin_nontemporal_store(q, d);
      else *d = q;
    }
    float *ds = reinterpret_cast<float *>(o + ob + 48 * Vh + ((oo - ob) >> 2));
    if (NT) __builtin_nontemporal_store(m, ds);
    else *ds = m;
  }
};

template <class R>
struct Half {
  cx<R> h[2][3];  // [spin 0/1][colour]
};

// U h (forward) and U^+ h (backward) on each of the two spins of a half
// spinor; u points at entry 0 of the link, entries are Vh apart.
template <class R>
__device__ inline void link_mul(const cx<R> *u, size_t Vh, const Half<R> &in,
                                Half<R> &out) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> u0 = ldc(u + (3 * a + 0) * Vh), u1 = ldc(u + (3 * a + 1) * Vh),
          u2 = ldc(u + (3 * a + 2) * Vh);
#pragma unroll
    for (int s = 0; s < 2; ++s) out.h[s][a] = u0 * in.h[s][0] + u1 * in.h[s][1] + u2 * in.h[s][2];
  }
}
template <class R>
__device__ inline void link_dag_mul(const cx<R> *u, size_t Vh, const Half<R> &in,
                                    Half<R> &out) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) out.h[s][a] = mk<R>(0, 0);
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    cx<R> u0 = ldc(u + (3 * b + 0) * Vh), u1 = ldc(u + (3 * b + 1) * Vh),
          u2 = ldc(u + (3 * b + 2) * Vh);
    // (U^+ h)_a = sum_b conj(U_ba) h_b
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      out.h[s][0] = out.h[s][0] + cmulc(u0, in.h[s][b]);
      out.h[s][1] = out.h[s][1] + cmulc(u1, in.h[s][b]);
      out.h[s][2] = out.h[s][2] + cmulc(u2, in.h[s][b]);
    }
  }
}

// Project psi (site i of the source, 12 components at stride Vh) for
// direction MU and sign (FWD: 1 - g_mu, else 1 + g_mu).  G5 applies
// g5 = diag(1,1,-1,-1) first.
template <class R, int MU, bool FWD, bool G5, class Src, class I>
__device__ inline void project(const Src &src, I i, size_t Vh, Half<R> &o) {
  const typename Src::Ctx sc = src.site(i);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> u0 = src.ld(sc, i, 0 * 3 + c, Vh), u1 = src.ld(sc, i, 1 * 3 + c, Vh);
    cx<R> l0 = src.ld(sc, i, 2 * 3 + c, Vh), l1 = src.ld(sc, i, 3 * 3 + c, Vh);
    if (G5) {
      l0 = -l0;
      l1 = -l1;
    }
    // FWD: h = u + i s_k l ; BWD: h = u - i s_k l ; t: h = u -+ l
    if (MU == 0) {  // i s_1 l = (i l1, i l0)
      o.h[0][c] = FWD ? u0 + iz(l1) : u0 - iz(l1);
      o.h[1][c] = FWD ? u1 + iz(l0) : u1 - iz(l0);
    } else if (MU == 1) {  // i s_2 l = (l1, -l0)
      o.h[0][c] = FWD ? u0 + l1 : u0 - l1;
      o.h[1][c] = FWD ? u1 - l0 : u1 + l0;
    } else if (MU == 2) {  // i s_3 l = (i l0, -i l1)
      o.h[0][c] = FWD ? u0 + iz(l0) : u0 - iz(l0);
      o.h[1][c] = FWD ? u1 - iz(l1) : u1 + iz(l1);
    } else {  // t
      o.h[0][c] = FWD ? u0 - l0 : u0 + l0;
      o.h[1][c] = FWD ? u1 - l1 : u1 + l1;
    }
  }
}

// Raw loads of one site's 12 components for the tiled stencil: fetch_at
// issues all of them, settle makes them complete together (one empty asm
// naming every loaded register), and project_raw then works from
// registers.  Without it the compiler interleaves the loads with the
// projection arithmetic and keeps only a few of them in flight per wave.
template <class Src>
struct Raw;
// get(k) is component k as stored times the site's scale; unscaled(k) and
// scale() split it, so that the linear steps (projection, link product)
// run on the unscaled values and the scale enters once, in the
// accumulation (One: plain fields, no scale).
// kMix: the projection adds run as FMAs with a unit factor, so that each
// folds the conversion of its two FP16 operands (v_fma_mix_f32).
struct One {};
template <class R>
struct Raw<SrcPlain<R>> {
  static constexpr bool kMix = false;
  cx<R> v[12];
  __device__ cx<R> get(int k) const { return v[k]; }
  __device__ cx<R> unscaled(int k) const { return v[k]; }
  __device__ One scale() const { return One{}; }
};
template <>
struct Raw<SrcPair> {
  static constexpr bool kMix = false;
  float4 q[6];
  __device__ cx<float> get(int k) const {
    const float4 v = q[k >> 1];
    return (k & 1) ? mk(v.z, v.w) : mk(v.x, v.y);
  }
  __device__ cx<float> unscaled(int k) const { return get(k); }
  __device__ One scale() const { return One{}; }
};
template <HKind K>
struct Raw<SrcHalf<K>> {
  static constexpr bool kMix = K == HKind::F16;
  uint4 q[3];
  float sc;
  __device__ uint32_t word(int k) const {
    const uint4 v = q[k >> 2];
    return (k & 3) == 0 ? v.x : (k & 3) == 1 ? v.y : (k & 3) == 2 ? v.z : v.w;
  }
  __device__ cx<float> get(int k) const {
    const cx<float> v = Codec<K>::unpack(word(k));
    return mk(sc * v.re, sc * v.im);
  }
  __device__ cx<float> unscaled(int k) const { return Codec<K>::unpack(word(k)); }
  __device__ float scale() const { return sc; }
};

// Explicit fused multiply-adds: the link products as chains of FMAs (one
// rounding per term) instead of products summed by separate adds.
__device__ inline double fmr(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float fmr(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// a b
template <class R>
__device__ inline cx<R> cmul_f(cx<R> a, cx<R> b) {
  return {fmr(a.re, b.re, -a.im * b.im), fmr(a.re, b.im, a.im * b.re)};
}
// a b + c
template <class R>
__device__ inline cx<R> cfma(cx<R> a, cx<R> b, cx<R> c) {
  return {fmr(a.re, b.re, fmr(-a.im, b.im, c.re)), fmr(a.re, b.im, fmr(a.im, b.re, c.im))};
}
// conj(a) b
template <class R>
__device__ inline cx<R> cmulc_f(cx<R> a, cx<R> b) {
  return {fmr(a.re, b.re, a.im * b.im), fmr(a.re, b.im, -a.im * b.re)};
}
// conj(a) b + c
template <class R>
__device__ inline cx<R> cfmac(cx<R> a, cx<R> b, cx<R> c) {
  return {fmr(a.re, b.re, fmr(a.im, b.im, c.re)), fmr(a.re, b.im, fmr(-a.im, b.re, c.im))};
}

// a + s b
template <class R>
__device__ inline cx<R> madd(cx<R> a, One, cx<R> b) {
  return a + b;
}
__device__ inline cx<float> madd(cx<float> a, float s, cx<float> b) {
  return mk(__builtin_fmaf(s, b.re, a.re), __builtin_fmaf(s, b.im, a.im));
}

template <class R>
__device__ inline void fetch_at(const SrcPlain<R> &s, uint32_t o, uint32_t, size_t Vh, Raw<SrcPlain<R>> &r) {
#pragma unroll
  for (int k = 0; k < 12; ++k) r.v[k] = s.ld_at(0, o, k, Vh);
}
__device__ inline void fetch_at(const SrcPair &s, uint32_t o, uint32_t, size_t Vh, Raw<SrcPair> &r) {
#pragma unroll
  for (int g = 0; g < 6; ++g)
    r.q[g] = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s.p + 2 * g * Vh) + o);
}
template <HKind K>
__device__ inline void fetch_at(const SrcHalf<K> &s, uint32_t o, uint32_t oslot, size_t Vh, Raw<SrcHalf<K>> &r) {
  r.sc = s.site_at(o, oslot);
#pragma unroll
  for (int g = 0; g < 3; ++g)
    r.q[g] = *reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(s.p + 4 * g * Vh) + o);
}

#define LQCD_V2(a) "+v"(a.re), "+v"(a.im)
template <class R>
__device__ inline void settle(Raw<SrcPlain<R>> &r) {
  asm volatile("" : LQCD_V2(r.v[0]), LQCD_V2(r.v[1]), LQCD_V2(r.v[2]), LQCD_V2(r.v[3]), LQCD_V2(r.v[4]),
               LQCD_V2(r.v[5]), LQCD_V2(r.v[6]), LQCD_V2(r.v[7]), LQCD_V2(r.v[8]), LQCD_V2(r.v[9]),
               LQCD_V2(r.v[10]), LQCD_V2(r.v[11]));
}
#undef LQCD_V2
#define LQCD_V4(a) "+v"(a.x), "+v"(a.y), "+v"(a.z), "+v"(a.w)
__device__ inline void settle(Raw<SrcPair> &r) {
  asm volatile("" : LQCD_V4(r.q[0]), LQCD_V4(r.q[1]), LQCD_V4(r.q[2]), LQCD_V4(r.q[3]), LQCD_V4(r.q[4]),
               LQCD_V4(r.q[5]));
}
template <HKind K>
__device__ inline void settle(Raw<SrcHalf<K>> &r) {
  asm volatile("" : LQCD_V4(r.q[0]), LQCD_V4(r.q[1]), LQCD_V4(r.q[2]), "+v"(r.sc));
}
#undef LQCD_V4

// project() on a settled raw site, without its scale (RawT::scale()).
// one must hold 1 in a register the compiler cannot see through: for kMix
// sources a + b is computed as fma(b, one, a), the same rounded sum.
template <class R, int MU, bool FWD, bool G5, class RawT>
__device__ inline void project_raw(const RawT &r, Half<R> &o, R one) {
  auto add = [one](cx<R> a, cx<R> b) {
    return RawT::kMix ? cx<R>{fmr(b.re, one, a.re), fmr(b.im, one, a.im)} : a + b;
  };
  auto sub = [&add](cx<R> a, cx<R> b) { return add(a, -b); };
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> u0 = r.unscaled(0 * 3 + c), u1 = r.unscaled(1 * 3 + c);
    cx<R> l0 = r.unscaled(2 * 3 + c), l1 = r.unscaled(3 * 3 + c);
    if (G5) {
      l0 = -l0;
      l1 = -l1;
    }
    if (MU == 0) {
      o.h[0][c] = FWD ? add(u0, iz(l1)) : sub(u0, iz(l1));
      o.h[1][c] = FWD ? add(u1, iz(l0)) : sub(u1, iz(l0));
    } else if (MU == 1) {
      o.h[0][c] = FWD ? add(u0, l1) : sub(u0, l1);
      o.h[1][c] = FWD ? sub(u1, l0) : add(u1, l0);
    } else if (MU == 2) {
      o.h[0][c] = FWD ? add(u0, iz(l0)) : sub(u0, iz(l0));
      o.h[1][c] = FWD ? sub(u1, iz(l1)) : add(u1, iz(l1));
    } else {
      o.h[0][c] = FWD ? sub(u0, l0) : add(u0, l0);
      o.h[1][c] = FWD ? sub(u1, l1) : add(u1, l1);
    }
  }
}

// acc += (g, R g) for direction MU, sign FWD (R = -i s_k / +i s_k / -+1).
template <class R, int MU, bool FWD>
__device__ inline void accumulate(cx<R> acc[4][3], const Half<R> &g) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> g0 = g.h[0][c], g1 = g.h[1][c];
    acc[0][c] = acc[0][c] + g0;
    acc[1][c] = acc[1][c] + g1;
    cx<R> r0, r1;
    if (MU == 0) {  // -i s_1 g = (-i g1, -i g0); +i s_1 g = (i g1, i g0)
      r0 = FWD ? miz(g1) : iz(g1);
      r1 = FWD ? miz(g0) : iz(g0);
    } else if (MU == 1) {  // -i s_2 g = (-g1, g0); +i s_2 g = (g1, -g0)
      r0 = FWD ? -g1 : g1;
      r1 = FWD ? g0 : -g0;
    } else if (MU == 2) {  // -i s_3 g = (-i g0, i g1); +i s_3 g = (i g0, -i g1)
      r0 = FWD ? miz(g0) : iz(g0);
      r1 = FWD ? iz(g1) : miz(g1);
    } else {  // -g / +g
      r0 = FWD ? -g0 : g0;
      r1 = FWD ? -g1 : g1;
    }
    acc[2][c] = acc[2][c] + r0;
    acc[3][c] = acc[3][c] + r1;
  }
}

// acc += sc (g, R g), the reconstruction of (U h) (FWD) or (U^+ h)
// (backward) for direction MU, one colour row at a time, so that the
// 6-complex product is never held whole.  u points at entry 0 of the link,
// entries ld apart.  The same terms in the same order as link_mul /
// link_dag_mul followed by accumulate, summed by FMA chains; sc is the
// source's per-site scale (One: none).
template <class R, int MU, bool FWD, class S>
__device__ inline void link_accumulate(cx<R> acc[4][3], const cx<R> *u, size_t ld, const Half<R> &h, S sc) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<R> g0, g1;
    if (FWD) {
      const cx<R> u0 = ldc(u + (3 * a + 0) * ld), u1 = ldc(u + (3 * a + 1) * ld), u2 = ldc(u + (3 * a + 2) * ld);
      g0 = cfma(u2, h.h[0][2], cfma(u1, h.h[0][1], cmul_f(u0, h.h[0][0])));
      g1 = cfma(u2, h.h[1][2], cfma(u1, h.h[1][1], cmul_f(u0, h.h[1][0])));
    } else {  // (U^+ h)_a = sum_b conj(U_ba) h_b
      const cx<R> u0 = ldc(u + (0 * 3 + a) * ld), u1 = ldc(u + (1 * 3 + a) * ld), u2 = ldc(u + (2 * 3 + a) * ld);
      g0 = cfmac(u2, h.h[0][2], cfmac(u1, h.h[0][1], cmulc_f(u0, h.h[0][0])));
      g1 = cfmac(u2, h.h[1][2], cfmac(u1, h.h[1][1], cmulc_f(u0, h.h[1][0])));
    }
    acc[0][a] = madd(acc[0][a], sc, g0);
    acc[1][a] = madd(acc[1][a], sc, g1);
    cx<R> r0, r1;
    if (MU == 0) {
      r0 = FWD ? miz(g1) : iz(g1);
      r1 = FWD ? miz(g0) : iz(g0);
    } else if (MU == 1) {
      r0 = FWD ? -g1 : g1;
      r1 = FWD ? g0 : -g0;
    } else if (MU == 2) {
      r0 = FWD ? miz(g0) : iz(g0);
      r1 = FWD ? iz(g1) : miz(g1);
    } else {
      r0 = FWD ? -g0 : g0;
      r1 = FWD ? -g1 : g1;
    }
    acc[2][a] = madd(acc[2][a], sc, r0);
    acc[3][a] = madd(acc[3][a], sc, r1);
  }
}

// Scheduling fence: forces the accumulators to be final here and keeps the
// next direction's loads after it.  Without it the compiler issues all
// eight neighbours' loads first and delays the arithmetic, so every loaded
// value stays live and the register file overflows.  The empty asm only
// names registers; it emits no instruction.
template <class R>
__device__ inline void fence(cx<R> acc[4][3]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) asm volatile("" : "+v"(acc[s][c].re), "+v"(acc[s][c].im)::"memory");
}

template <class R, int MU, bool G5IN, class Src>
__device__ inline void hop_dir(cx<R> acc[4][3], const cx<R> *U,
                               const Src &in, int p, int i, int nf, int nb,
                               size_t Vh) {
  Half<R> h, g;
  // forward: (1 - g_mu) U_mu(x) psi(x + mu); the link lives at x (parity p)
  project<R, MU, true, G5IN>(in, nf, Vh, h);
  link_mul<R>(U + ((size_t(p) * 4 + MU) * 9) * Vh + i, Vh, h, g);
  accumulate<R, MU, true>(acc, g);
  fence(acc);
  // backward: (1 + g_mu) U_mu(x - mu)^+ psi(x - mu); link at x - mu (parity 1-p)
  project<R, MU, false, G5IN>(in, nb, Vh, h);
  link_dag_mul<R>(U + ((size_t(1 - p) * 4 + MU) * 9) * Vh + nb, Vh, h, g);
  accumulate<R, MU, false>(acc, g);
  fence(acc);
}

}  // namespace st
}  // namespace lqcd
