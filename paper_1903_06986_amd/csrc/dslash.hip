// Wilson hopping stencil (Sec. 5.1 Eqs. (24)-(25)) on even/odd fields.
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
// Data layouts (per right-hand side, per parity; stencil.h): fields are
// stored as 16-byte granules per site, granule-major ([granules][Vh]), so a
// lane gathers a neighbour with 16-byte loads that a wavefront issues as
// contiguous 1 KiB runs: FP64 [12][Vh] complex, the FP32 odd temporary of
// the even/odd operator in component pairs [6][Vh], 16-bit storage in
// component quads [3][Vh] plus per-site scales.  The FP32 fields the
// solvers hold are component-major [12][Vh].  Links: [parity][mu][9][Vh].
//
// Kernels and launch logic; the device building blocks (half-spinor
// projection, link products, sources of plain or 16-bit fields) are in
// stencil.h.
#include "common.h"
#include "cplx.h"
#include "fields.h"
#include "half.h"
#include "stencil.h"

namespace lqcd {

namespace {

using namespace st;

// Thread mapping: the NB right-hand sides of a group are the fastest lane
// index, so the NB lanes that share a site issue the same link addresses
// and one wave load fetches each link once for all NB of them (links are
// 2/3 of a single right-hand side's bytes).  Spinor accesses stay in
// contiguous runs of 64/NB sites per right-hand side.
template <class R, bool G5IN, bool G5OUT, bool SELF, int NB, class SrcIn, class SrcSelf, class OutT>
// 3 waves per SIMD caps FP64 at 128 VGPRs (4 waves resident, no spills).
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8)))
    k_hop(Geom g, int p, const cx<R> *U, SrcIn in,
          SrcSelf self, cx<R> *out, cx<R> alpha, R beta,
          size_t in_stride, size_t self_stride, size_t out_stride, int nrhs, int xq, int ngr,
          int nbx, int site_major) {
  // XCD-aware block order: workgroups are dispatched round-robin over the
  // 8 XCDs, so hardware block h runs on XCD h % 8.  Logical block
  // (h % 8) * xq + h / 8 gives every XCD one contiguous range.  Within it
  // either the right-hand-side group varies fastest (all groups of a site
  // block run back to back on one XCD and share its links in L2), or, with
  // site_major, the site block does (an XCD sweeps whole right-hand sides,
  // so the window of neighbouring timeslices stays in its L2 while the
  // links are shared through the last-level cache).
  const int L = int(blockIdx.x % 8) * xq + int(blockIdx.x / 8);
  const int bx = site_major ? L % nbx : L / ngr, grp = site_major ? L / nbx : L % ngr;
  const int i = bx * (kBlock / NB) + threadIdx.x / NB;
  const int rr = grp * NB + threadIdx.x % NB;
  if (i >= g.Vh || rr >= nrhs) return;
  const size_t Vh = size_t(g.Vh);
  const size_t rhs = rr;
  in = in.at(rhs * in_stride);
  char *ob = reinterpret_cast<char *>(out) + rhs * out_stride * OutT::kElemBytes;
  const int Lxh = g.Lxh, Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
  const int xh = i % Lxh;
  int r = i / Lxh;
  const int y = r % Ly;
  r /= Ly;
  const int z = r % Lz;
  const int t = r / Lz;
  const int x = 2 * xh + ((p + y + z + t) & 1);
  const int rowb = i - xh;

  cx<R> acc[4][3];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[s][c] = mk<R>(0, 0);

  {  // x
    int xf = (x + 1 == Lx) ? 0 : x + 1, xb = (x == 0) ? Lx - 1 : x - 1;
    hop_dir<R, 0, G5IN>(acc, U, in, p, i, rowb + (xf >> 1), rowb + (xb >> 1), Vh);
  }
  {  // y
    const int s = Lxh;
    int nf = (y == Ly - 1) ? i - s * (Ly - 1) : i + s;
    int nb = (y == 0) ? i + s * (Ly - 1) : i - s;
    hop_dir<R, 1, G5IN>(acc, U, in, p, i, nf, nb, Vh);
  }
  {  // z
    const int s = Lxh * Ly;
    int nf = (z == Lz - 1) ? i - s * (Lz - 1) : i + s;
    int nb = (z == 0) ? i + s * (Lz - 1) : i - s;
    hop_dir<R, 2, G5IN>(acc, U, in, p, i, nf, nb, Vh);
  }
  {  // t
    const int s = Lxh * Ly * Lz;
    int nf = (t == Lt - 1) ? i - s * (Lt - 1) : i + s;
    int nb = (t == 0) ? i + s * (Lt - 1) : i - s;
    hop_dir<R, 3, G5IN>(acc, U, in, p, i, nf, nb, Vh);
  }

  if (SELF) self = self.at(rhs * self_stride);
  const typename SrcSelf::Ctx ssc = SELF ? self.site(i) : typename SrcSelf::Ctx{};
  cx<R> v[12];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[s * 3 + c] = beta * acc[s][c];
      if (SELF) {
        cx<R> w = self.ld(ssc, i, s * 3 + c, Vh);
        if (G5IN && s >= 2) w = -w;
        v[s * 3 + c] = v[s * 3 + c] + alpha * w;
      }
      if (G5OUT && s >= 2) v[s * 3 + c] = -v[s * 3 + c];
    }
  OutT::template store12<false>(ob, uint32_t(i) * OutT::kSiteBytes, 0u, Vh, v);
}

// Link-tiled form for many right-hand sides: a workgroup owns T
// consecutive output sites (T = 16, 32 or 64), stages their 8 links (4 forward
// at the sites, 4 backward at the neighbours x - mu) in LDS once, then
// applies the stencil to every right-hand side, RS = 256 / T of them at a
// time.  The lane index is the site within the tile, so each spinor access
// of a wave is one contiguous run of sites, and the links cross HBM once
// per launch instead of once per right-hand side.  Field accesses use a
// wave-uniform base (the wave's first right-hand side) and 32-bit lane byte
// offsets (the host checks that they fit).
// One of the 8 terms of the stencil (LEG = 2 mu + 0 forward / 1 backward)
// from a settled raw neighbour, with its link from the LDS tile.
template <class R, int LEG, bool G5IN, class RawT>
__device__ inline void hop_leg(cx<R> acc[4][3], const cx<R> *sU, int T, const RawT &raw, R one) {
  constexpr int MU = LEG / 2;
  constexpr bool FWD = (LEG % 2) == 0;
  Half<R> h;
  project_raw<R, MU, FWD, G5IN>(raw, h, one);
  link_accumulate<R, MU, FWD>(acc, sU + ((FWD ? 0 : 4) + MU) * 9 * T, T, h, raw.scale());
}

// Step LEG of the software pipeline over the 8 neighbours, D deep: the
// loads of neighbour LEG + D go out into the buffer that LEG has just
// consumed, so D neighbours' loads are in flight while one is computed.
template <class R, int LEG, int D, bool G5IN, class Src>
__device__ inline void hop_step(cx<R> acc[4][3], const cx<R> *sU, int T, const Src &in,
                                const uint32_t off[8], uint32_t ib, size_t Vh, Raw<Src> &buf, R one) {
  settle(buf);
  hop_leg<R, LEG, G5IN>(acc, sU, T, buf, one);
  if (LEG + D < 8) fetch_at(in, off[LEG + D < 8 ? LEG + D : 0], ib, Vh, buf);
  fence(acc);
}

// Steps LEG..7; the self term's loads go out at the first step that
// issues no neighbour load, into the registers that step has freed.
template <class R, int LEG, int D, bool G5IN, bool SELF, class Src, class SS>
__device__ inline void hop_steps(cx<R> acc[4][3], const cx<R> *sU, int T, const Src &in,
                                 const uint32_t off[8], uint32_t ib, size_t Vh, Raw<Src> (&buf)[D], R one,
                                 const SS &self, uint32_t so, uint32_t sb, Raw<SS> &rs) {
  if constexpr (LEG < 8) {
    hop_step<R, LEG, D, G5IN>(acc, sU, T, in, off, ib, Vh, buf[LEG % D], one);
    if constexpr (SELF && LEG + D == 8) fetch_at(self, so, sb, Vh, rs);
    hop_steps<R, LEG + 1, D, G5IN, SELF>(acc, sU, T, in, off, ib, Vh, buf, one, self, so, sb, rs);
  }
}

// Tile order of k_hop_tile.  tb == 0: tiles are T consecutive sites of the
// half lattice in index order.  tb > 0 (plane-blocked): a tile lies in one
// (z, t) plane of ppl = Lxh * Ly sites (nbp tiles per plane, the last one
// ragged), and the tile sequence runs over blocks of tb timeslices, z
// within a block, t fastest: the planes whose spinors a tile reads through
// its z and t neighbours are then at most tb planes of the sequence away,
// so they are still in the XCD's L2 when the next tile needs them.
// With rg > 0 the right-hand sides are split into groups of rg.  nest == 0:
// the logical workgroup index runs over (group, tile), group slowest: every
// XCD range then covers one group over part of the lattice, and its L2
// holds that group's spinors only (the links are read once per group).
// nest > 0 (plane order; nest = tiles per block of tb timeslices): the index
// runs over (block, group, tile within the block), so an XCD sweeps its own
// block once per group in turn: its L2 holds one group's planes at a time,
// and the block's links are read once per group (from the last-level cache
// after the first).
struct TileMap {
  int tb, nbp, ppl;
  int rg, ntg;  // right-hand sides per group (0: one group), tiles per group
  int nest;     // tiles per block of timeslices when groups are nested in blocks (0: not nested)
};

// Waves per SIMD the tiled stencil is compiled for: 4 (128 VGPRs) with
// 16-bit sources, whose three raw neighbours in flight fit there; 3 (168
// VGPRs) otherwise.
template <class R, class SrcIn>
constexpr int hop_tile_waves = (sizeof(R) == 4 && SrcIn::kElemBytes == 4) ? 4 : 3;

template <class R, bool G5IN, bool G5OUT, bool SELF, int T, class SrcIn, class SrcSelf, class OutT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(hop_tile_waves<R, SrcIn>, 8)))
    k_hop_tile(Geom g, int p, const cx<R> *U, SrcIn in, SrcSelf self, cx<R> *out, cx<R> alpha,
               R beta, size_t in_stride, size_t self_stride, size_t out_stride, int nrhs, int xq,
               TileMap tm) {
  static_assert(T == 16 || T == 32 || T == 64, "tile of 16, 32 or 64 sites");
  constexpr int RS = kBlock / T;    // right-hand sides per pass
  constexpr int SPW = 64 / T;       // right-hand-side slots per wave
  // neighbours' loads in flight per wave: 3 for 16-bit sources (128
  // VGPRs, 4 waves per SIMD), 2 for FP32 ones (a third spills at 168), 1 in
  // FP64 (a second raw FP64 site would cost a wave per SIMD)
  constexpr int D = sizeof(R) == 8 ? 1 : (SrcIn::kElemBytes == 4 ? 3 : 2);
  __shared__ cx<R> sU[8 * 9 * T];  // [direction: 4 forward, 4 backward][entry][site]
  // XCD-aware tile order (as in k_hop): each XCD walks one contiguous range
  const int lidx = int(blockIdx.x % 8) * xq + int(blockIdx.x / 8);
  int grp = 0, tile = lidx;
  if (tm.rg > 0 && tm.nest > 0) {
    const int ng = (nrhs + tm.rg - 1) / tm.rg, per = ng * tm.nest;
    const int rem = lidx % per;
    grp = rem / tm.nest;
    tile = (lidx / per) * tm.nest + rem % tm.nest;
  } else if (tm.rg > 0) {
    grp = lidx / tm.ntg;
    tile = lidx % tm.ntg;
  }
  const int rlo = grp * tm.rg, rhi = tm.rg > 0 ? min(nrhs, rlo + tm.rg) : nrhs;
  if (rlo >= nrhs) return;  // whole workgroup: padding of the grid
  int i0, lim;
  if (tm.tb == 0) {
    i0 = tile * T;
    lim = g.Vh;
  } else {
    const int b = tile % tm.nbp;
    int q = tile / tm.nbp;
    const int tt = q % tm.tb;
    q /= tm.tb;
    const int z = q % g.L[2], t = (q / g.L[2]) * tm.tb + tt;
    if (t >= g.L[3]) return;  // whole workgroup: a partial last block of timeslices
    const int pb = (t * g.L[2] + z) * tm.ppl;
    i0 = pb + b * T;
    lim = pb + tm.ppl;
  }
  if (i0 >= lim) return;  // whole workgroup: padding of the grid
  const size_t Vh = size_t(g.Vh);
  const int il = threadIdx.x % T, slot = threadIdx.x / T;
  const int slot0 = __builtin_amdgcn_readfirstlane(int(threadIdx.x / 64)) * SPW;  // wave's first slot
  const int i = i0 + il;
  const bool site_ok = i < lim;
  const int Lxh = g.Lxh, Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
  int nf[4] = {0, 0, 0, 0}, nb[4] = {0, 0, 0, 0};
  if (site_ok) {
    const int xh = i % Lxh;
    int r = i / Lxh;
    const int y = r % Ly;
    r /= Ly;
    const int z = r % Lz;
    const int t = r / Lz;
    const int x = 2 * xh + ((p + y + z + t) & 1);
    const int rowb = i - xh;
    nf[0] = rowb + (((x + 1 == Lx) ? 0 : x + 1) >> 1);
    nb[0] = rowb + (((x == 0) ? Lx - 1 : x - 1) >> 1);
    int st = Lxh;
    nf[1] = (y == Ly - 1) ? i - st * (Ly - 1) : i + st;
    nb[1] = (y == 0) ? i + st * (Ly - 1) : i - st;
    st *= Ly;
    nf[2] = (z == Lz - 1) ? i - st * (Lz - 1) : i + st;
    nb[2] = (z == 0) ? i + st * (Lz - 1) : i - st;
    st *= Lz;
    nf[3] = (t == Lt - 1) ? i - st * (Lt - 1) : i + st;
    nb[3] = (t == 0) ? i + st * (Lt - 1) : i - st;
    // stage: slot s loads the (direction, entry) pairs s, s + RS, ...
    for (int q = slot; q < 72; q += RS) {
      const int d = q / 9, e = q % 9;
      const size_t src = d < 4 ? ((size_t(p) * 4 + d) * 9 + e) * Vh + i
                               : ((size_t(1 - p) * 4 + (d - 4)) * 9 + e) * Vh + nb[d - 4];
      sU[q * T + il] = ldc_nt(U + src);  // read once per launch: keep L2 for the spinors
    }
  }
  __syncthreads();
  if (!site_ok) return;
  const cx<R> *su = sU + il;
  R one = 1;  // unit factor of the projection's FMAs, opaque to the compiler
  asm volatile("" : "+s"(one));
  // lane byte offsets within the wave's fields (loop-invariant)
  const uint32_t sl = uint32_t(slot - slot0);
  const uint32_t ib = sl * uint32_t(in_stride * SrcIn::kElemBytes),
                 sb = sl * uint32_t(self_stride * SrcSelf::kElemBytes), ob = sl * uint32_t(out_stride * OutT::kElemBytes);
  uint32_t of[4], obk[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    of[d] = ib + uint32_t(nf[d]) * SrcIn::kSiteBytes;
    obk[d] = ib + uint32_t(nb[d]) * SrcIn::kSiteBytes;
  }
  const uint32_t so = sb + uint32_t(i) * SrcSelf::kSiteBytes, oo = ob + uint32_t(i) * OutT::kSiteBytes;
#pragma unroll 1
  for (int r0 = rlo + slot0; r0 < rhi; r0 += RS) {
    if (r0 + int(sl) >= rhi) break;  // this lane's right-hand side is past the end
    const size_t rw = size_t(r0);     // wave-uniform
    const SrcIn inr = in.at(rw * in_stride);
    cx<R> acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[s][c] = mk<R>(0, 0);
    // Offsets pass through an empty asm each iteration so that the compiler
    // does not hoist per-component addresses out of the loop.  Order of the
    // neighbours: x forward, x backward, y forward, ..., t backward.
    uint32_t off[8];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      off[2 * d] = of[d];
      off[2 * d + 1] = obk[d];
      asm volatile("" : "+v"(off[2 * d]), "+v"(off[2 * d + 1]));
    }
    SrcSelf sr = self;
    if (SELF) sr = self.at(rw * self_stride);
    Raw<SrcSelf> rs;
    Raw<SrcIn> rb[D];
#pragma unroll
    for (int l = 0; l < D; ++l) fetch_at(inr, off[l], ib, Vh, rb[l]);
    hop_steps<R, 0, D, G5IN, SELF>(acc, su, T, inr, off, ib, Vh, rb, one, sr, so, sb, rs);
    char *o = reinterpret_cast<char *>(out) + rw * out_stride * OutT::kElemBytes;
    if (SELF) settle(rs);
    cx<R> v[12];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v[s * 3 + c] = beta * acc[s][c];
        if (SELF) {
          cx<R> w = rs.get(s * 3 + c);
          if (G5IN && s >= 2) w = -w;
          v[s * 3 + c] = v[s * 3 + c] + alpha * w;
        }
        if (G5OUT && s >= 2) v[s * 3 + c] = -v[s * 3 + c];
      }
    OutT::template store12<true>(o, oo, ob, Vh, v);
  }
}

template <class R, bool A, bool B, bool C, int T, class SI, class SS, class OT>
void launch_hop_tile(lqcd_ctx *c, Timed &tm, int p, const cx<R> *U, SI in, SS self, void *out,
                     cdouble alpha, double beta, int nrhs, size_t si, size_t ss, size_t so) {
  const Geom &g = c->g;
  TileMap map{c->hop_tblock[std::is_same<R, double>::value ? 0 : 1], 0, g.Lxh * g.L[1], 0, 0, 0};
  if (map.tb < 0)  // automatic: plane order when planes split into whole tiles, one block per XCD
    map.tb = (map.ppl % T == 0 && g.L[3] >= 8) ? (g.L[3] + 7) / 8 : 0;
  int ntile;
  if (map.tb > 0) {
    map.tb = std::min(map.tb, g.L[3]);
    map.nbp = (map.ppl + T - 1) / T;
    const int nblk = (g.L[3] + map.tb - 1) / map.tb;
    ntile = nblk * map.tb * g.L[2] * map.nbp;
  } else {
    ntile = int((g.Vh + T - 1) / T);
  }
  // nested groups: automatic (-1) in FP64 only, groups of 8 right-hand
  // sides, whose planes (8 x 192 B per site) then stay in an XCD's L2 across
  // its block (24^3 x 32, 16 right-hand sides: 741 -> 671 us and 650 -> 592
  // us for the two halves); in FP32 the staged links' cost per workgroup
  // outweighs it (288 -> 313 us), so off
  int rn = c->hop_rnest;
  if (rn < 0) rn = std::is_same<R, double>::value ? 8 : 0;
  const int rg = rn > 0 && map.tb > 0 ? rn : c->hop_rgroup;
  if (rg > 0 && rg < nrhs) {
    map.rg = rg;
    map.ntg = ntile;
    if (rn > 0 && map.tb > 0) map.nest = map.tb * g.L[2] * map.nbp;
    ntile *= (nrhs + rg - 1) / rg;
  }
  const int xq = (ntile + 7) / 8;
  LQCD_TLAUNCH(tm, true, true, (k_hop_tile<R, A, B, C, T, SI, SS, OT>), dim3(8 * xq), dim3(kBlock), 0, c->stream, g, p,
                     U, in, self, static_cast<cx<R> *>(out), mk<R>(R(alpha.real()), R(alpha.imag())),
                     R(beta), si, ss, so, nrhs, xq, map);
}

template <class R, bool A, bool B, bool C, int NB, class SI, class SS, class OT>
void launch_hop_nb(lqcd_ctx *c, Timed &tm, int p, const cx<R> *U, SI in, SS self, void *out,
                   cdouble alpha, double beta, int nrhs, size_t si, size_t ss, size_t so) {
  const Geom &g = c->g;
  const int nbx = int(nblocks(g.Vh, kBlock / NB));
  const int ngr = (nrhs + NB - 1) / NB;
  const int xq = (nbx * ngr + 7) / 8;  // logical blocks per XCD (the grid is padded to 8 * xq)
  dim3 grid(8 * xq);
  LQCD_TLAUNCH(tm, true, true, (k_hop<R, A, B, C, NB, SI, SS, OT>), grid, dim3(kBlock), 0, c->stream, g, p, U, in,
                     self, static_cast<cx<R> *>(out), mk<R>(R(alpha.real()), R(alpha.imag())), R(beta),
                     si, ss, so, nrhs, xq, ngr, nbx, c->hop_order);
}

// Bytes per site of one stored half field of a source type.
template <class S>
struct SrcBytes;
template <class R>
struct SrcBytes<SrcPlain<R>> {
  static constexpr double v = 12.0 * sizeof(cx<R>);
};
template <>
struct SrcBytes<SrcPair> {
  static constexpr double v = 96.0;
};
template <HKind K>
struct SrcBytes<SrcHalf<K>> {
  static constexpr double v = 52.0;
};

template <class R, bool A, bool B, bool C, class SI, class SS, class OT = OutPlain<R>>
void launch_hop_src(lqcd_ctx *c, int p, SI in, SS self, void *out, cdouble alpha,
                    double beta, int nrhs, size_t si, size_t ss, size_t so) {
  const Geom &g = c->g;
  const cx<R> *U = static_cast<const cx<R> *>(std::is_same<R, double>::value ? c->U64.ptr : c->U32.ptr);
  // algorithmic bytes: all 8 Vh links once, input and output half fields
  // (and the self term) once per right-hand side
  const double bytes = double(g.Vh) * (72.0 * sizeof(cx<R>) +
                                       nrhs * (SrcBytes<SI>::v + OT::kFieldBytes + (C ? SrcBytes<SS>::v : 0.0)));
  Timed tm(c, std::is_same<R, double>::value ? LQCD_KC_HOP64 : LQCD_KC_HOP32, bytes);
  const int pi = std::is_same<R, double>::value ? 0 : 1;
  const int nbmax = c->hop_nb[pi];
  // tiles of ts sites (links of 18 KiB in FP64, 9 KiB in FP32 per 16
  // sites in LDS), doubled while the launch has fewer right-hand sides
  // than one pass of the tile takes (256 / ts); FP64 tiles of 16 or 32
  // sites, FP32 16, 32 or 64
  constexpr int tmax = std::is_same<R, double>::value ? 32 : 64;
  int ts = c->hop_tsites[pi];
  while (ts < tmax && nrhs < kBlock / ts) ts *= 2;
  // the tiled form addresses a wave's fields by 32-bit byte offsets: one
  // right-hand-side stride per extra slot of a wave plus a half field
  auto fits = [&](size_t stride, double elem, double site) {
    return double(64 / ts - 1) * double(stride) * elem + double(g.Vh) * site < 4294967295.0;
  };
  const bool offs_ok = fits(si, SI::kElemBytes, SI::kSiteBytes) &&
                       (!C || fits(ss, SS::kElemBytes, SS::kSiteBytes)) && fits(so, OT::kElemBytes, OT::kSiteBytes);
  const bool tiled = c->hop_tile[pi] && offs_ok && ts <= tmax && nrhs >= kBlock / ts;
  if (tiled && ts == 16)
    launch_hop_tile<R, A, B, C, 16, SI, SS, OT>(c, tm, p, U, in, self, out, alpha, beta, nrhs, si, ss, so);
  else if (tiled && ts == 32)
    launch_hop_tile<R, A, B, C, 32, SI, SS, OT>(c, tm, p, U, in, self, out, alpha, beta, nrhs, si, ss, so);
  else if (tiled)
    launch_hop_tile<R, A, B, C, tmax, SI, SS, OT>(c, tm, p, U, in, self, out, alpha, beta, nrhs, si, ss, so);
  else if (nrhs >= 8 && nbmax >= 8)
    launch_hop_nb<R, A, B, C, 8, SI, SS, OT>(c, tm, p, U, in, self, out, alpha, beta, nrhs, si, ss, so);
  else if (nrhs >= 4 && nbmax >= 4)
    launch_hop_nb<R, A, B, C, 4, SI, SS, OT>(c, tm, p, U, in, self, out, alpha, beta, nrhs, si, ss, so);
  else if (nrhs >= 2 && nbmax >= 2)
    launch_hop_nb<R, A, B, C, 2, SI, SS, OT>(c, tm, p, U, in, self, out, alpha, beta, nrhs, si, ss, so);
  else launch_hop_nb<R, A, B, C, 1, SI, SS, OT>(c, tm, p, U, in, self, out, alpha, beta, nrhs, si, ss, so);
  LQCD_HIP(hipGetLastError());
}

template <class R, bool A, bool B, bool C>
void launch_hop(lqcd_ctx *c, int p, const void *in, const void *self, void *out, cdouble alpha,
                double beta, int nrhs, size_t si, size_t ss, size_t so) {
  launch_hop_src<R, A, B, C>(c, p, SrcPlain<R>{static_cast<const cx<R> *>(in)},
                             SrcPlain<R>{static_cast<const cx<R> *>(self)}, out, alpha, beta, nrhs, si,
                             ss, so);
}

}  // namespace

template <class R>
void hop_half(lqcd_ctx *c, int p, const void *in, const void *self, void *out, cdouble alpha,
              double beta, bool g5_in, bool g5_out, int nrhs, size_t si, size_t ss, size_t so) {
  if (nrhs <= 0) return;
  const bool hs = self != nullptr;
  if (!g5_in && !g5_out) {
    if (hs) launch_hop<R, false, false, true>(c, p, in, self, out, alpha, beta, nrhs, si, ss, so);
    else launch_hop<R, false, false, false>(c, p, in, self, out, alpha, beta, nrhs, si, ss, so);
  } else if (g5_in && !g5_out) {
    if (hs) launch_hop<R, true, false, true>(c, p, in, self, out, alpha, beta, nrhs, si, ss, so);
    else launch_hop<R, true, false, false>(c, p, in, self, out, alpha, beta, nrhs, si, ss, so);
  } else if (g5_in && g5_out) {
    if (hs) launch_hop<R, true, true, true>(c, p, in, self, out, alpha, beta, nrhs, si, ss, so);
    else launch_hop<R, true, true, false>(c, p, in, self, out, alpha, beta, nrhs, si, ss, so);
  } else {
    if (hs) launch_hop<R, false, true, true>(c, p, in, self, out, alpha, beta, nrhs, si, ss, so);
    else launch_hop<R, false, true, false>(c, p, in, self, out, alpha, beta, nrhs, si, ss, so);
  }
}

// Full-lattice operators: per rhs the field is [even half][odd half].
template <class R>
void apply_full(lqcd_ctx *c, lqcd_op op, const void *in, void *out, int nrhs, size_t sin,
                size_t sout) {
  const size_t hl = half_len(c->g);
  const double k = c->kappa;
  const R *ib = static_cast<const R *>(in);
  R *ob = static_cast<R *>(out);
  for (int p = 0; p < 2; ++p) {
    const void *src = ib + 2 * hl * (1 - p);  // opposite parity of the input
    const void *slf = ib + 2 * hl * p;
    void *dst = ob + 2 * hl * p;
    switch (op) {
      case LQCD_OP_HOP:
        hop_half<R>(c, p, src, nullptr, dst, cdouble(0, 0), 1.0, false, false, nrhs, sin, 0, sout);
        break;
      case LQCD_OP_M:
        hop_half<R>(c, p, src, slf, dst, cdouble(1, 0), -k, false, false, nrhs, sin, sin, sout);
        break;
      case LQCD_OP_MG5:
        hop_half<R>(c, p, src, slf, dst, cdouble(1, 0), -k, true, false, nrhs, sin, sin, sout);
        break;
      case LQCD_OP_MDAG:
        hop_half<R>(c, p, src, slf, dst, cdouble(1, 0), -k, true, true, nrhs, sin, sin, sout);
        break;
      default:
        LQCD_CHECK(false, LQCD_EINVAL, "apply_full: operator %d is not a full-lattice operator", int(op));
    }
  }
}

// Mhat x_e = x_e - kappa^2 D_eo D_oe x_e  (Sec. 7 even/odd reduction).  The
// odd temporary never leaves the operator: in FP32 it is written and read
// in component pairs (16-byte granules).
template <class R>
void apply_schur(lqcd_ctx *c, const void *in, void *out, void *tmp_odd, int nrhs, size_t sin,
                 size_t sout, size_t stmp) {
  const double k = c->kappa;
  if constexpr (std::is_same<R, float>::value) {
    if (nrhs <= 0) return;
    const SrcPlain<float> x{static_cast<const cx<float> *>(in)};
    launch_hop_src<float, false, false, false, SrcPlain<float>, SrcPlain<float>, OutPair>(
        c, 1, x, SrcPlain<float>{nullptr}, tmp_odd, cdouble(0, 0), 1.0, nrhs, sin, 0, stmp);
    launch_hop_src<float, false, false, true>(c, 0, SrcPair{static_cast<const cx<float> *>(tmp_odd)}, x, out,
                                              cdouble(1, 0), -k * k, nrhs, stmp, sin, sout);
  } else {
    hop_half<R>(c, 1, in, nullptr, tmp_odd, cdouble(0, 0), 1.0, false, false, nrhs, sin, 0, stmp);
    hop_half<R>(c, 0, tmp_odd, in, out, cdouble(1, 0), -k * k, false, false, nrhs, stmp, sin, sout);
  }
}

// Mhat on stored 16-bit even fields (in: words, vectors sin words apart),
// FP32 output and odd temporary.
template <int KIND>
void apply_schur_h(lqcd_ctx *c, const void *in, void *out, void *tmp_odd, int nrhs, size_t sin,
                   size_t sout, size_t stmp) {
  if (nrhs <= 0) return;
  constexpr HKind K = static_cast<HKind>(KIND);
  const double k = c->kappa;
  const size_t n = half_len(c->g);
  const SrcHalf<K> hin{static_cast<const uint32_t *>(in), n};
  const SrcPlain<float> none{nullptr};
  launch_hop_src<float, false, false, false, SrcHalf<K>, SrcPlain<float>, OutPair>(c, 1, hin, none, tmp_odd,
                                                                                   cdouble(0, 0), 1.0, nrhs, sin,
                                                                                   0, stmp);
  launch_hop_src<float, false, false, true>(c, 0, SrcPair{static_cast<const cx<float> *>(tmp_odd)}, hin, out,
                                            cdouble(1, 0), -k * k, nrhs, stmp, sin, sout);
}
template void apply_schur_h<0>(lqcd_ctx *, const void *, void *, void *, int, size_t, size_t, size_t);
template void apply_schur_h<1>(lqcd_ctx *, const void *, void *, void *, int, size_t, size_t, size_t);

// Mhat - 1 = -kappa^2 D_eo D_oe on a 16-bit stored even input, FP32
// output in the pair layout of the odd temporary (16-byte granules of two
// components): the s-step Arnoldi's shifted power basis.  Without the unit
// term the even half reads no self term.
template <int KIND>
void apply_dd_h_pair(lqcd_ctx *c, const void *in, void *out, void *tmp_odd, int nrhs, size_t sin, size_t sout,
                     size_t stmp) {
  if (nrhs <= 0) return;
  constexpr HKind K = static_cast<HKind>(KIND);
  const double k = c->kappa;
  const size_t n = half_len(c->g);
  const SrcHalf<K> hin{static_cast<const uint32_t *>(in), n};
  const SrcPlain<float> none{nullptr};
  launch_hop_src<float, false, false, false, SrcHalf<K>, SrcPlain<float>, OutPair>(c, 1, hin, none, tmp_odd,
                                                                                   cdouble(0, 0), 1.0, nrhs, sin,
                                                                                   0, stmp);
  launch_hop_src<float, false, false, false, SrcPair, SrcPlain<float>, OutPair>(
      c, 0, SrcPair{static_cast<const cx<float> *>(tmp_odd)}, none, out, cdouble(0, 0), -k * k, nrhs, stmp, 0,
      sout);
}
template void apply_dd_h_pair<0>(lqcd_ctx *, const void *, void *, void *, int, size_t, size_t, size_t);
template void apply_dd_h_pair<1>(lqcd_ctx *, const void *, void *, void *, int, size_t, size_t, size_t);

// Mhat - 1 from a 16-bit stored input to a 16-bit stored output (kind
// KIND, words strides), FP32 arithmetic, odd temporary in the pair layout.
template <int KIND>
void apply_dd_hh(lqcd_ctx *c, const void *in, void *out, void *tmp_odd, int nrhs, size_t sin, size_t sout,
                 size_t stmp) {
  if (nrhs <= 0) return;
  constexpr HKind K = static_cast<HKind>(KIND);
  const double k = c->kappa;
  const SrcHalf<K> hin{static_cast<const uint32_t *>(in), half_len(c->g)};
  const SrcPlain<float> none{nullptr};
  launch_hop_src<float, false, false, false, SrcHalf<K>, SrcPlain<float>, OutPair>(c, 1, hin, none, tmp_odd,
                                                                                   cdouble(0, 0), 1.0, nrhs, sin,
                                                                                   0, stmp);
  launch_hop_src<float, false, false, false, SrcPair, SrcPlain<float>, OutHalf<K>>(
      c, 0, SrcPair{static_cast<const cx<float> *>(tmp_odd)}, none, out, cdouble(0, 0), -k * k, nrhs, stmp, 0,
      sout);
}
template void apply_dd_hh<0>(lqcd_ctx *, const void *, void *, void *, int, size_t, size_t, size_t);
template void apply_dd_hh<1>(lqcd_ctx *, const void *, void *, void *, int, size_t, size_t, size_t);

// Mhat - 1 in FP32 with input, output and odd temporary in the pair layout.
void apply_dd_pair(lqcd_ctx *c, const void *in, void *out, void *tmp_odd, int nrhs, size_t sin, size_t sout,
                   size_t stmp) {
  if (nrhs <= 0) return;
  const double k = c->kappa;
  const SrcPlain<float> none{nullptr};
  launch_hop_src<float, false, false, false, SrcPair, SrcPlain<float>, OutPair>(
      c, 1, SrcPair{static_cast<const cx<float> *>(in)}, none, tmp_odd, cdouble(0, 0), 1.0, nrhs, sin, 0, stmp);
  launch_hop_src<float, false, false, false, SrcPair, SrcPlain<float>, OutPair>(
      c, 0, SrcPair{static_cast<const cx<float> *>(tmp_odd)}, none, out, cdouble(0, 0), -k * k, nrhs, stmp, 0,
      sout);
}

template void hop_half<double>(lqcd_ctx *, int, const void *, const void *, void *, cdouble, double,
                               bool, bool, int, size_t, size_t, size_t);
template void hop_half<float>(lqcd_ctx *, int, const void *, const void *, void *, cdouble, double,
                              bool, bool, int, size_t, size_t, size_t);
template void apply_full<double>(lqcd_ctx *, lqcd_op, const void *, void *, int, size_t, size_t);
template void apply_full<float>(lqcd_ctx *, lqcd_op, const void *, void *, int, size_t, size_t);
template void apply_schur<double>(lqcd_ctx *, const void *, void *, void *, int, size_t, size_t, size_t);
template void apply_schur<float>(lqcd_ctx *, const void *, void *, void *, int, size_t, size_t, size_t);

}  // namespace lqcd

using namespace lqcd;

namespace {

size_t prec_bytes(lqcd_prec p) { return p == LQCD_F64 ? 16 : 8; }

// Mhat with the 16-bit stored input (LEX complex128 in and out): the even
// half is packed to FP32, stored with per-site scales, and the stencil
// reads the stored form; the odd half of the output is zero.
template <int KIND>
void wilson_apply_h(lqcd_ctx *c, const void *in, void *out, int nrhs) {
  const size_t hl = half_len(c->g), fl = full_len(c->g);
  const size_t ldh = hvec_words(size_t(c->g.Vh));
  const int blk = std::max(1, std::min(nrhs, 16));
  void *a = c->ws[5].ensure(2 * hl * blk * sizeof(cx<float>));
  void *b = c->ws[6].ensure(2 * hl * blk * sizeof(cx<float>));
  void *q = c->ws[4].ensure(ldh * blk * sizeof(uint32_t));
  void *tmp = c->ws[7].ensure(hl * blk * sizeof(cx<float>));
  for (int r0 = 0; r0 < nrhs; r0 += blk) {
    const int nb = std::min(blk, nrhs - r0);
    pack_eo<float>(c, static_cast<const cdouble *>(in) + r0 * fl, a, nb, 2 * hl);
    hquantize<KIND>(c, a, 2 * hl, nullptr, q, ldh, hl, nb);
    apply_schur_h<KIND>(c, q, b, tmp, nb, ldh, 2 * hl, hl);
    for (int r = 0; r < nb; ++r)
      fill_zero(c, static_cast<cx<float> *>(b) + (2 * r + 1) * hl, hl * sizeof(cx<float>));
    unpack_eo<float>(c, b, static_cast<cdouble *>(out) + r0 * fl, nb, 2 * hl);
  }
}

template <class R>
void wilson_apply_t(lqcd_ctx *c, lqcd_op op, lqcd_layout layout, const void *in, void *out,
                    int nrhs) {
  const size_t hl = half_len(c->g);
  if (layout == LQCD_LAYOUT_EO) {
    if (op == LQCD_OP_SCHUR) {
      void *tmp = c->ws[7].ensure(hl * nrhs * sizeof(cx<R>));
      apply_schur<R>(c, in, out, tmp, nrhs, hl, hl, hl);
    } else {
      apply_full<R>(c, op, in, out, nrhs, 2 * hl, 2 * hl);
    }
    return;
  }
  // LEX: pack -> apply -> unpack, in blocks of right-hand sides so the
  // scratch stays bounded.
  const int blk = std::max(1, std::min(nrhs, 16));
  void *a = c->ws[5].ensure(2 * hl * blk * sizeof(cx<R>));
  void *b = c->ws[6].ensure(2 * hl * blk * sizeof(cx<R>));
  const size_t fl = full_len(c->g);
  for (int r0 = 0; r0 < nrhs; r0 += blk) {
    int nb = std::min(blk, nrhs - r0);
    const cdouble *src = static_cast<const cdouble *>(in) + r0 * fl;
    cdouble *dst = static_cast<cdouble *>(out) + r0 * fl;
    pack_eo<R>(c, src, a, nb, 2 * hl);
    if (op == LQCD_OP_SCHUR) {
      void *tmp = c->ws[7].ensure(hl * blk * sizeof(cx<R>));
      // even block of a -> even block of b; odd block of b zeroed
      apply_schur<R>(c, a, b, tmp, nb, 2 * hl, 2 * hl, hl);
      for (int r = 0; r < nb; ++r)
        fill_zero(c, static_cast<cx<R> *>(b) + (2 * r + 1) * hl, hl * sizeof(cx<R>));
    } else {
      apply_full<R>(c, op, a, b, nb, 2 * hl, 2 * hl);
    }
    unpack_eo<R>(c, b, dst, nb, 2 * hl);
  }
}

}  // namespace

extern "C" lqcd_status wilson_apply(lqcd_ctx *c, lqcd_op op, lqcd_prec prec, lqcd_layout layout,
                                    const void *in, void *out, int nrhs) {
  return guarded([&] {
    LQCD_CHECK(c && in && out, LQCD_EINVAL, "wilson_apply: null argument");
    LQCD_CHECK(nrhs >= 0, LQCD_EINVAL, "wilson_apply: nrhs < 0");
    LQCD_CHECK(op >= LQCD_OP_M && op <= LQCD_OP_SCHUR, LQCD_EINVAL, "wilson_apply: bad operator");
    LQCD_CHECK(layout == LQCD_LAYOUT_LEX || layout == LQCD_LAYOUT_EO, LQCD_EINVAL,
               "wilson_apply: bad layout");
    LQCD_CHECK(in != out, LQCD_EINVAL, "wilson_apply: in and out must differ");
    if (nrhs == 0) return;
    if (prec == LQCD_F64) wilson_apply_t<double>(c, op, layout, in, out, nrhs);
    else if (prec == LQCD_F32) wilson_apply_t<float>(c, op, layout, in, out, nrhs);
    else if (prec == LQCD_F16 || prec == LQCD_BF16) {
      LQCD_CHECK(op == LQCD_OP_SCHUR && layout == LQCD_LAYOUT_LEX, LQCD_EINVAL,
                 "wilson_apply: 16-bit storage is available for LQCD_OP_SCHUR in LQCD_LAYOUT_LEX");
      if (prec == LQCD_F16) wilson_apply_h<0>(c, in, out, nrhs);
      else wilson_apply_h<1>(c, in, out, nrhs);
    } else LQCD_CHECK(false, LQCD_EINVAL, "wilson_apply: precision %d not available", int(prec));
    (void)prec_bytes;
  });
}
