// The point-split vector operator of Table 2: for direction mu,
//   (Theta(mu) psi)(x) = kappa [ (1 + g_mu) U_mu(x - mu)^+ psi(x - mu)
//                              - (1 - g_mu) U_mu(x) psi(x + mu) ],
// kappa times the backward minus the forward hop of P along mu.  Operator
// codes 5..8 of the C ABI are mu = 0..3 (x, y, z, t).
#pragma once

#include "cplx.h"
#include "gamma.h"

namespace lqcd {

constexpr int kNumPS = 4;                   // point-split directions
constexpr int kNumOps = kNumTheta + kNumPS;  // operator codes 0..8

// Link U_mu at lexicographic coordinates (x, y, z, t) in the even/odd layout
// [parity][mu][9][Vh]; entries Vh apart.
__device__ inline const cx<double> *ps_link(const cx<double> *U, const Geom &g, int x, int y, int z,
                                            int t, int mu) {
  const int p = (x + y + z + t) & 1;
  const int s = x + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
  return U + ((size_t(p) * 4 + mu) * 9) * g.Vh + (s >> 1);
}

// One half of a^+ Theta(mu) b at a site: FWD = a^+ (1 - g_mu) U b with
// b = b(x + mu), u = U_mu(x); else a^+ (1 + g_mu) U^+ b with b = b(x - mu),
// u = U_mu(x - mu) (link entries Vh apart).  Then
//   a^+ Theta(mu) b = kappa (half<false> - half<true>).
// The spin factor acts first (it commutes with the colour link): h =
// (1 -+ g_mu) b, whose partner spin is 3 - s for mu = 0, 1 and s ^ 2 for
// mu = 2, 3 in this basis (selected between two fixed indices, so no
// array is indexed at run time); then a^+ U h row by row of U.
template <bool FWD>
__device__ inline cx<double> ps_half(const cx<double> a[12], const cx<double> b[12],
                                     const cx<double> *u, size_t Vh, int mu) {
  const SpinPerm &gm = kGamma[1 + mu];
  cx<double> h[12];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const cx<double> gv = mk(FWD ? -gm.re[s] : gm.re[s], FWD ? -gm.im[s] : gm.im[s]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const cx<double> partner = mu < 2 ? b[3 * (3 - s) + k] : b[3 * (s ^ 2) + k];
      h[3 * s + k] = b[3 * s + k] + gv * partner;
    }
  }
  cx<double> acc = mk(0.0, 0.0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cx<double> r0, r1, r2;  // row i of U, or of U^+
    if (FWD) {
      r0 = ldc(u + (3 * i + 0) * Vh);
      r1 = ldc(u + (3 * i + 1) * Vh);
      r2 = ldc(u + (3 * i + 2) * Vh);
    } else {
      const cx<double> c0 = ldc(u + (0 * 3 + i) * Vh), c1 = ldc(u + (1 * 3 + i) * Vh),
                       c2 = ldc(u + (2 * 3 + i) * Vh);
      r0 = mk(c0.re, -c0.im);
      r1 = mk(c1.re, -c1.im);
      r2 = mk(c2.re, -c2.im);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
      acc = acc + cmulc(a[3 * s + i], r0 * h[3 * s] + r1 * h[3 * s + 1] + r2 * h[3 * s + 2]);
  }
  return acc;
}

}  // namespace lqcd
