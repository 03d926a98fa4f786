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
template <bool FWD>
__device__ inline cx<double> ps_half(const cx<double> a[12], const cx<double> b[12],
                                     const cx<double> *u, size_t Vh, int mu) {
  cx<double> w[12];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cx<double> v = mk(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k)
        v = v + (FWD ? ldc(u + (3 * i + k) * Vh) * b[3 * s + k]        // U b
                     : cmulc(ldc(u + (3 * k + i) * Vh), b[3 * s + k]));  // U^+ b
      w[3 * s + i] = v;
    }
  const SpinPerm &gm = kGamma[1 + mu];
  cx<double> acc = mk(0.0, 0.0);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int col = gm.col[s];
    const cx<double> gv = mk(FWD ? -gm.re[s] : gm.re[s], FWD ? -gm.im[s] : gm.im[s]);
#pragma unroll
    for (int i = 0; i < 3; ++i) acc = acc + cmulc(a[3 * s + i], w[3 * s + i] + gv * w[3 * col + i]);
  }
  return acc;
}

}  // namespace lqcd
