// Dirac matrices of the library's convention (Euclidean, hermitian, chiral
// basis): g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0, 1], [1, 0]],
// g_5 = g_1 g_2 g_3 g_4 = diag(1, 1, -1, -1).  Operator codes Theta:
// 0 = identity, 1..4 = g_1..g_4 (Table 2 of the paper: scalar and local
// vector).  Every row of these matrices has a single nonzero entry, stored
// as (column, value): (Theta psi)_s = val[s] * psi_{col[s]}.
#pragma once

#include <complex>

namespace lqcd {

struct SpinPerm {
  int col[4];
  double re[4], im[4];
};

// index 0..4: identity, g1, g2, g3, g4; index 5: g5
constexpr SpinPerm kGamma[6] = {
    {{0, 1, 2, 3}, {1, 1, 1, 1}, {0, 0, 0, 0}},
    {{3, 2, 1, 0}, {0, 0, 0, 0}, {-1, -1, 1, 1}},     // g1: -i, -i, i, i
    {{3, 2, 1, 0}, {-1, 1, 1, -1}, {0, 0, 0, 0}},     // g2: -1, 1, 1, -1
    {{2, 3, 0, 1}, {0, 0, 0, 0}, {-1, 1, 1, -1}},     // g3: -i, i, i, -i
    {{2, 3, 0, 1}, {1, 1, 1, 1}, {0, 0, 0, 0}},       // g4
    {{0, 1, 2, 3}, {1, 1, -1, -1}, {0, 0, 0, 0}},     // g5
};

// Dense 4x4 form (host), M[row][col].
inline void gamma_dense(int idx, std::complex<double> M[4][4]) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) M[r][c] = 0;
  for (int r = 0; r < 4; ++r)
    M[r][kGamma[idx].col[r]] = std::complex<double>(kGamma[idx].re[r], kGamma[idx].im[r]);
}

}  // namespace lqcd
