// Deflation space and solver internals shared by the solver and the
// hermitian-forced subtraction.
#pragma once

#include <mutex>

#include "common.h"
#include "smallla.h"

// Opaque handle of the C ABI: the deflation data A V_k = V_{k+1} Hbar_k
// left by GMRES-DR (Sec. 7), for the operator it was built with.
// A deflation space may serve several contexts of its lattice and kappa,
// also from different host threads: its caches (the FP32 copy, eigenpairs
// and their trace bilinears, 1/xi' values, lexicographic copies, ES data)
// are filled once under fill_mu, and the filling context's stream is
// synchronised before the lock is released, so the other contexts read
// complete data on their own streams.  All users of one space take the
// same number of eigenpairs Q.
struct lqcd_defl {
  std::mutex fill_mu;
  lqcd_op op = LQCD_OP_SCHUR;   // SCHUR: even-site vectors; MG5: full-lattice vectors
  int k = 0;                     // number of deflation vectors
  size_t n = 0;                  // vector length in complex numbers
  int dims[4] = {0, 0, 0, 0};    // lattice the space belongs to
  double kappa = 0;
  lqcd::DevBuf V;                // V_{k+1}, FP64, vectors n apart
  lqcd::DevBuf V32;              // FP32 copy for mixed-precision inner solves
  bool have_v32 = false;
  lqcd::la::Mat H;               // Hbar_k, (k+1) x k
  std::vector<lqcd::cdouble> theta;   // harmonic Ritz values of the final restart
  std::vector<double> theta_resid;    // |A y - theta y| of each
  lqcd::la::QR Hqr;              // QR of Hbar_k for the projection least squares
  // Rayleigh-Ritz eigenpairs (hermitian operator), filled on request.
  int Qe = 0;
  std::vector<double> lam, lam_resid;
  lqcd::DevBuf E;                // Q eigenvectors (FP64, n apart)
  // Caches that depend only on the eigenpairs (reset when they change):
  // per-mode trace bilinears sum_{x in t} e_q^+ Theta g5 e_q, [q][theta][t],
  // and 1/xi'_q per polynomial (coefficients -> values).
  std::vector<lqcd::cdouble> bil;
  std::vector<std::pair<std::vector<lqcd::cdouble>, std::vector<lqcd::cdouble>>> xi_cache;
  // The Q eigenvectors and g5 times them in the lexicographic layout of the
  // C ABI's fields (made on first use: a projection then reads the caller's
  // fields in place); lex_Q = 0 until made.
  int lex_Q = 0;
  lqcd::DevBuf Elex, G5Elex;
  // Eigenvalue subtraction (non-hermitian space, op SCHUR), filled on
  // request: eigenvalues of M, right and left full-lattice eigenvectors
  // (even/odd layout, FP64, full_len apart; L^+ R = 1 per mode) and their
  // per-mode trace bilinears sum_{x in t} l_q^+ Theta r_q, [q][theta][t].
  int Qes = 0;
  std::vector<lqcd::cdouble> es_lam;
  lqcd::DevBuf ER, EL;
  std::vector<lqcd::cdouble> es_bil;
};

namespace lqcd {

// Rayleigh-Ritz eigenpairs of a hermitian deflation space (op MG5): fills
// d->lam, d->lam_resid and d->E with the Q pairs of smallest |lambda|.
void defl_eigpairs(lqcd_ctx *c, lqcd_defl *d, int Q);

}  // namespace lqcd
