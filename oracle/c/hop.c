/* Wilson hopping matrix P of Sec. 5.1 Eqs. (24)-(25), written out site by
 * site in plain C (oracle; test and workload infrastructure only).
 *
 *   (P psi)(x) = sum_mu [ (1 - g_mu) U_mu(x) psi(x + mu)
 *                       + (1 + g_mu) U_mu(x - mu)^dagger psi(x - mu) ]
 *
 * Fields are complex128 arrays [t][z][y][x][spin 4][colour 3] (interleaved
 * re, im), links [t][z][y][x][mu 4][3][3]; periodic boundaries.  The spin
 * factors (1 -+ g_mu) come in as dense 4x4 complex matrices pm[mu] (for
 * 1 - g_mu) and pp[mu] (for 1 + g_mu), so no gamma convention lives here.
 * Used where the numpy form is too slow (the eigenvalue search on the
 * largest lattice); pinned to the numpy form by the tests.  Sites are
 * split over OpenMP threads. */
#include <complex.h>
#include <stddef.h>

typedef double _Complex cplx;

/* parity < 0: every site; parity 0 / 1: only output sites with
 * (x + y + z + t) % 2 == parity are computed, the others are set to zero
 * (one block of the even/odd decomposition). */
void oracle_hop_parity(const int dims[4], const cplx *U, const cplx *pm, const cplx *pp,
                       const cplx *psi, cplx *out, int parity, int nthreads) {
  const int Lx = dims[0], Ly = dims[1], Lz = dims[2], Lt = dims[3];
  const long V = (long)Lx * Ly * Lz * Lt;
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (long s = 0; s < V; ++s) {
    int c[4] = {(int)(s % Lx), (int)((s / Lx) % Ly), (int)((s / ((long)Lx * Ly)) % Lz),
                (int)(s / ((long)Lx * Ly * Lz))};
    const int L[4] = {Lx, Ly, Lz, Lt};
    cplx acc[4][3] = {{0}};
    if (parity >= 0 && ((c[0] + c[1] + c[2] + c[3]) & 1) != parity) {
      for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) out[(s * 4 + sp) * 3 + a] = 0;
      continue;
    }
    for (int mu = 0; mu < 4; ++mu) {
      int f[4] = {c[0], c[1], c[2], c[3]}, b[4] = {c[0], c[1], c[2], c[3]};
      f[mu] = (c[mu] + 1) % L[mu];
      b[mu] = (c[mu] + L[mu] - 1) % L[mu];
      const long sf = f[0] + (long)Lx * (f[1] + (long)Ly * (f[2] + (long)Lz * f[3]));
      const long sb = b[0] + (long)Lx * (b[1] + (long)Ly * (b[2] + (long)Lz * b[3]));
      const cplx *Uf = U + (s * 4 + mu) * 9;   /* U_mu(x) */
      const cplx *Ub = U + (sb * 4 + mu) * 9;  /* U_mu(x - mu) */
      /* colour products: w_f[sp] = U_mu(x) psi_sp(x + mu), w_b[sp] = U_mu(x - mu)^+ psi_sp(x - mu) */
      cplx wf[4][3], wb[4][3];
      for (int sp = 0; sp < 4; ++sp)
        for (int a = 0; a < 3; ++a) {
          cplx vf = 0, vb = 0;
          for (int k = 0; k < 3; ++k) {
            vf += Uf[a * 3 + k] * psi[(sf * 4 + sp) * 3 + k];
            vb += conj(Ub[k * 3 + a]) * psi[(sb * 4 + sp) * 3 + k];
          }
          wf[sp][a] = vf;
          wb[sp][a] = vb;
        }
      for (int sp = 0; sp < 4; ++sp)
        for (int tq = 0; tq < 4; ++tq) {
          const cplx m = pm[(mu * 4 + sp) * 4 + tq], p = pp[(mu * 4 + sp) * 4 + tq];
          for (int a = 0; a < 3; ++a) acc[sp][a] += m * wf[tq][a] + p * wb[tq][a];
        }
    }
    for (int sp = 0; sp < 4; ++sp)
      for (int a = 0; a < 3; ++a) out[(s * 4 + sp) * 3 + a] = acc[sp][a];
  }
}

void oracle_hop(const int dims[4], const cplx *U, const cplx *pm, const cplx *pp,
                const cplx *psi, cplx *out, int nthreads) {
  oracle_hop_parity(dims, U, pm, pp, psi, out, -1, nthreads);
}
