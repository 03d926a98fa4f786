// Vector kernels used by the solvers and the subtraction code.
//
// A "vector" is n complex numbers of real type R (double or float) stored
// contiguously; batched calls act on nrhs vectors that are `rs` complex
// elements apart.  A "basis" is J vectors ldv elements apart (per rhs).
// All reductions accumulate in FP64 and are deterministic: every block
// writes its partial sums and a second kernel adds them in a fixed order.
#pragma once

#include "common.h"

namespace lqcd {

void fill_zero(lqcd_ctx *c, void *p, size_t bytes);
template <class RI, class RO>
void convert(lqcd_ctx *c, const void *in, void *out, size_t n);

// Strided batch descriptor (complex-element strides).
struct Batch {
  int nrhs;
  size_t rs;  // distance between the vectors of consecutive right-hand sides
};

// out[r * out_rs + j] = sum_i conj(V_r[j][i]) w_r[i], j < J   (device cdouble).
// With a device flag array, right-hand sides whose flag is 0 are skipped
// (their output is set to zero).
template <class R>
void multi_dot(lqcd_ctx *c, const void *V, size_t ldv, size_t V_rs, int J, const void *w,
               size_t w_rs, size_t n, int nrhs, cdouble *out, size_t out_rs,
               const int *flag = nullptr);

// w_r[i] -= sum_j V_r[j][i] coef[r * coef_rs + j]; if norm2_out is not null,
// norm2_out[r] = |w_r|^2 after the update (device doubles).  With a device
// flag array, right-hand sides whose flag is 0 are left untouched.
template <class R>
void multi_axpy(lqcd_ctx *c, const void *V, size_t ldv, size_t V_rs, int J,
                const cdouble *coef, size_t coef_rs, void *w, size_t w_rs, size_t n, int nrhs,
                double *norm2_out, const int *flag = nullptr);

// norm2_out[r] = |x_r|^2
template <class R>
void norm2(lqcd_ctx *c, const void *x, size_t x_rs, size_t n, int nrhs, double *norm2_out);

// y_r = a_r * x_r + b_r * y_r with host complex scalars (arrays of nrhs, or
// a single value broadcast when the pointer's count is 1).
template <class R>
void axpby(lqcd_ctx *c, const cdouble *a, const void *x, size_t x_rs, const cdouble *b, void *y,
           size_t y_rs, size_t n, int nrhs, bool per_rhs);

// y_r = x_r * scale_dev[r]   (device scale; e.g. 1 / |w| for Arnoldi)
template <class R>
void scale_dev(lqcd_ctx *c, const void *x, size_t x_rs, const double *scale, void *y,
               size_t y_rs, size_t n, int nrhs);

// Y_r[b][i] += sum_j V_r[j][i] C_r[j][b]  (C column-major with leading
// dimension ldc, per-rhs stride C_rs; device complex); alpha = +1 or -1.
template <class R>
void gemm_nn(lqcd_ctx *c, const void *V, size_t ldv, size_t V_rs, int J, const cdouble *C,
             size_t ldc, size_t C_rs, void *Y, size_t ldy, size_t Y_rs, int nb, size_t n,
             int nrhs, double alpha);

// C[j + ldc * b] = sum_i conj(V[j][i]) X[b][i] for j < J, b < nb (device).
template <class R>
void gemm_tn(lqcd_ctx *c, const void *V, size_t ldv, int J, const void *X, size_t ldx, int nb,
             size_t n, cdouble *C, size_t ldc);

// In place: V[j] <- sum_l V[l] P[l + ldp * j], j < Jout, over Jin input
// vectors (Jout <= Jin); P device complex.
template <class R>
void recombine(lqcd_ctx *c, void *V, size_t ldv, int Jin, const cdouble *P, size_t ldp, int Jout,
               size_t n);

// 16-bit stored bases (half.h; KIND 0 = FP16, 1 = BF16): V is a basis of
// stored vectors ldv words apart (V_rs words between right-hand sides), w/Y
// FP32 vectors of n = 12 Vh elements.  Semantics as the FP32 versions.
// With w16 the vector w is itself a stored 16-bit vector (w_rs in words).
template <int KIND>
void hmulti_dot(lqcd_ctx *c, const void *V, size_t ldv, size_t V_rs, int J, const void *w,
                size_t w_rs, size_t n, int nrhs, cdouble *out, size_t out_rs, const int *flag,
                bool w16 = false);
template <int KIND>
void hmulti_axpy(lqcd_ctx *c, const void *V, size_t ldv, size_t V_rs, int J, const cdouble *coef,
                 size_t coef_rs, void *w, size_t w_rs, size_t n, int nrhs, double *norm2_out,
                 const int *flag);
// out_r = stored(w_r - V_r coef_r), unnormalised (per-site scales), with
// |stored|^2 in norm2_out; w null: w_r is out_r itself (in place).
template <int KIND>
void hmulti_axpy_q(lqcd_ctx *c, const void *V, size_t ldv, size_t V_rs, int J, const cdouble *coef,
                   size_t coef_rs, const void *w, size_t w_rs, void *out, size_t out_rs, size_t n, int nrhs,
                   double *norm2_out, const int *flag);
// s-step Arnoldi on a 16-bit basis, S = 2 .. 6 vectors, FP32 in the pair
// layout or (W16) 16-bit stored (vector k of right-hand side r at w + r
// w_rs + k w_vs, in complex elements, or in words): out[r][k J + j] = V_j^H w_k (rows out_rs apart), with
// gpart (optional) the per-workgroup partials of the w_k's own Gram matrix,
// gpart[(r nblk + b) S^2 + q] (|w_l|^2 at q = l, Re and Im of w_l^H w_m,
// l < m, from q = S on, pairs in the order (0, 1), (0, 2), .., (1, 2), ..;
// sized by the caller: nrhs x nblk x S^2 doubles, nblk = ceil(n / 12 /
// 256)); hmulti_axpys: w_k -= V c_k in place (coef[r][k J + j]) with
// per-workgroup partials of the Gram matrix of the results in part (same
// layout; returns nblk); hmulti_axpys_store: the right-hand sides whose
// flag is clear store slot m = stored(sum_{l <= m} F[l][m] (w_l - V c_l))
// directly, F = f[r][S][S] complex (w is not written); hsstore: slot m =
// stored(sum_{l <= m} F[l][m] w_l), slot m of right-hand side r at out + r
// out_rs + m out_vs words, for the right-hand sides whose flag is set (all
// without flags).
template <int KIND, int S, bool W16>
void hmulti_dots(lqcd_ctx *c, const void *V, size_t ldv, size_t V_rs, int J, const void *w, size_t w_vs,
                 size_t w_rs, size_t n, int nrhs, cdouble *out, size_t out_rs, const int *flag, double *gpart);
template <int KIND, int S, bool W16>
int hmulti_axpys(lqcd_ctx *c, const void *V, size_t ldv, size_t V_rs, int J, const cdouble *coef,
                 size_t coef_rs, void *w, size_t w_vs, size_t w_rs, size_t n, int nrhs, double *part,
                 const int *flag);
template <int KIND, int S, bool W16>
void hmulti_axpys_store(lqcd_ctx *c, const void *V, size_t ldv, size_t V_rs, int J, const cdouble *coef,
                        size_t coef_rs, const void *w, size_t w_vs, size_t w_rs, size_t n, int nrhs, const int *flag,
                        const cdouble *f, void *out, size_t out_vs, size_t out_rs);
template <int KIND, int S, bool W16>
void hsstore(lqcd_ctx *c, const void *w, size_t w_vs, size_t w_rs, const cdouble *f, void *out, size_t out_vs,
             size_t out_rs, size_t n, int nrhs, const int *flag);
// Index of the Gram entry w_l^H w_m (l <= m) in those partials.
__host__ __device__ constexpr int gram_pair_idx(int S, int l, int m) {
  return l == m ? l : S + 2 * (l * (2 * S - l - 1) / 2 + (m - l - 1));
}
// Per-site scales of nrhs stored vectors (x_rs words apart) times f[r]
// (device array).
void hscale_dev(lqcd_ctx *c, void *x, size_t x_rs, size_t n, int nrhs, const double *f);
template <int KIND>
void hgemm_nn(lqcd_ctx *c, const void *V, size_t ldv, size_t V_rs, int J, const cdouble *C,
              size_t ldc, size_t C_rs, void *Y, size_t ldy, size_t Y_rs, int nb, size_t n, int nrhs,
              double alpha);
// out_r = stored(scale_dev[r] * w_r) with per-site scales (scale_dev may
// be null: factor 1); and the decode.
template <int KIND>
void hquantize(lqcd_ctx *c, const void *w, size_t w_rs, const double *scale_dev, void *out,
               size_t out_rs, size_t n, int nrhs);
template <int KIND>
void hdequantize(lqcd_ctx *c, const void *x, size_t x_rs, void *y, size_t y_rs, size_t n, int nrhs);
// inv[r] = 1 / sqrt(nrm2[r]) (0 for 0 or non-finite), device arrays.
void inv_sqrt_dev(lqcd_ctx *c, const double *nrm2, double *inv, int nb);

}  // namespace lqcd
