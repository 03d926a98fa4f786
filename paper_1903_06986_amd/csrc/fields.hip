// Field-level kernels: Z(4) noise, lexicographic <-> even/odd packing,
// fills and precision conversion.
#include "common.h"
#include "cplx.h"
#include "fields.h"

namespace lqcd {

namespace {

// Z(4) noise of Sec. 2 from the SplitMix64 counter generator (Steele, Lea,
// Flood, OOPSLA 2014; the increment and finaliser constants of Vigna's
// public-domain splitmix64.c): the c-th output of the stream seeded with
// `seed` finalises seed + (c + 1) * 0x9E3779B97F4A7C15 (mod 2^64).
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_noise(uint64_t seed, int64_t first, uint64_t nvec, uint64_t total,
                        cx<double> *__restrict__ eta, uint8_t *__restrict__ codes) {
  uint64_t gi = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gi >= total) return;
  uint64_t n = uint64_t(first) + gi / nvec;
  uint64_t i = gi % nvec;
  unsigned k = unsigned(splitmix64_at(seed, n * nvec + i) >> 62);
  // i^k: 1, i, -1, -i
  double re = (k == 0) ? 1.0 : (k == 2 ? -1.0 : 0.0);
  double im = (k == 1) ? 1.0 : (k == 3 ? -1.0 : 0.0);
  if (eta) stc(eta + gi, mk(re, im));
  if (codes) codes[gi] = uint8_t(k);
}

// lex [rhs][V][12] complex128  ->  eo [rhs](stride)[2][12][Vh] of R
template <class R>
__global__ void k_pack(Geom g, const cx<double> *__restrict__ lex, cx<R> *__restrict__ eo,
                       size_t eo_stride) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const size_t rhs = blockIdx.y;
  const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
  const int x = s % Lx, y = (s / Lx) % Ly, z = (s / (Lx * Ly)) % Lz, t = s / (Lx * Ly * Lz);
  const int p = (x + y + z + t) & 1;
  const size_t Vh = g.Vh;
  const cx<double> *src = lex + (rhs * g.V + s) * 12;
  cx<R> *dst = eo + rhs * eo_stride + p * 12 * Vh + (s >> 1);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    cx<double> v = ldc(src + c);
    stc(dst + c * Vh, mk<R>(R(v.re), R(v.im)));
  }
}

template <class R>
__global__ void k_unpack(Geom g, const cx<R> *__restrict__ eo, cx<double> *__restrict__ lex,
                         size_t eo_stride) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const size_t rhs = blockIdx.y;
  const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2];
  const int x = s % Lx, y = (s / Lx) % Ly, z = (s / (Lx * Ly)) % Lz, t = s / (Lx * Ly * Lz);
  const int p = (x + y + z + t) & 1;
  const size_t Vh = g.Vh;
  const cx<R> *src = eo + rhs * eo_stride + p * 12 * Vh + (s >> 1);
  cx<double> *dst = lex + (rhs * g.V + s) * 12;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    cx<R> v = ldc(src + c * Vh);
    stc(dst + c, mk<double>(double(v.re), double(v.im)));
  }
}

__global__ void k_fill_zero(uint4 *__restrict__ p, size_t n16) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

template <class RI, class RO>
__global__ void k_convert(const cx<RI> *__restrict__ in, cx<RO> *__restrict__ out, size_t n) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) {
    cx<RI> v = ldc(in + i);
    stc(out + i, mk<RO>(RO(v.re), RO(v.im)));
  }
}

// g5 = diag(1, 1, -1, -1) on LEX complex128 fields [site][spin][colour]:
// element i has spin (i % 12) / 3.  In place allowed.
__global__ void k_g5_lex(const cx<double> *in, cx<double> *out, size_t n) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < n; i += stride) {
    const cx<double> v = ldc(in + i);
    stc(out + i, (i % 12) >= 6 ? -v : v);
  }
}

}  // namespace

void fill_noise(lqcd_ctx *c, uint64_t seed, int64_t first, int nrhs, void *eta, uint8_t *codes) {
  const uint64_t nvec = full_len(c->g);
  const uint64_t total = nvec * uint64_t(nrhs);
  if (total == 0) return;
  hipLaunchKernelGGL(k_noise, dim3(nblocks(total)), dim3(kBlock), 0, c->stream, seed, first, nvec,
                     total, static_cast<cx<double> *>(eta), codes);
  LQCD_HIP(hipGetLastError());
}

template <class R>
void pack_eo(lqcd_ctx *c, const void *lex, void *eo, int nrhs, size_t eo_stride) {
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(k_pack<R>, dim3(nblocks(c->g.V), nrhs), dim3(kBlock), 0, c->stream, c->g,
                     static_cast<const cx<double> *>(lex), static_cast<cx<R> *>(eo), eo_stride);
  LQCD_HIP(hipGetLastError());
}

template <class R>
void unpack_eo(lqcd_ctx *c, const void *eo, void *lex, int nrhs, size_t eo_stride) {
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(k_unpack<R>, dim3(nblocks(c->g.V), nrhs), dim3(kBlock), 0, c->stream, c->g,
                     static_cast<const cx<R> *>(eo), static_cast<cx<double> *>(lex), eo_stride);
  LQCD_HIP(hipGetLastError());
}

void fill_zero(lqcd_ctx *c, void *p, size_t bytes) {
  if (bytes == 0) return;
  LQCD_CHECK(bytes % 16 == 0 && (reinterpret_cast<uintptr_t>(p) % 16) == 0, LQCD_EINVAL,
             "fill_zero: misaligned buffer");
  size_t n16 = bytes / 16;
  unsigned nb = unsigned(std::min<size_t>(nblocks(n16), 4096));
  hipLaunchKernelGGL(k_fill_zero, dim3(nb), dim3(kBlock), 0, c->stream, static_cast<uint4 *>(p), n16);
  LQCD_HIP(hipGetLastError());
}

template <class RI, class RO>
void convert(lqcd_ctx *c, const void *in, void *out, size_t n) {
  if (n == 0) return;
  unsigned nb = unsigned(std::min<size_t>(nblocks(n), 8192));
  hipLaunchKernelGGL((k_convert<RI, RO>), dim3(nb), dim3(kBlock), 0, c->stream,
                     static_cast<const cx<RI> *>(in), static_cast<cx<RO> *>(out), n);
  LQCD_HIP(hipGetLastError());
}

template void pack_eo<double>(lqcd_ctx *, const void *, void *, int, size_t);
template void pack_eo<float>(lqcd_ctx *, const void *, void *, int, size_t);
template void unpack_eo<double>(lqcd_ctx *, const void *, void *, int, size_t);
template void unpack_eo<float>(lqcd_ctx *, const void *, void *, int, size_t);
template void convert<double, float>(lqcd_ctx *, const void *, void *, size_t);
template void convert<float, double>(lqcd_ctx *, const void *, void *, size_t);
template void convert<double, double>(lqcd_ctx *, const void *, void *, size_t);
template void convert<float, float>(lqcd_ctx *, const void *, void *, size_t);

}  // namespace lqcd

using namespace lqcd;

extern "C" lqcd_status lqcd_noise_z4(lqcd_ctx *c, uint64_t seed, int64_t first, int nrhs,
                                     void *eta, uint8_t *codes) {
  return guarded([&] {
    LQCD_CHECK(c, LQCD_EINVAL, "lqcd_noise_z4: null context");
    LQCD_CHECK(nrhs >= 0 && first >= 0, LQCD_EINVAL, "lqcd_noise_z4: negative count or index");
    LQCD_CHECK(eta || codes || nrhs == 0, LQCD_EINVAL, "lqcd_noise_z4: no output");
    fill_noise(c, seed, first, nrhs, eta, codes);
  });
}

extern "C" lqcd_status lqcd_pack_eo(lqcd_ctx *c, lqcd_prec prec, const void *lex, void *eo,
                                    int nrhs) {
  return guarded([&] {
    LQCD_CHECK(c && lex && eo, LQCD_EINVAL, "lqcd_pack_eo: null argument");
    const size_t fl = full_len(c->g);
    if (prec == LQCD_F64) pack_eo<double>(c, lex, eo, nrhs, fl);
    else if (prec == LQCD_F32) pack_eo<float>(c, lex, eo, nrhs, fl);
    else LQCD_CHECK(false, LQCD_EINVAL, "lqcd_pack_eo: precision %d not available", int(prec));
  });
}

extern "C" lqcd_status lqcd_unpack_eo(lqcd_ctx *c, lqcd_prec prec, const void *eo, void *lex,
                                      int nrhs) {
  return guarded([&] {
    LQCD_CHECK(c && lex && eo, LQCD_EINVAL, "lqcd_unpack_eo: null argument");
    const size_t fl = full_len(c->g);
    if (prec == LQCD_F64) unpack_eo<double>(c, eo, lex, nrhs, fl);
    else if (prec == LQCD_F32) unpack_eo<float>(c, eo, lex, nrhs, fl);
    else LQCD_CHECK(false, LQCD_EINVAL, "lqcd_unpack_eo: precision %d not available", int(prec));
  });
}

extern "C" lqcd_status lqcd_gamma5(lqcd_ctx *c, const void *in, void *out, int nrhs) {
  return guarded([&] {
    LQCD_CHECK(c && in && out, LQCD_EINVAL, "lqcd_gamma5: null argument");
    LQCD_CHECK(nrhs >= 0, LQCD_EINVAL, "lqcd_gamma5: nrhs < 0");
    const size_t n = full_len(c->g) * size_t(nrhs);
    if (n == 0) return;
    hipLaunchKernelGGL(k_g5_lex, dim3(std::min<size_t>(nblocks(n), 8192)), dim3(kBlock), 0, c->stream,
                       static_cast<const cx<double> *>(in), static_cast<cx<double> *>(out), n);
    LQCD_HIP(hipGetLastError());
  });
}
