// Internal declarations of the gfx950 library (not part of the C ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/lqcd.h"

namespace lqcd {

using cdouble = std::complex<double>;

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);

struct Error {
  lqcd_status code;
};

#define LQCD_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t _e = (call);                                                            \
    if (_e != hipSuccess) {                                                            \
      ::lqcd::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call, hipGetErrorString(_e)); \
      throw ::lqcd::Error{LQCD_EDEVICE};                                               \
    }                                                                                  \
  } while (0)

#define LQCD_CHECK(cond, code, ...)    \
  do {                                 \
    if (!(cond)) {                     \
      ::lqcd::set_error(__VA_ARGS__);  \
      throw ::lqcd::Error{code};       \
    }                                  \
  } while (0)

// Runs f(), converting exceptions to a status (nothing crosses the ABI).
template <class F>
lqcd_status guarded(F &&f) {
  try {
    f();
    return LQCD_OK;
  } catch (const Error &e) {
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return LQCD_ENOMEM;
  } catch (...) {
    set_error("unexpected C++ exception");
    return LQCD_EDEVICE;
  }
}

// -------------------------------------------------------- device buffers
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  // Grow (never shrink) to at least `need` bytes; contents are not kept.
  void *ensure(size_t need) {
    if (need <= bytes) return ptr;
    release();
    hipError_t e = hipMalloc(&ptr, need);
    if (e != hipSuccess) {
      ptr = nullptr;
      set_error("hipMalloc(%zu bytes) failed: %s", need, hipGetErrorString(e));
      throw Error{LQCD_ENOMEM};
    }
    bytes = need;
    return ptr;
  }
  template <class T>
  T *as() const { return static_cast<T *>(ptr); }
};

// ------------------------------------------------------------ geometry
struct Geom {
  int L[4];   // Lx, Ly, Lz, Lt
  int V, Vh;  // volume, half volume
  int Lxh;    // Lx / 2
};

// Precomputed table of Tr_t(Theta P^j) for j <= kMaxOrder (closed walks).
constexpr int kMaxOrder = 7;
constexpr int kNumTheta = 5;

// Optional per-kernel-class timing with HIP events on the context stream
// (classes as in lqcd.h: LQCD_KC_*).  Each timed launch records a start
// and a stop event; pairs are harvested when the pool fills and on read.
struct KTimer {
  bool on = false;
  std::vector<hipEvent_t> ev;      // 2 per slot
  std::vector<int> cls;
  std::vector<double> bytes;
  int used = 0;
  double ms[LQCD_KC_COUNT] = {};
  double by[LQCD_KC_COUNT] = {};
  long long cnt[LQCD_KC_COUNT] = {};
};

}  // namespace lqcd

// The opaque context of the C ABI.
struct lqcd_ctx {
  lqcd::Geom g;
  double kappa;
  hipStream_t stream;
  int device;
  // Links in the even/odd layout [parity][mu][9][Vh] of complex numbers
  // (row-major 3x3), FP64 and FP32.
  lqcd::DevBuf U64, U32;
  // Exact per-timeslice traces Tr_t(Theta P^j), j = 0..kMaxOrder,
  // Theta = 1, g1..g4: host [j][theta][Lt], filled on first use.
  bool have_walk_traces = false;  // orders from walks of length <= 6
  bool have_walk_len8 = false;    // point-split order 7 (walks of length 8)
  std::vector<lqcd::cdouble> walk_traces;
  // Scratch buffers reused across calls (grown on demand).
  lqcd::DevBuf ws[8];
  lqcd::DevBuf red;      // reduction partials
  lqcd::DevBuf red_out;  // reduction results (device)
  lqcd::DevBuf sw[16];   // solver fields
  lqcd::DevBuf small[2]; // solver small matrices
  lqcd::DevBuf sstep;    // two-step Arnoldi: coefficients, Gram partials and factors
  lqcd::DevBuf grad[3];  // loop_gradient: right-hand sides, solutions, adjoint source matrices
  lqcd::KTimer timer;
  int hop_nb[2] = {2, 1};  // largest lane-grouped right-hand-side count: FP64, FP32
  int hop_tile[2] = {1, 1};  // link-tiled stencil for many right-hand sides: FP64, FP32
  int hop_order = 0;         // lane-grouped stencil block order: 0 rhs-group fastest, 1 site fastest
  int hop_tblock[2] = {-1, -1};  // tiled stencil: timeslices per plane block (0: flat order, -1: auto), FP64, FP32
  int hop_tsites[2] = {32, 32};  // tiled stencil: sites per tile, FP64 (16, 32), FP32 (16, 32, 64)
  int hop_rgroup = 0;            // tiled stencil: right-hand sides per group (0: all in one)
  int hop_rnest = -1;            // tiled stencil: groups swept in turn within each block (0: off, -1: auto)
  int gemm_mfma = 1;             // V C with one shared basis on the matrix cores (0: FMA kernel)
  int cycle_reorth = 0;          // 1: second Gram-Schmidt pass on every GMRES-Proj step
  int kept_period = 16;          // MINRES-DR: steps between tests against the kept vectors
  int arnoldi_steps = 4;         // 16-bit GMRES-Proj cycles: Arnoldi steps per basis pass (1..6)
  int sstep_z16 = 0;             // s-step power vectors stored in 16-bit form (0: FP32)
  int recombine_regs = 1;        // restart recombination with its outputs in registers (0: LDS-tiled form)
  ~lqcd_ctx();
};

namespace lqcd {

// ------------------------------------------------------------- launches
constexpr int kBlock = 256;
inline unsigned nblocks(size_t n, int block = kBlock) {
  return static_cast<unsigned>((n + block - 1) / block);
}

// ---------------------------------------------------- field-level helpers
// Element counts: a half field (one parity) holds 12 * Vh complex numbers,
// a full field 24 * Vh = 12 V.
inline size_t half_len(const Geom &g) { return size_t(12) * g.Vh; }
inline size_t full_len(const Geom &g) { return size_t(12) * g.V; }

// dslash.hip ------------------------------------------------------------
// Generic stencil on even/odd fields of real type R (double or float):
//   out_p = G_out( alpha * G_in(self_p) + beta * D_{p,1-p} G_in(in_{1-p}) )
// for output parity p (out, self, in are half fields of Vh sites, in of the
// opposite parity), over nrhs right-hand sides with the given strides
// (in complex elements).  G = g5 when the flag is set.  self may be null.
template <class R>
void hop_half(lqcd_ctx *c, int out_parity, const void *in, const void *self, void *out,
              cdouble alpha, double beta, bool g5_in, bool g5_out, int nrhs,
              size_t in_stride, size_t self_stride, size_t out_stride);

// Operators on internal fields (precision R).  Full fields are [2][12][Vh]
// per rhs (even block first); Schur fields are [12][Vh] (even sites).
template <class R>
void apply_full(lqcd_ctx *c, lqcd_op op, const void *in, void *out, int nrhs,
                size_t stride_in, size_t stride_out);
template <class R>
void apply_schur(lqcd_ctx *c, const void *in, void *out, void *tmp_odd, int nrhs,
                 size_t stride_in, size_t stride_out, size_t stride_tmp);

// Mhat on 16-bit stored even fields (half.h kind KIND; in: words, vectors
// sin words apart); FP32 output and odd temporary.
template <int KIND>
void apply_schur_h(lqcd_ctx *c, const void *in, void *out, void *tmp_odd, int nrhs, size_t sin,
                   size_t sout, size_t stmp);
// Mhat - 1 = -kappa^2 D_eo D_oe with the FP32 output in the pair layout
// (16-byte granules of two components, as the odd temporary: component c
// of site i at complex element 2 ((c / 2) Vh + i) + c % 2), on a 16-bit
// stored input (kind KIND) or on an FP32 input in that layout.
template <int KIND>
void apply_dd_h_pair(lqcd_ctx *c, const void *in, void *out, void *tmp_odd, int nrhs, size_t sin, size_t sout,
                     size_t stmp);
void apply_dd_pair(lqcd_ctx *c, const void *in, void *out, void *tmp_odd, int nrhs, size_t sin, size_t sout,
                   size_t stmp);
// Mhat - 1 from a 16-bit stored input to a 16-bit stored output (the
// per-site scaled form of half.h, kind KIND; strides in words).
template <int KIND>
void apply_dd_hh(lqcd_ctx *c, const void *in, void *out, void *tmp_odd, int nrhs, size_t sin, size_t sout,
                 size_t stmp);

// context.cpp: event timing of one launch (no-op unless the timer is on).
// The events ride on the kernel dispatch itself (hipExtLaunchKernelGGL),
// so the elapsed time is the kernel's own start-to-end time; launches go
// through LQCD_TLAUNCH.  A slot whose scope launched nothing is dropped.
int timer_start(lqcd_ctx *c, int cls, double bytes);
void timer_stop(lqcd_ctx *c, int slot, bool used);
hipEvent_t timer_event(lqcd_ctx *c, int slot, int which);
struct Timed {
  lqcd_ctx *c;
  int slot;
  bool used = false;
  Timed(lqcd_ctx *cc, int cls, double bytes) : c(cc), slot(timer_start(cc, cls, bytes)) {}
  ~Timed() { timer_stop(c, slot, used); }
  hipEvent_t ev(int which) const { return timer_event(c, slot, which); }
};

// Launch under a Timed scope: `first` attaches the start event, `last` the
// stop event (a scope with several launches spans first to last).
#define LQCD_TLAUNCH(tm, first, last, kern, grid, block, shm, stream, ...)                        \
  do {                                                                                           \
    if ((tm).slot >= 0) {                                                                        \
      (tm).used = true;                                                                          \
      hipExtLaunchKernelGGL(kern, grid, block, shm, stream, (first) ? (tm).ev(0) : nullptr,      \
                            (last) ? (tm).ev(1) : nullptr, 0, __VA_ARGS__);                      \
    } else {                                                                                     \
      hipLaunchKernelGGL(kern, grid, block, shm, stream, __VA_ARGS__);                           \
    }                                                                                            \
  } while (0)

// fields.hip -----------------------------------------------------------
template <class R>
void pack_eo(lqcd_ctx *c, const void *lex, void *eo, int nrhs, size_t eo_stride);
template <class R>
void unpack_eo(lqcd_ctx *c, const void *eo, void *lex, int nrhs, size_t eo_stride);
void fill_noise(lqcd_ctx *c, uint64_t seed, int64_t first, int nrhs, void *eta, uint8_t *codes);

}  // namespace lqcd
