// Context creation, link import (even/odd layout) and error reporting.
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace lqcd {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

}  // namespace lqcd

using namespace lqcd;

extern "C" const char *lqcd_last_error(void) { return g_err; }

// Links arrive lexicographic [s][mu][3][3]; the device keeps, for each
// parity p, direction mu and matrix entry e, the Vh sites of that parity in
// checkerboard order (cb = s >> 1): U[((p * 4 + mu) * 9 + e) * Vh + cb].
// This puts the same entry of consecutive sites next to each other so that
// the stencil's per-thread loads coalesce.
extern "C" lqcd_status lqcd_create(const int dims[4], const double *links_host, double kappa,
                                   void *hip_stream, lqcd_ctx **out) {
  return guarded([&] {
    LQCD_CHECK(dims && links_host && out, LQCD_EINVAL, "lqcd_create: null argument");
    *out = nullptr;
    for (int i = 0; i < 4; ++i)
      LQCD_CHECK(dims[i] >= 2 && dims[i] % 2 == 0, LQCD_EINVAL,
                 "lqcd_create: extent %d = %d must be even and >= 2", i, dims[i]);
    long long V = 1;
    for (int i = 0; i < 4; ++i) V *= dims[i];
    LQCD_CHECK(V < (1LL << 30), LQCD_EINVAL, "lqcd_create: volume too large");
    auto *c = new lqcd_ctx();
    try {
      for (int i = 0; i < 4; ++i) c->g.L[i] = dims[i];
      c->g.V = int(V);
      c->g.Vh = int(V / 2);
      c->g.Lxh = dims[0] / 2;
      c->kappa = kappa;
      c->stream = static_cast<hipStream_t>(hip_stream);
      LQCD_HIP(hipGetDevice(&c->device));
      const int Vh = c->g.Vh;
      const int Lx = dims[0], Ly = dims[1], Lz = dims[2];
      std::vector<double> h64(size_t(2) * 4 * 9 * Vh * 2);
      std::vector<float> h32(h64.size());
      for (long long s = 0; s < V; ++s) {
        int x = int(s % Lx), y = int((s / Lx) % Ly), z = int((s / (Lx * Ly)) % Lz),
            t = int(s / (Lx * Ly * Lz));
        int p = (x + y + z + t) & 1;
        int cb = int(s >> 1);
        for (int mu = 0; mu < 4; ++mu)
          for (int e = 0; e < 9; ++e) {
            size_t dst = ((size_t(p) * 4 + mu) * 9 + e) * Vh + cb;
            size_t src = (size_t(s) * 4 + mu) * 9 + e;
            h64[2 * dst] = links_host[2 * src];
            h64[2 * dst + 1] = links_host[2 * src + 1];
            h32[2 * dst] = float(links_host[2 * src]);
            h32[2 * dst + 1] = float(links_host[2 * src + 1]);
          }
      }
      c->U64.ensure(h64.size() * sizeof(double));
      c->U32.ensure(h32.size() * sizeof(float));
      LQCD_HIP(hipMemcpy(c->U64.ptr, h64.data(), h64.size() * sizeof(double), hipMemcpyHostToDevice));
      LQCD_HIP(hipMemcpy(c->U32.ptr, h32.data(), h32.size() * sizeof(float), hipMemcpyHostToDevice));
    } catch (...) {
      delete c;
      throw;
    }
    *out = c;
  });
}

extern "C" lqcd_status lqcd_set_kappa(lqcd_ctx *c, double kappa) {
  return guarded([&] {
    LQCD_CHECK(c, LQCD_EINVAL, "lqcd_set_kappa: null context");
    c->kappa = kappa;
  });
}

extern "C" lqcd_status lqcd_set_stream(lqcd_ctx *c, void *hip_stream) {
  return guarded([&] {
    LQCD_CHECK(c, LQCD_EINVAL, "lqcd_set_stream: null context");
    c->stream = static_cast<hipStream_t>(hip_stream);
  });
}

namespace lqcd {

namespace {
constexpr int kTimerSlots = 4096;

void harvest(lqcd_ctx *c) {
  KTimer &T = c->timer;
  if (T.used == 0) return;
  LQCD_HIP(hipStreamSynchronize(c->stream));
  for (int i = 0; i < T.used; ++i) {
    if (T.cls[i] < 0) continue;  // scope launched nothing
    float ms = 0;
    LQCD_HIP(hipEventElapsedTime(&ms, T.ev[2 * i], T.ev[2 * i + 1]));
    T.ms[T.cls[i]] += ms;
    T.by[T.cls[i]] += T.bytes[i];
    T.cnt[T.cls[i]] += 1;
  }
  T.used = 0;
}
}  // namespace

int timer_start(lqcd_ctx *c, int cls, double bytes) {
  KTimer &T = c->timer;
  if (!T.on) return -1;
  if (T.ev.empty()) {
    T.ev.resize(2 * kTimerSlots);
    for (auto &e : T.ev) LQCD_HIP(hipEventCreate(&e));
    T.cls.resize(kTimerSlots);
    T.bytes.resize(kTimerSlots);
  }
  if (T.used == kTimerSlots) harvest(c);
  int s = T.used++;
  T.cls[s] = cls;
  T.bytes[s] = bytes;
  return s;
}

void timer_stop(lqcd_ctx *c, int slot, bool used) {
  if (slot >= 0 && !used) c->timer.cls[slot] = -1;
}

hipEvent_t timer_event(lqcd_ctx *c, int slot, int which) { return c->timer.ev[2 * slot + which]; }

}  // namespace lqcd

lqcd_ctx::~lqcd_ctx() {
  for (auto &e : timer.ev) (void)hipEventDestroy(e);
}

extern "C" lqcd_status lqcd_timer_enable(lqcd_ctx *c, int on) {
  return guarded([&] {
    LQCD_CHECK(c, LQCD_EINVAL, "lqcd_timer_enable: null context");
    LQCD_HIP(hipStreamSynchronize(c->stream));
    c->timer.used = 0;
    for (int k = 0; k < LQCD_KC_COUNT; ++k) {
      c->timer.ms[k] = 0;
      c->timer.by[k] = 0;
      c->timer.cnt[k] = 0;
    }
    c->timer.on = on != 0;
  });
}

extern "C" lqcd_status lqcd_timer_read(lqcd_ctx *c, int k, double *ms, double *bytes,
                                       int64_t *launches) {
  return guarded([&] {
    LQCD_CHECK(c && k >= 0 && k < LQCD_KC_COUNT, LQCD_EINVAL, "lqcd_timer_read: bad argument");
    harvest(c);
    if (ms) *ms = c->timer.ms[k];
    if (bytes) *bytes = c->timer.by[k];
    if (launches) *launches = c->timer.cnt[k];
  });
}

extern "C" lqcd_status lqcd_tune_set(lqcd_ctx *c, lqcd_tune_param param, int value) {
  return guarded([&] {
    LQCD_CHECK(c, LQCD_EINVAL, "lqcd_tune_set: null context");
    switch (param) {
      case LQCD_TUNE_HOP_NB64:
      case LQCD_TUNE_HOP_NB32:
        LQCD_CHECK(value == 1 || value == 2 || value == 4 || value == 8, LQCD_EINVAL,
                   "lqcd_tune_set: right-hand-side group must be 1, 2, 4 or 8");
        c->hop_nb[param == LQCD_TUNE_HOP_NB64 ? 0 : 1] = value;
        break;
      case LQCD_TUNE_HOP_TILE64:
      case LQCD_TUNE_HOP_TILE32:
        LQCD_CHECK(value == 0 || value == 1, LQCD_EINVAL, "lqcd_tune_set: tiled stencil switch must be 0 or 1");
        c->hop_tile[param == LQCD_TUNE_HOP_TILE64 ? 0 : 1] = value;
        break;
      case LQCD_TUNE_HOP_ORDER:
        LQCD_CHECK(value == 0 || value == 1, LQCD_EINVAL, "lqcd_tune_set: block order must be 0 or 1");
        c->hop_order = value;
        break;
      case LQCD_TUNE_HOP_TBLOCK64:
      case LQCD_TUNE_HOP_TBLOCK32:
        LQCD_CHECK(value >= -1 && value <= 1024, LQCD_EINVAL,
                   "lqcd_tune_set: timeslices per plane block must be in -1..1024");
        c->hop_tblock[param == LQCD_TUNE_HOP_TBLOCK64 ? 0 : 1] = value;
        break;
      case LQCD_TUNE_HOP_RGROUP:
        LQCD_CHECK(value >= 0 && value <= 4096, LQCD_EINVAL, "lqcd_tune_set: right-hand sides per group in 0..4096");
        c->hop_rgroup = value;
        break;
      case LQCD_TUNE_HOP_TSITES32:
        LQCD_CHECK(value == 16 || value == 32 || value == 64, LQCD_EINVAL,
                   "lqcd_tune_set: sites per FP32 tile must be 16, 32 or 64");
        c->hop_tsites[1] = value;
        break;
      case LQCD_TUNE_HOP_TSITES64:
        LQCD_CHECK(value == 16 || value == 32, LQCD_EINVAL, "lqcd_tune_set: sites per FP64 tile must be 16 or 32");
        c->hop_tsites[0] = value;
        break;
      case LQCD_TUNE_HOP_RNEST:
        LQCD_CHECK(value >= -1 && value <= 4096, LQCD_EINVAL,
                   "lqcd_tune_set: right-hand sides per nested group in -1..4096");
        c->hop_rnest = value;
        break;
      case LQCD_TUNE_ARNOLDI_STEPS:
        LQCD_CHECK(value >= 1 && value <= 6, LQCD_EINVAL, "lqcd_tune_set: Arnoldi steps per basis pass in 1..6");
        c->arnoldi_steps = value;
        break;
      case LQCD_TUNE_RECOMBINE_REGS:
        LQCD_CHECK(value == 0 || value == 1, LQCD_EINVAL, "lqcd_tune_set: recombination form must be 0 or 1");
        c->recombine_regs = value;
        break;
      case LQCD_TUNE_SSTEP_Z16:
        LQCD_CHECK(value == 0 || value == 1, LQCD_EINVAL, "lqcd_tune_set: 16-bit power vectors switch must be 0 or 1");
        c->sstep_z16 = value;
        break;
      case LQCD_TUNE_KEPT_PERIOD:
        LQCD_CHECK(value >= 1 && value <= 64, LQCD_EINVAL, "lqcd_tune_set: kept-vector test period in 1..64");
        c->kept_period = value;
        break;
      case LQCD_TUNE_CYCLE_REORTH:
        LQCD_CHECK(value == 0 || value == 1, LQCD_EINVAL, "lqcd_tune_set: cycle second-pass switch must be 0 or 1");
        c->cycle_reorth = value;
        break;
      case LQCD_TUNE_GEMM_MFMA:
        LQCD_CHECK(value == 0 || value == 1, LQCD_EINVAL, "lqcd_tune_set: matrix-core switch must be 0 or 1");
        c->gemm_mfma = value;
        break;
      default:
        LQCD_CHECK(false, LQCD_EINVAL, "lqcd_tune_set: unknown parameter %d", int(param));
    }
  });
}

extern "C" lqcd_status lqcd_destroy(lqcd_ctx *c) {
  return guarded([&] {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    delete c;
  });
}
