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

extern "C" lqcd_status lqcd_destroy(lqcd_ctx *c) {
  return guarded([&] {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    delete c;
  });
}
