// Entry points not implemented yet: they report EINVAL with a message.
#include "common.h"

using namespace lqcd;

#define PENDING(name) \
  return guarded([&] { LQCD_CHECK(false, LQCD_EINVAL, "%s: not implemented yet", name); })

extern "C" {
lqcd_status deflate_project(lqcd_ctx *, lqcd_defl *, int, lqcd_defl_mode, const double *, int,
                            const int *, int, const void *, void *, int, double *, double *) {
  PENDING("deflate_project");
}
lqcd_status pert_subtract(lqcd_ctx *, int, const int *, int, const void *, void *, int, double *) {
  PENDING("pert_subtract");
}
lqcd_status poly_subtract(lqcd_ctx *, int, const void *, double *, double *, const int *, int,
                          const void *, void *, int, double *) {
  PENDING("poly_subtract");
}
lqcd_status loop_estimate(lqcd_ctx *, const int *, int, const void *, const void *, const void *,
                          int, const double *, double *, double *, double *) {
  PENDING("loop_estimate");
}
}
