// adjoint.hip -- placeholder until the discrete adjoint is built.
#include "runtime.h"

namespace imb {
void free_adjoint(imb_sim*) {}
}  // namespace imb

extern "C" int imb_adjoint(imb_sim* s, int32_t, int32_t, const double*, const double*,
                           const double*, double*, double*, double*, double*, double*, double*,
                           double*) {
  (void)s;
  return IMB_EUNSUPPORTED;
}
