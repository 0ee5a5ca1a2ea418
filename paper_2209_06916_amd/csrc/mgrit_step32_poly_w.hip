// Float32 instances of the generic step kernel for SDIRK steps (polynomial in W = (I + gamma c L_p)^{-1}): the inner solves of
// mixed-precision MGRIT.
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"
#include "mgrit_step.h"

}  // namespace

hipError_t launch_step32_poly_w(const LevelDesc *desc, const Layout &lay, const PassArgs32 &pa, size_t lds,
                           hipStream_t stream) {
  return launch_kind<OP_POLY_W, float>(desc, lay, pa, lds, stream);
}

hipError_t configure_step32_poly_w(size_t bytes) { return set_lds_all<OP_POLY_W, float>(bytes); }

}  // namespace mgrit
