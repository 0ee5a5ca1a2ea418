// Float32 instances of the generic step kernel for explicit Runge-Kutta steps (polynomial in Z = -c L_p): the inner solves of
// mixed-precision MGRIT.
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"
#include "mgrit_step.h"

}  // namespace

hipError_t launch_step32_poly_z(const LevelDesc *desc, const Layout &lay, const PassArgs32 &pa, size_t lds,
                           hipStream_t stream) {
  return launch_kind<OP_POLY_Z, float>(desc, lay, pa, lds, stream);
}

hipError_t configure_step32_poly_z(size_t bytes) { return set_lds_all<OP_POLY_Z, float>(bytes); }

}  // namespace mgrit
