// Instances of the generic step kernel for explicit Runge-Kutta steps (Horner form in z = -c L_p).
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"
#include "mgrit_step.h"

}  // namespace

hipError_t launch_step_poly_z(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, size_t lds,
                         hipStream_t stream) {
  return launch_kind<OP_POLY_Z, double>(desc, lay, pa, lds, stream);
}

hipError_t configure_step_poly_z(size_t bytes) { return set_lds_all<OP_POLY_Z, double>(bytes); }

}  // namespace mgrit
