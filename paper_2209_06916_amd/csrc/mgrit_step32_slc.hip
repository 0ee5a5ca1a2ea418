// Float32 instances of the generic step kernel for semi-Lagrangian coarse steps with the periodic banded solve: the inner solves of
// mixed-precision MGRIT.
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"
#include "mgrit_step.h"

}  // namespace

hipError_t launch_step32_slc(const LevelDesc *desc, const Layout &lay, const PassArgs32 &pa, size_t lds,
                           hipStream_t stream) {
  return launch_kind<OP_SLC, float>(desc, lay, pa, lds, stream);
}

hipError_t configure_step32_slc(size_t bytes) { return set_lds_all<OP_SLC, float>(bytes); }

}  // namespace mgrit
