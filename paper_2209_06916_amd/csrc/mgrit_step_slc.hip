// Instances of the generic step kernel for semi-Lagrangian coarse steps with the periodic banded solve.
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"
#include "mgrit_step.h"

}  // namespace

hipError_t launch_step_slc(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, size_t lds,
                         hipStream_t stream) {
  return launch_kind<OP_SLC, double>(desc, lay, pa, lds, stream);
}

hipError_t configure_step_slc(size_t bytes) { return set_lds_all<OP_SLC, double>(bytes); }

}  // namespace mgrit
