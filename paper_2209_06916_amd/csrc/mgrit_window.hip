// Float64 instances of the windowed step kernel (truncated-carry periodic
// recurrences): SDIRK fine steps and corrected semi-Lagrangian coarse steps
// whose factor recurrences decay within a few chunks.
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"
#include "mgrit_step.h"
#include "mgrit_window.h"

}  // namespace

#define MGRIT_WIN_T double
#define MGRIT_WIN_ARGS PassArgs
#define MGRIT_WIN_LAUNCH launch_window
#define MGRIT_WIN_CONFIGURE configure_window_kernels64
#include "mgrit_window_inst.h"

}  // namespace mgrit
