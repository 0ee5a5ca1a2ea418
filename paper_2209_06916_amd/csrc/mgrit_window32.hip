// Float32 instances of the windowed step kernel (the inner solves of mixed
// precision).
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"
#include "mgrit_step.h"
#include "mgrit_window.h"

}  // namespace

#define MGRIT_WIN_T float
#define MGRIT_WIN_ARGS PassArgs32
#define MGRIT_WIN_LAUNCH launch_window32
#define MGRIT_WIN_CONFIGURE configure_window_kernels32
#include "mgrit_window_inst.h"

}  // namespace mgrit
