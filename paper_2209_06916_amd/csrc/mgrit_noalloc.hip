// mgrit_solve_noalloc: the float64 MGRIT solve of mgrit_solve for callers
// that cannot allocate, with its workspace in a file-scope device array.
#include <map>
#include <mutex>

#include "mgrit.h"
#include "mgrit_internal.h"

namespace mgrit {
mgrit_status noalloc_solve(const mgrit_problem *P, const mgrit_options *O, void *stream, void *ws,
                           uint64_t ws_bytes, const double *u0, const double *v_init, double *u_out,
                           double *u_final, mgrit_stats *stats);
}  // namespace mgrit

namespace {

// The workspace of every allocation-free solve on a device: each GPU the
// library runs on holds its own copy for the life of the process.  In host
// code this name is only a handle for hipGetSymbolAddress; kernels receive
// the device address that call returns.
__device__ __align__(256) char scratch[MGRIT_NOALLOC_BYTES];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> address of its scratch array

}  // namespace

extern "C" mgrit_status mgrit_solve_noalloc(const mgrit_problem *problem, const mgrit_options *options,
                                            void *hip_stream, const double *u0_dev, const double *v_init_dev,
                                            double *u_out_dev, double *u_final_dev, mgrit_stats *stats) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MGRIT_EDEVICE;
  void *ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
      // once per device, with the device current
      if (hipGetSymbolAddress(&ws, HIP_SYMBOL(scratch)) != hipSuccess || !ws) return MGRIT_EDEVICE;
      g_scratch_ptr[dev] = ws;
    } else {
      ws = it->second;
    }
  }
  return mgrit::noalloc_solve(problem, options, hip_stream, ws, MGRIT_NOALLOC_BYTES, u0_dev, v_init_dev, u_out_dev,
                              u_final_dev, stats);
}
