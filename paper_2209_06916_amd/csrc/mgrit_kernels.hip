// Small kernels (deterministic norm reduction, row gather, fill) and the
// host-side dispatch to the kernel families: the generic step kernel
// (mgrit_step.h), the lean coarse-step kernel (mgrit_lean.hip) and the
// level-0 wavefront tiles (mgrit_tile.h).
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"

constexpr int RED_T = 1024;

// Sum of part[0..n) by one workgroup of RED_T threads, in a fixed order (the
// result does not depend on timing): every thread adds its strided elements
// with four loads in flight, each wavefront folds its lanes with butterfly
// shuffles (every lane ends with the same sum), and thread 0 adds the
// wavefront sums in order.  Only thread 0's return value is the total.
__device__ double block_sum(const double *__restrict__ part, int64_t n, double *red) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 3 * RED_T < n; i += 4 * RED_T) {
    const double a = part[i], b = part[i + RED_T], c = part[i + 2 * RED_T], d = part[i + 3 * RED_T];
    s0 += a;
    s1 += b;
    s2 += c;
    s3 += d;
  }
  for (; i < n; i += RED_T) s0 += part[i];
  double s = (s0 + s1) + (s2 + s3);
  for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    s = red[0];
    for (int w = 1; w < RED_T / WAVE; ++w) s += red[w];
  }
  return s;
}

__global__ void __launch_bounds__(RED_T) reduce_kernel(const double *__restrict__ part, int64_t n,
                                                        double *__restrict__ out) {
  __shared__ double red[RED_T / WAVE];
  const double s = block_sum(part, n, red);
  if (threadIdx.x == 0) out[0] = s;
}

// Residual norm of one MGRIT iteration and the stopping test (Sec. 2.2: stop
// once ||r_it|| <= rtol ||r_0||), in the order the solver applies them:
// non-finite, converged, stalled (inner float32 solves only), iteration
// limit, growth past diverge_factor ||r_0||.
__global__ void __launch_bounds__(RED_T) solve_ctl_kernel(const double *__restrict__ part, int64_t n,
                                                         SolveCtl *ctl, SolveCtl *ctl_host, const GridSync *gs,
                                                         StopRule rule) {
  __shared__ double red[RED_T / WAVE];
  const double ss = block_sum(part, n, red);
  if (threadIdx.x != 0) return;
  if (ctl->stop != STOP_NONE) {  // a stop is final (the passes before this launch were skipped)
    if (ctl_host) *ctl_host = *ctl;
    return;
  }
  const double rho = sqrt(ss);
  const int it = ctl->it;
  const double prev = ctl->rho;
  const double res0 = it == 0 ? rho : ctl->res0;
  ctl->res0 = res0;
  ctl->rho = rho;
  int stop = STOP_NONE;
  if (gs && __hip_atomic_load(&gs->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
    stop = STOP_DEVICE;
  else if (!isfinite(rho))
    stop = STOP_NONFINITE;
  else if (rho <= rule.rtol * res0)
    stop = STOP_CONVERGED;
  else if (rule.stall > 0 && it >= 1 && rho > rule.stall * prev)
    stop = STOP_STALLED;
  else if (it >= rule.max_iter)
    stop = STOP_MAX_ITER;
  else if (rule.diverge_factor > 0 && rho > rule.diverge_factor * res0)
    stop = STOP_DIVERGED;
  ctl->stop = stop;
  if (stop == STOP_NONE) ctl->it = it + 1;
  if (ctl_host) *ctl_host = *ctl;  // pinned host memory, visible once the kernel has completed
}

__global__ void gather_rows_kernel(const double *__restrict__ src, int64_t stride, double *__restrict__ dst,
                                   int64_t rows, int nx) {
  const int64_t total = rows * (int64_t)nx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / nx;
    const int64_t c = i - r * nx;
    dst[i] = src[r * stride * nx + c];
  }
}

// Seeded U[0,1) rows from SplitMix64 in counter form: dst row r holds time
// point n = n0 + r * dn, and point (n, i) takes output k = (n-1) nx + i, i.e.
// the state seed + (k+1) * gamma mixed, its top 53 bits scaled by 2^-53.
__global__ void splitmix_rows_kernel(double *__restrict__ dst, int64_t rows, int64_t n0, int64_t dn, int nx,
                                     uint64_t seed) {
  const int64_t total = rows * (int64_t)nx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / nx;
    const int64_t col = i - r * nx;
    const uint64_t k = (uint64_t)((n0 + r * dn - 1) * (int64_t)nx + col);
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    dst[i] = (double)(z >> 11) * 0x1p-53;
  }
}

__global__ void fill_kernel(double *__restrict__ dst, int64_t n, double value, const int *stop) {
  if (stop && *stop) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = value;
}

__global__ void fill32_kernel(float *__restrict__ dst, int64_t n, const int *stop) {
  if (stop && *stop) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = 0.0f;
}

__global__ void round32_kernel(const double *__restrict__ src, float *__restrict__ dst, int64_t n, const int *stop) {
  if (stop && *stop) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

__global__ void add32_kernel(double *__restrict__ u, const float *__restrict__ e, int64_t n, const int *stop) {
  if (stop && *stop) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    u[i] += (double)e[i];
}

// Start a solve's iteration state: zero, or already stopped (STOP_OUTER)
// when the gate is set (the outer refinement loop has stopped, so the inner
// solve queued behind its decision does nothing).
__global__ void ctl_reset_kernel(SolveCtl *ctl, const int *gate) {
  if (threadIdx.x != 0) return;
  SolveCtl c{};
  c.stop = (gate && *gate) ? STOP_OUTER : STOP_NONE;
  *ctl = c;
}

unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 65536); }

}  // namespace

size_t lds_bytes_for(const Layout &lay, int has_solve) {
  return (size_t)lds_offsets(lay, has_solve).total * sizeof(double);
}

hipError_t configure_kernels(size_t bytes) {
  hipError_t e;
  if ((e = configure_lean_kernels(bytes))) return e;
  if ((e = configure_window_kernels64(bytes))) return e;
  if ((e = configure_window_kernels32(bytes))) return e;
  if ((e = configure_gmres_kernels(bytes))) return e;
  if ((e = configure_step_poly_z(bytes))) return e;
  if ((e = configure_step_poly_w(bytes))) return e;
  if ((e = configure_step_slc(bytes))) return e;
  if ((e = configure_step32_poly_z(bytes))) return e;
  if ((e = configure_step32_poly_w(bytes))) return e;
  return configure_step32_slc(bytes);
}

hipError_t launch_pass32(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs32 &pa,
                         hipStream_t stream) {
  if (pa.nint <= 0) return hipSuccess;
  if (lean_slc_applies(op, lay)) return launch_lean32(desc, op, lay, pa, stream);
  if (window_applies(op, lay)) return launch_window32(desc, op, lay, pa, stream);
  const size_t lds = lds_bytes_for(lay, op.has_solve);
  switch (op.kind) {
    case OP_POLY_Z: return launch_step32_poly_z(desc, lay, pa, lds, stream);
    case OP_POLY_W: return launch_step32_poly_w(desc, lay, pa, lds, stream);
    case OP_SLC: return launch_step32_slc(desc, lay, pa, lds, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill32(float *dst, int64_t n, hipStream_t stream, const int *stop) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill32_kernel, dim3(grid_for(n)), dim3(256), 0, stream, dst, n, stop);
  return hipGetLastError();
}

hipError_t launch_round32(const double *src, float *dst, int64_t n, hipStream_t stream, const int *stop) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(round32_kernel, dim3(grid_for(n)), dim3(256), 0, stream, src, dst, n, stop);
  return hipGetLastError();
}

hipError_t launch_add32(double *u, const float *e, int64_t n, hipStream_t stream, const int *stop) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(add32_kernel, dim3(grid_for(n)), dim3(256), 0, stream, u, e, n, stop);
  return hipGetLastError();
}

hipError_t launch_ctl_reset(SolveCtl *ctl, const int *gate, hipStream_t stream) {
  hipLaunchKernelGGL(ctl_reset_kernel, dim3(1), dim3(64), 0, stream, ctl, gate);
  return hipGetLastError();
}

hipError_t launch_pass(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs &pa,
                       hipStream_t stream) {
  if (pa.nint <= 0) return hipSuccess;
  if (op.kind == OP_SLC && op.gmres_max > 0) return launch_gmres(desc, op, lay, pa, stream);
  if (lean_slc_applies(op, lay)) return launch_lean(desc, op, lay, pa, stream);
  if (window_applies(op, lay)) return launch_window(desc, op, lay, pa, stream);
  const size_t lds = lds_bytes_for(lay, op.has_solve);
  switch (op.kind) {
    case OP_POLY_Z: return launch_step_poly_z(desc, lay, pa, lds, stream);
    case OP_POLY_W: return launch_step_poly_w(desc, lay, pa, lds, stream);
    case OP_SLC: return launch_step_slc(desc, lay, pa, lds, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tiles(const LevelDesc *desc, const TileGeom &tg, const TileArgs &ta, hipStream_t stream) {
  if (ta.nint <= 0) return hipSuccess;
  switch (tg.P) {
    case 4: return launch_tiles_4(desc, tg, ta, stream);
    case 8: return launch_tiles_8(desc, tg, ta, stream);
    case 16: return launch_tiles_16(desc, tg, ta, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tiles32(const LevelDesc *desc, const TileGeom &tg, const TileArgs32 &ta, hipStream_t stream) {
  if (ta.nint <= 0) return hipSuccess;
  switch (tg.P) {
    case 4: return launch_tiles_4(desc, tg, ta, stream);
    case 8: return launch_tiles_8(desc, tg, ta, stream);
    case 16: return launch_tiles_16(desc, tg, ta, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce(const double *part, int64_t n, double *out, hipStream_t stream) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(RED_T), 0, stream, part, n, out);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const double *src, int64_t stride, double *dst, int64_t rows, int nx,
                              hipStream_t stream) {
  const int64_t total = rows * (int64_t)nx;
  if (total <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks), dim3(256), 0, stream, src, stride, dst, rows, nx);
  return hipGetLastError();
}

hipError_t launch_splitmix_rows(double *dst, int64_t rows, int64_t n0, int64_t dn, int nx, uint64_t seed,
                                hipStream_t stream) {
  const int64_t total = rows * (int64_t)nx;
  if (total <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(splitmix_rows_kernel, dim3(blocks), dim3(256), 0, stream, dst, rows, n0, dn, nx, seed);
  return hipGetLastError();
}

hipError_t launch_fill(double *dst, int64_t n, double value, hipStream_t stream, const int *stop) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, stream, dst, n, value, stop);
  return hipGetLastError();
}

hipError_t launch_solve_ctl(const double *part, int64_t n, SolveCtl *ctl, SolveCtl *ctl_host, const GridSync *gs,
                            StopRule rule, hipStream_t stream) {
  hipLaunchKernelGGL(solve_ctl_kernel, dim3(1), dim3(RED_T), 0, stream, part, n, ctl, ctl_host, gs, rule);
  return hipGetLastError();
}

}  // namespace mgrit