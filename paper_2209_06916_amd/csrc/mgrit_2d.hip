// gfx950 kernels of the 2D extension (dimension-split reading): the fused
// explicit Runge-Kutta step on 2D tiles, the batched slab transpose that
// lets the 1D coarse-step kernels run along y, and small batched slab
// operations.  Slabs are [ny][nx] float64, x contiguous; a batch of nb slabs
// has a stride (in elements) between consecutive slabs.
#include "mgrit_internal.h"

namespace mgrit {

namespace {

constexpr int TX = 64, TY = 16;  // output tile of one workgroup (256 threads)

// One explicit Runge-Kutta step Phi = R(Z), Z = -(c_x L_p^(x) + c_y L_p^(y)),
// as the Horner form y <- coef[i] u + Z y, on one TX x TY output tile of one
// slab.  The tile and a halo of s*l (left/below) and s*r (right/above)
// points on each axis sit in LDS; every stencil application shrinks the
// valid region by the stencil extent, so after the s applications exactly
// the output tile is valid.  dst = Phi(src) (+ g).
template <class T>
__global__ void __launch_bounds__(256) step2d_kernel(Step2dArgsT<T> a) {
  extern __shared__ double lds_raw[];
  T *lds = reinterpret_cast<T *>(lds_raw);
  const int nx = a.nx, ny = a.ny;
  const int s = a.ncoef - 1;  // stencil applications
  const int hl = s * a.sl, hr = s * a.sr;
  const int wx = TX + hl + hr, wy = TY + hl + hr;
  const int area = wx * wy;
  T *u = lds, *y0 = lds + area, *y1 = lds + 2 * area;
  const int tiles_x = (nx + TX - 1) / TX, tiles_y = (ny + TY - 1) / TY;
  const int64_t item = blockIdx.x;
  const int64_t b = item / ((int64_t)tiles_x * tiles_y);
  const int t = (int)(item - b * tiles_x * tiles_y);
  const int x0 = (t % tiles_x) * TX - hl, y0g = (t / tiles_x) * TY - hl;
  const T *src = a.src + b * a.src_stride;
  const T top = (T)a.coef[a.ncoef - 1];
  // Every loop below walks a w x h region in row-major order, 256 points
  // apart: each thread keeps its (x, y) and advances it by (256 mod w,
  // 256 div w) with one carry, so no lane idles and nothing divides.
  const int tid = threadIdx.x;
  {
    int lx = tid % wx, ly = tid / wx;
    const int dx = 256 % wx, dy = 256 / wx;
    for (; ly < wy;) {
      int gy = y0g + ly;
      while (gy < 0) gy += ny;
      while (gy >= ny) gy -= ny;
      int gx = x0 + lx;
      while (gx < 0) gx += nx;
      while (gx >= nx) gx -= nx;
      const T v = src[(int64_t)gy * nx + gx];
      u[ly * wx + lx] = v;
      y0[ly * wx + lx] = top * v;
      lx += dx;
      ly += dy;
      if (lx >= wx) {
        lx -= wx;
        ++ly;
      }
    }
  }
  __syncthreads();
  const int nt_ = a.sl + a.sr + 1;
  T tapx[MAXTAPS], tapy[MAXTAPS];
#pragma unroll
  for (int k = 0; k < MAXTAPS; ++k) {
    tapx[k] = (T)a.tx[k];
    tapy[k] = (T)a.ty[k];
  }
  T *yin = y0, *yout = y1;
  for (int k = 1; k <= s; ++k) {
    const T ci = (T)a.coef[a.ncoef - 1 - k];
    // valid after this application: [k*sl, w - k*sr) on both axes
    const int lo = k * a.sl, hx = wx - k * a.sr, hy = wy - k * a.sr;
    const int cw = hx - lo, ch = hy - lo;
    int lx = tid % cw, ly = tid / cw;
    const int dx = 256 % cw, dy = 256 / cw;
    for (; ly < ch;) {
      const int c = (ly + lo) * wx + lx + lo;
      T acc = ci * u[c];
#pragma unroll
      for (int tt = 0; tt < MAXTAPS; ++tt) {
        if (tt < nt_) {
          const int d = tt - a.sl;
          acc = fma(tapx[tt], yin[c + d], acc);
          acc = fma(tapy[tt], yin[c + d * wx], acc);
        }
      }
      yout[c] = acc;
      lx += dx;
      ly += dy;
      if (lx >= cw) {
        lx -= cw;
        ++ly;
      }
    }
    __syncthreads();
    T *tmp = yin;
    yin = yout;
    yout = tmp;
  }
  T *dst = a.dst + b * a.dst_stride;
  const T *g = a.g ? a.g + b * a.g_stride : nullptr;
  const T gs = (T)a.g_scale;
  for (int i = tid; i < TX * TY; i += 256) {
    const int ox = i & (TX - 1), oy = i / TX;  // TX is a power of two
    const int gy = y0g + hl + oy;
    const int gx = x0 + hl + ox;
    if (gx >= nx || gy >= ny) continue;
    const int64_t o = (int64_t)gy * nx + gx;
    T v = yin[(oy + hl) * wx + ox + hl];
    if (g) v = fma(gs, g[o], v);
    dst[o] = v;
  }
}

// Whole-wavefront shift of a double by one lane: WAVE_SHR1 (0x138) gives lane
// l the value of lane l-1, WAVE_SHL1 (0x130) that of lane l+1; the lane
// without a source reads 0.
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffff), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// The same step with no LDS, for stencils whose halo fits a wavefront: one
// wavefront owns a tile of 64 columns (lane = column) by WY rows, every value
// in registers.  x-neighbours come from whole-wavefront lane shifts, y
// neighbours from the lane's own registers; each of the NS stencil
// applications leaves one more ring of SL (left, below) / SR (right, above)
// points invalid, which the halo absorbs.  Output: the TXR = 64 - NS (SL +
// SR) middle columns of rows NS SL .. WY - NS SR.  Four independent tiles per
// workgroup.
template <int SL, int SR, int NS, int WY, class T>
__global__ void __launch_bounds__(256) step2d_reg_kernel(Step2dArgsT<T> a) {
  constexpr int HL = NS * SL, HR = NS * SR;
  constexpr int TXR = WAVE - HL - HR, TYR = WY - HL - HR;
  constexpr int NT = SL + SR + 1;
  const int nx = a.nx, ny = a.ny;
  const int tiles_x = (nx + TXR - 1) / TXR, tiles_y = (ny + TYR - 1) / TYR;
  const int64_t per_slab = (int64_t)tiles_x * tiles_y;
  const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= per_slab * a.nb) return;  // whole wavefront leaves together
  const int64_t b = item / per_slab;
  const int t = (int)(item - b * per_slab);
  const int lane = threadIdx.x & (WAVE - 1);
  const int x0 = (t % tiles_x) * TXR - HL, y0 = (t / tiles_x) * TYR - HL;
  int gx = x0 + lane;
  while (gx < 0) gx += nx;
  while (gx >= nx) gx -= nx;
  const T *src = a.src + b * a.src_stride;
  T u[WY], y[WY];
  const T top = (T)a.coef[NS];
#pragma unroll
  for (int r = 0; r < WY; ++r) {
    int gy = y0 + r;
    while (gy < 0) gy += ny;
    while (gy >= ny) gy -= ny;
    u[r] = src[(int64_t)gy * nx + gx];
    y[r] = top * u[r];
  }
  T tx[NT], ty[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    tx[k] = (T)a.tx[k];
    ty[k] = (T)a.ty[k];
  }
#pragma unroll
  for (int k = 1; k <= NS; ++k) {
    const T ci = (T)a.coef[NS - k];
    // rows are updated in place, bottom to top; the SL previous rows' old
    // values wait in a ring for the rows above that still read them
    T ring[SL > 0 ? SL : 1];
#pragma unroll
    for (int j = 0; j < SL; ++j) ring[j] = y[k * SL - SL + j];
#pragma unroll
    for (int r = k * SL; r < WY - k * SR; ++r) {
      // x-neighbours y(x + d), d = -SL..SR, by lane shifts
      T xs[NT];
      xs[SL] = y[r];
#pragma unroll
      for (int d = 1; d <= SL; ++d) xs[SL - d] = lane_shift<0x138>(xs[SL - d + 1]);
#pragma unroll
      for (int d = 1; d <= SR; ++d) xs[SL + d] = lane_shift<0x130>(xs[SL + d - 1]);
      T ax = ci * u[r], ay = T(0);
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        ax = fma(tx[tt], xs[tt], ax);
        ay = fma(ty[tt], tt < SL ? ring[tt < SL ? tt : 0] : y[r + tt - SL], ay);
      }
#pragma unroll
      for (int j = 0; j + 1 < SL; ++j) ring[j] = ring[j + 1];
      if (SL > 0) ring[SL > 0 ? SL - 1 : 0] = y[r];
      y[r] = ax + ay;
    }
  }
  const int ox = x0 + lane;
  if (lane < HL || lane >= HL + TXR || ox >= nx) return;
  T *dst = a.dst + b * a.dst_stride;
  const T *g = a.g ? a.g + b * a.g_stride : nullptr;
  const T gs = (T)a.g_scale;
#pragma unroll
  for (int r = HL; r < HL + TYR; ++r) {
    const int oy = y0 + r;
    if (oy >= ny) break;
    const int64_t o = (int64_t)oy * nx + ox;
    T v = y[r];
    if (g) v = fma(gs, g[o], v);
    dst[o] = v;
  }
}

template <int SL, int SR, int NS, int WY, class T>
hipError_t launch_step2d_reg(const Step2dArgsT<T> &a, hipStream_t stream) {
  constexpr int TXR = WAVE - NS * (SL + SR), TYR = WY - NS * (SL + SR);
  const int64_t tiles = (int64_t)((a.nx + TXR - 1) / TXR) * ((a.ny + TYR - 1) / TYR) * a.nb;
  hipLaunchKernelGGL((step2d_reg_kernel<SL, SR, NS, WY, T>), dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

// dst slab b = transpose of src slab b ([rows][cols] -> [cols][rows]),
// plus g slab b (already in the destination layout) when given.
template <class T>
__global__ void __launch_bounds__(256) transpose_kernel(const T *__restrict__ src, int64_t src_stride,
                                                         T *__restrict__ dst, int64_t dst_stride,
                                                         const T *__restrict__ g, int64_t g_stride, int rows,
                                                         int cols) {
  __shared__ T tile[32][33];
  const int tiles_c = (cols + 31) / 32, tiles_r = (rows + 31) / 32;
  const int64_t item = blockIdx.x;
  const int64_t b = item / ((int64_t)tiles_c * tiles_r);
  const int t = (int)(item - b * tiles_c * tiles_r);
  const int c0 = (t % tiles_c) * 32, r0 = (t / tiles_c) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const T *s = src + b * src_stride;
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = s[(int64_t)r * cols + c];
  }
  __syncthreads();
  T *d = dst + b * dst_stride;
  const T *gg = g ? g + b * g_stride : nullptr;
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;  // destination row c, column r
    if (r < rows && c < cols) {
      const int64_t o = (int64_t)c * rows + r;
      T v = tile[tx][k];
      if (gg) v += gg[o];
      d[o] = v;
    }
  }
}

// dst slab b (+)= src slab b, n points per slab
template <class T>
__global__ void __launch_bounds__(256) slab_axpy_kernel(T *__restrict__ dst, int64_t dst_stride,
                                                         const T *__restrict__ src, int64_t src_stride, int64_t nb,
                                                         int64_t n, int accumulate) {
  const int64_t total = nb * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / n, j = i - b * n;
    const T v = src[b * src_stride + j];
    T *p = dst + b * dst_stride + j;
    *p = accumulate ? *p + v : v;
  }
}

// r slab b = a slab b - c slab b (c NULL: 0); part[b * blocks_per_slab + k] =
// sum of squares over block k of slab b, in float64 (fixed order:
// deterministic)
template <class T>
__global__ void __launch_bounds__(256) slab_resid_kernel(const T *__restrict__ a, const T *__restrict__ c,
                                                          T *__restrict__ r, int64_t n, int blocks_per_slab,
                                                          double *__restrict__ part) {
  __shared__ double red[256];
  const int64_t b = blockIdx.x / blocks_per_slab;
  const int k = (int)(blockIdx.x - b * blocks_per_slab);
  const int64_t chunk = (n + blocks_per_slab - 1) / blocks_per_slab;
  const int64_t j0 = k * chunk, j1 = min(n, j0 + chunk);
  double ss = 0.0;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
    const T v = c ? a[b * n + j] - c[b * n + j] : a[b * n + j];
    if (r) r[b * n + j] = v;
    ss = fma((double)v, (double)v, ss);
  }
  red[threadIdx.x] = ss;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

unsigned blocks_for(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 65536); }

}  // namespace

size_t step2d_lds_bytes(int ncoef, int sl, int sr) {
  const int s = ncoef - 1;
  return (size_t)3 * (TX + s * (sl + sr)) * (TY + s * (sl + sr)) * sizeof(double);
}

hipError_t configure_2d_kernels(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)step2d_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e) return e;
  return hipFuncSetAttribute((const void *)step2d_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <class T>
hipError_t launch_step2d(const Step2dArgsT<T> &a, hipStream_t stream) {
  if (a.nb <= 0) return hipSuccess;
  // register tiles where the halo leaves most of a wavefront: the common
  // ERK1 + U1 and ERK3 + U3 steps; the LDS tiles otherwise
  if (a.use_reg && a.sl == 2 && a.sr == 1 && a.ncoef == 4) return launch_step2d_reg<2, 1, 3, 24>(a, stream);
  if (a.use_reg && a.sl == 1 && a.sr == 0 && a.ncoef == 2) return launch_step2d_reg<1, 0, 1, 32>(a, stream);
  const int64_t tiles = (int64_t)((a.nx + TX - 1) / TX) * ((a.ny + TY - 1) / TY);
  const size_t lds = step2d_lds_bytes(a.ncoef, a.sl, a.sr);
  hipLaunchKernelGGL(step2d_kernel<T>, dim3((unsigned)(tiles * a.nb)), dim3(256), lds, stream, a);
  return hipGetLastError();
}

template <class T>
hipError_t launch_transpose(const T *src, int64_t src_stride, T *dst, int64_t dst_stride, const T *g, int64_t g_stride,
                            int64_t nb, int rows, int cols, hipStream_t stream) {
  if (nb <= 0) return hipSuccess;
  const int64_t tiles = (int64_t)((cols + 31) / 32) * ((rows + 31) / 32);
  hipLaunchKernelGGL(transpose_kernel<T>, dim3((unsigned)(tiles * nb)), dim3(256), 0, stream, src, src_stride, dst,
                     dst_stride, g, g_stride, rows, cols);
  return hipGetLastError();
}

template <class T>
hipError_t launch_slab_axpy(T *dst, int64_t dst_stride, const T *src, int64_t src_stride, int64_t nb, int64_t n,
                            bool accumulate, hipStream_t stream) {
  if (nb <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(slab_axpy_kernel<T>, dim3(blocks_for(nb * n)), dim3(256), 0, stream, dst, dst_stride, src,
                     src_stride, nb, n, accumulate ? 1 : 0);
  return hipGetLastError();
}

template <class T>
hipError_t launch_slab_resid(const T *a, const T *c, T *r, int64_t nb, int64_t n, int blocks_per_slab, double *part,
                             hipStream_t stream) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(slab_resid_kernel<T>, dim3((unsigned)(nb * blocks_per_slab)), dim3(256), 0, stream, a, c, r, n,
                     blocks_per_slab, part);
  return hipGetLastError();
}

hipError_t launch_slab_norm(const double *a, int64_t nb, int64_t n, int blocks_per_slab, double *part,
                            hipStream_t stream) {
  return launch_slab_resid<double>(a, nullptr, nullptr, nb, n, blocks_per_slab, part, stream);
}

template hipError_t launch_step2d<double>(const Step2dArgsT<double> &, hipStream_t);
template hipError_t launch_step2d<float>(const Step2dArgsT<float> &, hipStream_t);
template hipError_t launch_transpose<double>(const double *, int64_t, double *, int64_t, const double *, int64_t,
                                             int64_t, int, int, hipStream_t);
template hipError_t launch_transpose<float>(const float *, int64_t, float *, int64_t, const float *, int64_t, int64_t,
                                            int, int, hipStream_t);
template hipError_t launch_slab_axpy<double>(double *, int64_t, const double *, int64_t, int64_t, int64_t, bool,
                                             hipStream_t);
template hipError_t launch_slab_axpy<float>(float *, int64_t, const float *, int64_t, int64_t, int64_t, bool,
                                            hipStream_t);
template hipError_t launch_slab_resid<double>(const double *, const double *, double *, int64_t, int64_t, int,
                                              double *, hipStream_t);
template hipError_t launch_slab_resid<float>(const float *, const float *, float *, int64_t, int64_t, int, double *,
                                             hipStream_t);

}  // namespace mgrit
