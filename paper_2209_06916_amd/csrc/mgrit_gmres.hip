// gfx950 kernel for coarse steps whose periodic solve is approximate: the
// corrected semi-Lagrangian step Psi = T^{-1} S (eq. MOL-SL-corrected) with
// T x = S u solved by GMRES from a zero start until the residual falls by
// gmres_rtol or after gmres_max iterations, the coarse solver of the paper's
// multilevel ERK runs (Sec. 6.3).
//
// One workgroup per vector (a CF-interval's slab), L points per thread as in
// the generic step kernel.  The Arnoldi basis lives in global memory, one
// slab of (gmres_max + 1) vectors per workgroup, each thread reading back only
// the chunk it wrote.  T is applied as its symmetric stencil through a padded
// LDS vector; inner products are workgroup reductions in a fixed order
// (every thread gets the same value), so every thread takes the same
// decisions; the Givens rotations and the final triangular solve run on
// thread 0 in LDS.  Modified Gram-Schmidt, as the textbook algorithm.
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"
#include "mgrit_step.h"

// LDS layout (doubles): padded vector, two banks of per-wavefront partial
// sums, the Hessenberg column, the rotated R (kmax x kmax), cosines, sines,
// the rotated right-hand side, the least-squares solution, a stop flag, and
// the reduction scratch of the pass (block_sum).
struct GmresLds {
  int red, hcol, R, cs, sn, g, y, flag, bsum, total;
};
__host__ __device__ inline GmresLds gmres_lds(int nx, int kmax) {
  GmresLds o{};
  int off = nx + (nx >> 4) + 1;
  o.red = off;
  off += 2 * MAXWAVES;
  o.hcol = off;
  off += kmax + 1;
  o.R = off;
  off += kmax * kmax;
  o.cs = off;
  off += kmax;
  o.sn = off;
  off += kmax;
  o.g = off;
  off += kmax + 1;
  o.y = off;
  off += kmax;
  o.flag = off;
  off += 1;
  o.bsum = off;
  off += MAXWAVES;
  o.total = off;
  return o;
}

// sum over the workgroup of a . b (this thread's cnt points), the same
// value in every thread; rb alternates between the two banks so that a
// reduction never overwrites partial sums another thread has yet to read
template <int L>
__device__ __forceinline__ double bdot(const double (&a)[L], const double (&b)[L], int cnt, double *red, int &rb) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < L; ++j)
    if (j < cnt) s = fma(a[j], b[j], s);
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
  double *bank = red + rb * MAXWAVES;
  if ((threadIdx.x & (WAVE - 1)) == 0) bank[threadIdx.x >> 6] = s;
  __syncthreads();
  const int nw = blockDim.x >> 6;
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += bank[w];
  rb ^= 1;
  return t;
}

template <int L>
__device__ __forceinline__ void load_own(const double *__restrict__ v, int base, int cnt, double (&x)[L]) {
#pragma unroll
  for (int j = 0; j < L; ++j) x[j] = (j < cnt) ? v[base + j] : 0.0;
}

template <int L>
__device__ __forceinline__ void store_own(double *__restrict__ v, int base, int cnt, const double (&x)[L]) {
#pragma unroll
  for (int j = 0; j < L; ++j)
    if (j < cnt) v[base + j] = x[j];
}

// x <- approximately T^{-1} b by GMRES (x0 = 0); V: this workgroup's basis slab.
template <int L>
__device__ void gmres_solve(const double (&b)[L], double (&x)[L], int cnt, int nx, const StepOp &op, double *V,
                            double *vec, double *sm, const GmresLds &lo) {
  const int tid = threadIdx.x;
  const int base = tid * L;
  const int kmax = op.gmres_max;
  const double rtol = op.gmres_rtol;
  double *red = sm + lo.red, *hcol = sm + lo.hcol, *R = sm + lo.R, *cs = sm + lo.cs, *sn = sm + lo.sn;
  double *g = sm + lo.g, *ys = sm + lo.y, *flag = sm + lo.flag;
  double tt[MAXTAPS];
#pragma unroll
  for (int t = 0; t < MAXTAPS; ++t) tt[t] = op.ttaps[t];
  const int width = 2 * op.t_k + 1;
  int rb = 0;
  const double beta = sqrt(bdot<L>(b, b, cnt, red, rb));
#pragma unroll
  for (int j = 0; j < L; ++j) x[j] = 0.0;
  if (beta == 0.0) return;  // b = 0 (the same in every thread): x = 0
  double vj[L];
#pragma unroll
  for (int j = 0; j < L; ++j) vj[j] = b[j] / beta;
  store_own<L>(V, base, cnt, vj);
  if (tid == 0) g[0] = beta;
  int k = 0;
  for (int j = 0; j < kmax; ++j) {
    // w = T v_j through the padded LDS vector
    double w[L];
    __syncthreads();
    chunk_to_lds<L>(vec, base, cnt, vj);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < L; ++q) w[q] = 0.0;
    window_combine<L>(vec, wrap_lo(base - op.t_k, nx), cnt, width, nx, tt, w);
    // modified Gram-Schmidt against v_0 .. v_j
    for (int i = 0; i <= j; ++i) {
      double vi[L];
      if (i == j) {
#pragma unroll
        for (int q = 0; q < L; ++q) vi[q] = vj[q];
      } else {
        load_own<L>(V + (int64_t)i * nx, base, cnt, vi);
      }
      const double h = bdot<L>(w, vi, cnt, red, rb);
#pragma unroll
      for (int q = 0; q < L; ++q) w[q] = fma(-h, vi[q], w[q]);
      if (tid == 0) hcol[i] = h;
    }
    const double hn = sqrt(bdot<L>(w, w, cnt, red, rb));
    if (tid == 0) {
      hcol[j + 1] = hn;
      for (int i = 0; i < j; ++i) {
        const double a = hcol[i], c = hcol[i + 1];
        hcol[i] = cs[i] * a + sn[i] * c;
        hcol[i + 1] = -sn[i] * a + cs[i] * c;
      }
      const double den = hypot(hcol[j], hcol[j + 1]);
      cs[j] = hcol[j] / den;
      sn[j] = hcol[j + 1] / den;
      for (int i = 0; i < j; ++i) R[i * kmax + j] = hcol[i];
      R[j * kmax + j] = den;
      const double gj = g[j];
      g[j] = cs[j] * gj;
      g[j + 1] = -sn[j] * gj;
      flag[0] = (fabs(g[j + 1]) <= rtol * beta || den == 0.0 || j + 1 == kmax || hn == 0.0) ? 1.0 : 0.0;
    }
    __syncthreads();
    k = j + 1;
    if (flag[0] != 0.0) break;
#pragma unroll
    for (int q = 0; q < L; ++q) vj[q] = w[q] / hn;
    store_own<L>(V + (int64_t)(j + 1) * nx, base, cnt, vj);
  }
  // least squares: R y = g (upper triangular), then x = V y
  if (tid == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int c = i + 1; c < k; ++c) s -= R[i * kmax + c] * ys[c];
      ys[i] = s / R[i * kmax + i];
    }
  }
  __syncthreads();
  for (int i = 0; i < k; ++i) {
    double vi[L];
    load_own<L>(V + (int64_t)i * nx, base, cnt, vi);
    const double yi = ys[i];
#pragma unroll
    for (int q = 0; q < L; ++q) x[q] = fma(yi, vi[q], x[q]);
  }
}

template <int L, int MAXT>
__global__ void __launch_bounds__(MAXT) gmres_step_kernel(const LevelDesc *__restrict__ desc, PassArgs pa) {
  if (pa.stop && *pa.stop) return;  // the solve has already stopped
  extern __shared__ double smem[];
  const Layout lay = desc->lay;
  const StepOp &op = desc->op;
  const int nx = lay.nx;
  const int tid = threadIdx.x;
  const int base = tid * L;
  const int cnt = min(max(nx - base, 0), L);
  const GmresLds lo = gmres_lds(nx, op.gmres_max);
  double *vec = smem;
  double *V = op.krylov + (int64_t)blockIdx.x * (op.gmres_max + 1) * nx;
  double w[MAXTAPS];
#pragma unroll
  for (int t = 0; t < MAXTAPS; ++t) w[t] = op.slw[t];
  const int width = op.sl_l + op.sl_r + 1;
  const int off = op.sl_K + op.sl_l;
  run_chain<L, double>(pa, nx, cnt, smem + lo.bsum, [&](double (&u)[L]) {
    for (int rep = 0; rep < op.repeat; ++rep) {
      // the semi-Lagrangian step S u
      __syncthreads();
      chunk_to_lds<L>(vec, base, cnt, u);
      __syncthreads();
      double y[L];
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = 0.0;
      window_combine<L>(vec, wrap_lo(base - off, nx), cnt, width, nx, w, y);
      gmres_solve<L>(y, u, cnt, nx, op, V, vec, smem, lo);
    }
  });
}

template <int L>
hipError_t gmres_launch_l(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, size_t lds,
                          hipStream_t stream) {
  if (lay.T <= 256)
    hipLaunchKernelGGL((gmres_step_kernel<L, 256>), dim3((unsigned)pa.nint), dim3(lay.T), lds, stream, desc, pa);
  else
    hipLaunchKernelGGL((gmres_step_kernel<L, 1024>), dim3((unsigned)pa.nint), dim3(lay.T), lds, stream, desc, pa);
  return hipGetLastError();
}

}  // namespace

size_t gmres_lds_bytes(const Layout &lay, int kmax) { return (size_t)gmres_lds(lay.nx, kmax).total * sizeof(double); }

// One launch per chunk of at most krylov_cap vectors, in stream order so that
// the chunks reuse the same basis slabs (only MODE_APPLY can ask for more
// workgroups than the level has intervals).
hipError_t launch_gmres(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs &pa,
                        hipStream_t stream) {
  if (pa.nint <= 0) return hipSuccess;
  if (op.gmres_max < 1 || op.gmres_max > GMRES_MAX || !op.krylov || op.krylov_cap < 1) return hipErrorInvalidValue;
  if (lay.T < WAVE || lay.T > 1024 || lay.T % WAVE) return hipErrorInvalidValue;
  if (pa.nint > op.krylov_cap && pa.mode != MODE_APPLY) return hipErrorInvalidValue;
  const size_t lds = gmres_lds_bytes(lay, op.gmres_max);
  for (int64_t b0 = 0; b0 < pa.nint; b0 += op.krylov_cap) {
    PassArgs p = pa;
    p.nint = std::min<int64_t>(op.krylov_cap, pa.nint - b0);
    if (pa.mode == MODE_APPLY) {
      p.cin = pa.cin + b0 * lay.nx;
      p.cout = pa.cout + b0 * lay.nx;
    }
    hipError_t e = hipSuccess;
    switch (lay.L) {
      case 2: e = gmres_launch_l<2>(desc, lay, p, lds, stream); break;
      case 4: e = gmres_launch_l<4>(desc, lay, p, lds, stream); break;
      case 8: e = gmres_launch_l<8>(desc, lay, p, lds, stream); break;
      case 16: e = gmres_launch_l<16>(desc, lay, p, lds, stream); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t configure_gmres_kernels(size_t bytes) {
  hipError_t e = hipSuccess;
#define MGRIT_GMRES_ATTR(Lv)                                                                                 \
  if (e == hipSuccess)                                                                                      \
    e = hipFuncSetAttribute((const void *)gmres_step_kernel<Lv, 256>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                            (int)bytes);                                                                    \
  if (e == hipSuccess)                                                                                      \
    e = hipFuncSetAttribute((const void *)gmres_step_kernel<Lv, 1024>,                                       \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  MGRIT_GMRES_ATTR(2)
  MGRIT_GMRES_ATTR(4)
  MGRIT_GMRES_ATTR(8)
  MGRIT_GMRES_ATTR(16)
#undef MGRIT_GMRES_ATTR
  return e;
}

}  // namespace mgrit
