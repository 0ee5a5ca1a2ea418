// gfx950 kernels for MGRIT on method-of-lines advection.
//
// One workgroup advances one spatial vector (a CF-interval's slab, Sec. 2.2)
// through a chain of time steps.  The vector lives in registers as contiguous
// per-thread chunks of L points; LDS holds a padded copy whenever a step needs
// neighbours (the upwind stencil of -c L_p, Sec. 4.1) or a long-range gather
// (the semi-Lagrangian interpolation of S_p, Sec. 3).
//
// Periodic banded solves (SDIRK stages, Sec. 4.3 footnote; the corrected
// coarse operator, eq. MOL-SL-corrected) use the host-computed factorisation
//     T = C * F(S^-1) * B(S),
// F with its roots inside the unit circle and B with its roots outside, so
//     T^{-1} x = C^{-1} * (backward recurrence) o (forward recurrence) x.
// Each periodic recurrence y_i = x_i + sum_m a_m y_{i-m} is evaluated as a
// workgroup-wide scan over threads: a zero-state pass per chunk, an
// intra-wavefront Kogge-Stone scan of the k-dimensional chunk states with the
// constant transfer matrix H = M^L (M the companion matrix), a carry across
// wavefronts through LDS, the closed-form periodic wrap s_0 = W (...), and a
// homogeneous correction pass.  No MFMA: nothing here is a dense contraction.
#include "mgrit_internal.h"

namespace mgrit {

namespace {

constexpr int SCR = MAXWAVES * KMAX + KMAX;  // doubles of scan scratch per recurrence

__device__ __forceinline__ int padix(int i) { return i + (i >> 4); }

__device__ __forceinline__ int wrap_hi(int i, int nx) {
  while (i >= nx) i -= nx;
  return i;
}

__device__ __forceinline__ int wrap_lo(int i, int nx) {
  while (i < 0) i += nx;
  return i;
}

template <int L>
__device__ __forceinline__ void load_chunk(const double *__restrict__ row, int base, int cnt, double (&x)[L]) {
#pragma unroll
  for (int j = 0; j < L; ++j) x[j] = (j < cnt) ? row[base + j] : 0.0;
}

template <int L>
__device__ __forceinline__ void store_chunk(double *__restrict__ row, int base, int cnt, const double (&x)[L]) {
#pragma unroll
  for (int j = 0; j < L; ++j)
    if (j < cnt) row[base + j] = x[j];
}

template <int L>
__device__ __forceinline__ void add_chunk_from(const double *__restrict__ row, int base, int cnt, double (&x)[L]) {
#pragma unroll
  for (int j = 0; j < L; ++j)
    if (j < cnt) x[j] += row[base + j];
}

template <int L>
__device__ __forceinline__ void add_chunk_into(double *__restrict__ row, int base, int cnt, const double (&x)[L]) {
#pragma unroll
  for (int j = 0; j < L; ++j)
    if (j < cnt) row[base + j] += x[j];
}

template <int L>
__device__ __forceinline__ void chunk_to_lds(double *vec, int base, int cnt, const double (&x)[L]) {
#pragma unroll
  for (int j = 0; j < L; ++j)
    if (j < cnt) vec[padix(base + j)] = x[j];
}

// out[j] = acc * out[j] + w[0] * v[start+j] + ... + w[width-1] * v[start+j+width-1]
// (indices periodic), reading the padded LDS copy v; 0 <= start < nx.  Each
// LDS value is read once and scattered into the outputs it feeds, so no
// extended window is held in registers.
template <int L>
__device__ __forceinline__ void window_combine(const double *vec, int start, int cnt, int width, int nx,
                                               const double *w, double (&out)[L]) {
#pragma unroll
  for (int e = 0; e < L + MAXTAPS - 1; ++e) {
    if (e < cnt + width - 1) {
      const double v = vec[padix(wrap_hi(start + e, nx))];
#pragma unroll
      for (int t = 0; t < MAXTAPS; ++t) {
        const int j = e - t;
        if (j >= 0 && j < L && t < width) out[j] = fma(w[t], v, out[j]);
      }
    }
  }
}

template <int K>
__device__ __forceinline__ void matvec_add(const double *__restrict__ H, const double (&x)[K], double (&acc)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double s = acc[i];
#pragma unroll
    for (int j = 0; j < K; ++j) s = fma(H[i * K + j], x[j], s);
    acc[i] = s;
  }
}

// Periodic recurrence over the workgroup.  x holds this thread's chunk in
// processing order (REV: register j is processed as element L-1-j, used when
// the backward recurrence runs over the same chunks in reversed thread order).
// vt: this thread's position in processing order; A: threads owning points.
template <int L, int K, bool REV>
__device__ void recurrence(double (&x)[L], int cnt, int vt, int A, int T, const Recurrence &R, double *scr) {
  const double *__restrict__ tab = R.tab;
  constexpr int KK = K * K;
  double a[K];
#pragma unroll
  for (int m = 0; m < K; ++m) a[m] = R.a[m];

  // 1. zero-state pass over the chunk
  double s[K];
#pragma unroll
  for (int m = 0; m < K; ++m) s[m] = 0.0;
#pragma unroll
  for (int e = 0; e < L; ++e) {
    const int j = REV ? (L - 1 - e) : e;
    if (e < cnt) {
      double y = x[j];
#pragma unroll
      for (int m = 0; m < K; ++m) y = fma(a[m], s[m], y);
#pragma unroll
      for (int m = K - 1; m > 0; --m) s[m] = s[m - 1];
      s[0] = y;
      x[j] = y;
    }
  }

  // 2. inclusive scan of chunk states within the wavefront
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x >> 6;
  const int nw = T >> 6;
  const int vl = REV ? (WAVE - 1 - lane) : lane;
  const int vw = REV ? (nw - 1 - wv) : wv;
  double inc[K];
#pragma unroll
  for (int m = 0; m < K; ++m) inc[m] = s[m];
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const int src = (REV ? (lane + d) : (lane - d)) & (WAVE - 1);
    double o[K];
#pragma unroll
    for (int m = 0; m < K; ++m) o[m] = __shfl(inc[m], src, WAVE);
    if (vl >= d) matvec_add<K>(tab + d * KK, o, inc);
  }

  // 3. wavefront totals -> LDS
  if (vl == WAVE - 1) {
#pragma unroll
    for (int m = 0; m < K; ++m) scr[vw * K + m] = inc[m];
  }
  __syncthreads();

  // 4. exclusive prefix: within the wavefront plus the carry of earlier ones
  double E[K];
  {
    const int src = (REV ? (lane + 1) : (lane - 1)) & (WAVE - 1);
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const double o = __shfl(inc[m], src, WAVE);
      E[m] = (vl >= 1) ? o : 0.0;
    }
  }
  if (vw > 0) {
    double X[K];
#pragma unroll
    for (int m = 0; m < K; ++m) X[m] = 0.0;
    const double *__restrict__ H64 = tab + WAVE * KK;
    for (int w2 = 0; w2 < vw; ++w2) {
      double nxt[K];
#pragma unroll
      for (int m = 0; m < K; ++m) nxt[m] = scr[w2 * K + m];
      matvec_add<K>(H64, X, nxt);
#pragma unroll
      for (int m = 0; m < K; ++m) X[m] = nxt[m];
    }
    matvec_add<K>(tab + vl * KK, X, E);
  }

  // 5. periodic wrap: the state entering the first chunk
  double *s0 = scr + MAXWAVES * K;
  if (vt == A - 1) {
    const double *__restrict__ Hlast = tab + (T + 1) * KK;
    const double *__restrict__ Wwrap = Hlast + KK;
    double tq[K];
#pragma unroll
    for (int m = 0; m < K; ++m) tq[m] = s[m];
    matvec_add<K>(Hlast, E, tq);
    double r0[K];
#pragma unroll
    for (int m = 0; m < K; ++m) r0[m] = 0.0;
    matvec_add<K>(Wwrap, tq, r0);
#pragma unroll
    for (int m = 0; m < K; ++m) s0[m] = r0[m];
  }
  __syncthreads();

  // 6. state entering this chunk, 7. homogeneous correction
  if (cnt > 0) {
    double z0[K];
#pragma unroll
    for (int m = 0; m < K; ++m) z0[m] = s0[m];
    double st[K];
#pragma unroll
    for (int m = 0; m < K; ++m) st[m] = E[m];
    matvec_add<K>(tab + vt * KK, z0, st);
#pragma unroll
    for (int e = 0; e < L; ++e) {
      const int j = REV ? (L - 1 - e) : e;
      if (e < cnt) {
        double hv = 0.0;
#pragma unroll
        for (int m = 0; m < K; ++m) hv = fma(a[m], st[m], hv);
#pragma unroll
        for (int m = K - 1; m > 0; --m) st[m] = st[m - 1];
        st[0] = hv;
        x[j] += hv;
      }
    }
  }
}

template <int L, bool REV>
__device__ __forceinline__ void recurrence_k(double (&x)[L], int cnt, int vt, int A, int T, const Recurrence &R,
                                             double *scr) {
  switch (R.k) {
    case 1: recurrence<L, 1, REV>(x, cnt, vt, A, T, R, scr); break;
    case 2: recurrence<L, 2, REV>(x, cnt, vt, A, T, R, scr); break;
    case 3: recurrence<L, 3, REV>(x, cnt, vt, A, T, R, scr); break;
    default: break;
  }
}

// y <- T^{-1} y
template <int L>
__device__ void solve(double (&y)[L], int cnt, const StepOp &op, const Layout &lay, double *vec, double *scr_f,
                      double *scr_b) {
  const int tid = threadIdx.x;
  const int nx = lay.nx;
  if (op.fw.k > 0) recurrence_k<L, false>(y, cnt, tid, lay.A, lay.T, op.fw, scr_f);
  if (op.bw.k > 0) {
    if (!lay.ragged) {
      recurrence_k<L, true>(y, cnt, lay.T - 1 - tid, lay.A, lay.T, op.bw, scr_b);
    } else {
      // redistribute so that thread t owns indices nx-1-(tL+j), j = 0..cnt-1
      const int base = tid * L;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (j < cnt) vec[padix(base + j)] = y[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = (j < cnt) ? vec[padix(nx - 1 - (base + j))] : 0.0;
      recurrence_k<L, false>(y, cnt, tid, lay.A, lay.T, op.bw, scr_b);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (j < cnt) vec[padix(nx - 1 - (base + j))] = y[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = (j < cnt) ? vec[padix(base + j)] : 0.0;
    }
  }
  const double ci = op.cinv;
#pragma unroll
  for (int j = 0; j < L; ++j) y[j] *= ci;
}

// u <- Phi u  (every thread of the workgroup must call this)
template <int L, int KIND>
__device__ void apply_step(double (&u)[L], int cnt, const StepOp &op, const Layout &lay, double *vec,
                           double *scr_f, double *scr_b) {
  const int nx = lay.nx;
  const int base = threadIdx.x * L;
  double y[L];
  for (int rep = 0; rep < op.repeat; ++rep) {
    if (KIND == OP_SLC) {
      __syncthreads();
      chunk_to_lds<L>(vec, base, cnt, u);
      __syncthreads();
      const int start = wrap_lo(base - op.sl_K - op.sl_l, nx);
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = 0.0;
      window_combine<L>(vec, start, cnt, op.sl_l + op.sl_r + 1, nx, op.slw, y);
      if (op.has_solve) solve<L>(y, cnt, op, lay, vec, scr_f, scr_b);
#pragma unroll
      for (int j = 0; j < L; ++j) u[j] = y[j];
    } else if (KIND == OP_POLY_Z) {
      const double top = op.coef[op.ncoef - 1];
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = top * u[j];
      const int start = wrap_lo(base - op.st_l, nx);
      for (int i = op.ncoef - 2; i >= 0; --i) {
        __syncthreads();
        chunk_to_lds<L>(vec, base, cnt, y);
        __syncthreads();
        const double ci = op.coef[i];
#pragma unroll
        for (int j = 0; j < L; ++j) y[j] = ci * u[j];
        window_combine<L>(vec, start, cnt, op.st_l + op.st_r + 1, nx, op.taps, y);
      }
#pragma unroll
      for (int j = 0; j < L; ++j) u[j] = y[j];
    } else {  // OP_POLY_W
      const double top = op.coef[op.ncoef - 1];
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = top * u[j];
      for (int i = op.ncoef - 2; i >= 0; --i) {
        solve<L>(y, cnt, op, lay, vec, scr_f, scr_b);
        const double ci = op.coef[i];
#pragma unroll
        for (int j = 0; j < L; ++j) y[j] = fma(ci, u[j], y[j]);
      }
#pragma unroll
      for (int j = 0; j < L; ++j) u[j] = y[j];
    }
  }
}

// Sum over the workgroup, deterministic order; result valid in thread 0.
__device__ double block_sum(double v, double *red) {
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_down(v, d, WAVE);
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) tot += red[w];
  }
  return tot;
}

template <int L, int KIND, int MAXT>
__global__ void __launch_bounds__(MAXT) step_kernel(const LevelDesc *__restrict__ desc, PassArgs pa) {
  extern __shared__ double smem[];
  const StepOp &op = desc->op;
  const Layout &lay = desc->lay;
  const int nx = lay.nx;
  double *vec = smem;
  double *scr_f = smem + (nx + (nx >> 4) + 1);
  double *scr_b = scr_f + SCR;
  double *red = scr_b + SCR;

  const int tid = threadIdx.x;
  const int base = tid * L;
  const int cnt = min(max(nx - base, 0), L);
  const int64_t b = blockIdx.x;
  const int64_t nxl = nx;
  const int m = pa.m;
  double u[L];

  switch (pa.mode) {
    case MODE_PASS_A: {
      if (pa.zero_init) {
#pragma unroll
        for (int j = 0; j < L; ++j) u[j] = 0.0;
      } else {
        load_chunk<L>(pa.cin + b * nxl, base, cnt, u);
      }
      if (b == 0) store_chunk<L>(pa.cout, base, cnt, u);
      for (int j = 1; j <= m; ++j) {
        apply_step<L, KIND>(u, cnt, op, lay, vec, scr_f, scr_b);
        if (pa.g) add_chunk_from<L>(pa.g + (b * m + j - 1) * nxl, base, cnt, u);
      }
      store_chunk<L>(pa.cout + (b + 1) * nxl, base, cnt, u);
      break;
    }
    case MODE_PASS_B: {
      load_chunk<L>(pa.cin + b * nxl, base, cnt, u);
      for (int j = 1; j <= m; ++j) {
        apply_step<L, KIND>(u, cnt, op, lay, vec, scr_f, scr_b);
        if (pa.g) add_chunk_from<L>(pa.g + (b * m + j - 1) * nxl, base, cnt, u);
      }
      const double *__restrict__ c1 = pa.cin + (b + 1) * nxl;
      double ss = 0.0;
#pragma unroll
      for (int j = 0; j < L; ++j) {
        if (j < cnt) {
          u[j] -= c1[base + j];
          ss = fma(u[j], u[j], ss);
        }
      }
      store_chunk<L>(pa.r + b * nxl, base, cnt, u);
      const double tot = block_sum(ss, red);
      if (tid == 0) pa.normpart[b] = tot;
      break;
    }
    case MODE_POST_F: {
      load_chunk<L>(pa.cin + b * nxl, base, cnt, u);
      add_chunk_into<L>(pa.parent + (b * m) * nxl, base, cnt, u);
      for (int j = 1; j < m; ++j) {
        apply_step<L, KIND>(u, cnt, op, lay, vec, scr_f, scr_b);
        if (pa.g) add_chunk_from<L>(pa.g + (b * m + j - 1) * nxl, base, cnt, u);
        add_chunk_into<L>(pa.parent + (b * m + j) * nxl, base, cnt, u);
      }
      if (b == pa.nint - 1) {
        load_chunk<L>(pa.cin + pa.nint * nxl, base, cnt, u);
        add_chunk_into<L>(pa.parent + (pa.nint * m) * nxl, base, cnt, u);
      }
      break;
    }
    case MODE_FINAL_F: {
      load_chunk<L>(pa.cin + b * nxl, base, cnt, u);
      store_chunk<L>(pa.out + (b * m) * nxl, base, cnt, u);
      for (int j = 1; j < m; ++j) {
        apply_step<L, KIND>(u, cnt, op, lay, vec, scr_f, scr_b);
        store_chunk<L>(pa.out + (b * m + j) * nxl, base, cnt, u);
      }
      if (b == pa.nint - 1) {
        load_chunk<L>(pa.cin + pa.nint * nxl, base, cnt, u);
        store_chunk<L>(pa.out + (pa.nint * m) * nxl, base, cnt, u);
      }
      break;
    }
    case MODE_SEQ: {
      if (pa.zero_init) {
#pragma unroll
        for (int j = 0; j < L; ++j) u[j] = 0.0;
      } else {
        load_chunk<L>(pa.cin, base, cnt, u);
      }
      if (pa.out) store_chunk<L>(pa.out, base, cnt, u);
      for (int n = 1; n <= m; ++n) {
        apply_step<L, KIND>(u, cnt, op, lay, vec, scr_f, scr_b);
        if (pa.g) add_chunk_from<L>(pa.g + (int64_t)(n - 1) * nxl, base, cnt, u);
        if (pa.parent) add_chunk_into<L>(pa.parent + (int64_t)n * nxl, base, cnt, u);
        if (pa.out) store_chunk<L>(pa.out + (int64_t)n * nxl, base, cnt, u);
      }
      break;
    }
    case MODE_APPLY: {
      load_chunk<L>(pa.cin + b * nxl, base, cnt, u);
      for (int j = 0; j < m; ++j) apply_step<L, KIND>(u, cnt, op, lay, vec, scr_f, scr_b);
      __syncthreads();  // in-place use: every thread has read its input row
      store_chunk<L>(pa.cout + b * nxl, base, cnt, u);
      break;
    }
    case MODE_RESID: {
      load_chunk<L>(pa.cin + b * nxl, base, cnt, u);
      apply_step<L, KIND>(u, cnt, op, lay, vec, scr_f, scr_b);
      const double *__restrict__ c1 = pa.cin + (b + 1) * nxl;
      double ss = 0.0;
#pragma unroll
      for (int j = 0; j < L; ++j) {
        if (j < cnt) {
          u[j] -= c1[base + j];
          ss = fma(u[j], u[j], ss);
        }
      }
      if (pa.r) store_chunk<L>(pa.r + b * nxl, base, cnt, u);
      const double tot = block_sum(ss, red);
      if (tid == 0) pa.normpart[b] = tot;
      break;
    }
    default:
      break;
  }
}

__global__ void __launch_bounds__(256) reduce_kernel(const double *__restrict__ part, int64_t n,
                                                      double *__restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if (threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
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

__global__ void fill_kernel(double *__restrict__ dst, int64_t n, double value) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = value;
}

}  // namespace

size_t lds_bytes_for(const Layout &lay) {
  const size_t doubles = (size_t)(lay.nx + (lay.nx >> 4) + 1) + 2 * SCR + MAXWAVES;
  return doubles * sizeof(double);
}

namespace {

template <int L, int KIND>
hipError_t set_lds(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)step_kernel<L, KIND, 256>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e) return e;
  return hipFuncSetAttribute((const void *)step_kernel<L, KIND, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <int KIND>
hipError_t set_lds_all(size_t bytes) {
  hipError_t e;
  if ((e = set_lds<1, KIND>(bytes))) return e;
  if ((e = set_lds<2, KIND>(bytes))) return e;
  if ((e = set_lds<4, KIND>(bytes))) return e;
  if ((e = set_lds<8, KIND>(bytes))) return e;
  return set_lds<16, KIND>(bytes);
}

template <int L, int KIND>
void launch_l(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, hipStream_t stream) {
  const dim3 grid((unsigned)pa.nint);
  const dim3 block((unsigned)lay.T);
  const size_t lds = lds_bytes_for(lay);
  if (lay.T <= 256)
    hipLaunchKernelGGL((step_kernel<L, KIND, 256>), grid, block, lds, stream, desc, pa);
  else
    hipLaunchKernelGGL((step_kernel<L, KIND, 1024>), grid, block, lds, stream, desc, pa);
}

template <int KIND>
hipError_t launch_kind(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, hipStream_t stream) {
  if (lay.T < WAVE || lay.T > 1024 || lay.T % WAVE) return hipErrorInvalidValue;
  switch (lay.L) {
    case 1: launch_l<1, KIND>(desc, lay, pa, stream); break;
    case 2: launch_l<2, KIND>(desc, lay, pa, stream); break;
    case 4: launch_l<4, KIND>(desc, lay, pa, stream); break;
    case 8: launch_l<8, KIND>(desc, lay, pa, stream); break;
    case 16: launch_l<16, KIND>(desc, lay, pa, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t configure_kernels(size_t bytes) {
  hipError_t e;
  if ((e = set_lds_all<OP_POLY_Z>(bytes))) return e;
  if ((e = set_lds_all<OP_POLY_W>(bytes))) return e;
  return set_lds_all<OP_SLC>(bytes);
}

hipError_t launch_pass(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs &pa,
                       hipStream_t stream) {
  if (pa.nint <= 0) return hipSuccess;
  switch (op.kind) {
    case OP_POLY_Z: return launch_kind<OP_POLY_Z>(desc, lay, pa, stream);
    case OP_POLY_W: return launch_kind<OP_POLY_W>(desc, lay, pa, stream);
    case OP_SLC: return launch_kind<OP_SLC>(desc, lay, pa, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce(const double *part, int64_t n, double *out, hipStream_t stream) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, stream, part, n, out);
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

hipError_t launch_fill(double *dst, int64_t n, double value, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, stream, dst, n, value);
  return hipGetLastError();
}

}  // namespace mgrit
