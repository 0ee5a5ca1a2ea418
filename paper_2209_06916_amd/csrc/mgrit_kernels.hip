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
// constant transfer matrix H = M^L (M the companion matrix), one thread that
// folds the wavefront totals and the closed-form periodic wrap
// s_0 = W (H_last E_{A-1} + q_{A-1}) into per-wavefront carries, and a
// homogeneous correction pass.  Everything the scan reads (powers of H, the
// wrap matrix) is staged in LDS once per launch; operator coefficients are
// held in registers.  No MFMA: nothing here is a dense contraction.
#include "mgrit_internal.h"

namespace mgrit {

namespace {

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
  if (cnt == L) {
#pragma unroll
    for (int j = 0; j < L; ++j) x[j] = row[base + j];
  } else {
#pragma unroll
    for (int j = 0; j < L; ++j) x[j] = (j < cnt) ? row[base + j] : 0.0;
  }
}

template <int L>
__device__ __forceinline__ void store_chunk(double *__restrict__ row, int base, int cnt, const double (&x)[L]) {
  if (cnt == L) {
#pragma unroll
    for (int j = 0; j < L; ++j) row[base + j] = x[j];
  } else {
#pragma unroll
    for (int j = 0; j < L; ++j)
      if (j < cnt) row[base + j] = x[j];
  }
}

template <int L>
__device__ __forceinline__ void chunk_to_lds(double *vec, int base, int cnt, const double (&x)[L]) {
  if (cnt == L) {
#pragma unroll
    for (int j = 0; j < L; ++j) vec[padix(base + j)] = x[j];
  } else {
#pragma unroll
    for (int j = 0; j < L; ++j)
      if (j < cnt) vec[padix(base + j)] = x[j];
  }
}

// out[j] += w[0] * v[start+j] + ... + w[width-1] * v[start+j+width-1]
// (indices periodic), reading the padded LDS copy v; 0 <= start < nx.  Each
// LDS value is read once and scattered into the outputs it feeds.  Full
// chunks whose window does not wrap take a branch-free path.
template <int L>
__device__ __forceinline__ void window_combine(const double *vec, int start, int cnt, int width, int nx,
                                               const double (&w)[MAXTAPS], double (&out)[L]) {
  if (cnt == L && start + L + width - 1 <= nx) {
#pragma unroll
    for (int e = 0; e < L + MAXTAPS - 1; ++e) {
      if (e < L + width - 1) {  // uniform
        const double v = vec[padix(start + e)];
#pragma unroll
        for (int t = 0; t < MAXTAPS; ++t) {
          const int j = e - t;
          if (j >= 0 && j < L && t < width) out[j] = fma(w[t], v, out[j]);
        }
      }
    }
    return;
  }
  int idx = start;
#pragma unroll
  for (int e = 0; e < L + MAXTAPS - 1; ++e) {
    if (e < cnt + width - 1) {
      const double v = vec[padix(idx)];
#pragma unroll
      for (int t = 0; t < MAXTAPS; ++t) {
        const int j = e - t;
        if (j >= 0 && j < L && t < width) out[j] = fma(w[t], v, out[j]);
      }
      idx = wrap_hi(idx + 1, nx);
    }
  }
}

template <int K>
__device__ __forceinline__ void matvec_add(const double *H, const double (&x)[K], double (&acc)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double s = acc[i];
#pragma unroll
    for (int j = 0; j < K; ++j) s = fma(H[i * K + j], x[j], s);
    acc[i] = s;
  }
}

// Periodic recurrence over the workgroup.  x holds this thread's chunk (REV:
// register j is processed as element L-1-j: the backward recurrence over the
// same chunks in reversed thread order).  vt: this thread's position in
// processing order; A: threads owning points; tab: LDS copy of
// [Hpow[0..64], Hlast, Wwrap] (K*K each); scr: LDS scratch of 2*MAXWAVES*K.
template <int L, int K, bool REV>
__device__ __forceinline__ void recurrence(double (&x)[L], int cnt, int vt, int A, int T, const double (&ain)[KMAX],
                                           const double *tab, double *scr) {
  constexpr int KK = K * K;
  double a[K];
#pragma unroll
  for (int m = 0; m < K; ++m) a[m] = ain[m];

  // 1. zero-state pass over the chunk (branch-free when the chunk is full)
  const bool full = (cnt == L);
  double s[K];
#pragma unroll
  for (int m = 0; m < K; ++m) s[m] = 0.0;
#pragma unroll
  for (int e = 0; e < L; ++e) {
    const int j = REV ? (L - 1 - e) : e;
    double y = x[j];
#pragma unroll
    for (int m = 0; m < K; ++m) y = fma(a[m], s[m], y);
    const bool on = full || e < cnt;
#pragma unroll
    for (int m = K - 1; m > 0; --m) s[m] = on ? s[m - 1] : s[m];
    s[0] = on ? y : s[0];
    x[j] = on ? y : x[j];
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
    double t[K];
#pragma unroll
    for (int m = 0; m < K; ++m) t[m] = inc[m];
    matvec_add<K>(tab + d * KK, o, t);
    const bool take = vl >= d;
#pragma unroll
    for (int m = 0; m < K; ++m) inc[m] = take ? t[m] : inc[m];
  }
  // exclusive value within the wavefront
  double ex[K];
  {
    const int src = (REV ? (lane + 1) : (lane - 1)) & (WAVE - 1);
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const double o = __shfl(inc[m], src, WAVE);
      ex[m] = (vl >= 1) ? o : 0.0;
    }
  }

  // 3. wavefront totals -> LDS
  double *Q = scr;
  double *Xc = scr + MAXWAVES * K;
  if (vl == WAVE - 1) {
#pragma unroll
    for (int m = 0; m < K; ++m) Q[vw * K + m] = inc[m];
  }
  __syncthreads();

  // 4. one thread: carry into its wavefront, the periodic wrap s_0, and the
  //    carries X'_w (with s_0 folded in) of every wavefront
  if (vt == A - 1) {
    const double *H64 = tab + WAVE * KK;
    const double *Hlast = tab + (WAVE + 1) * KK;
    const double *Wwrap = tab + (WAVE + 2) * KK;
    double X[K];
#pragma unroll
    for (int m = 0; m < K; ++m) X[m] = 0.0;
    for (int w2 = 0; w2 < vw; ++w2) {
      double nx_[K];
#pragma unroll
      for (int m = 0; m < K; ++m) nx_[m] = Q[w2 * K + m];
      matvec_add<K>(H64, X, nx_);
#pragma unroll
      for (int m = 0; m < K; ++m) X[m] = nx_[m];
    }
    double E[K];
#pragma unroll
    for (int m = 0; m < K; ++m) E[m] = ex[m];
    matvec_add<K>(tab + vl * KK, X, E);
    double tq[K];
#pragma unroll
    for (int m = 0; m < K; ++m) tq[m] = s[m];
    matvec_add<K>(Hlast, E, tq);
    double xp[K];
#pragma unroll
    for (int m = 0; m < K; ++m) xp[m] = 0.0;
    matvec_add<K>(Wwrap, tq, xp);  // s_0
#pragma unroll
    for (int m = 0; m < K; ++m) Xc[m] = xp[m];
    for (int w2 = 0; w2 + 1 < nw; ++w2) {
      double nx_[K];
#pragma unroll
      for (int m = 0; m < K; ++m) nx_[m] = Q[w2 * K + m];
      matvec_add<K>(H64, xp, nx_);
#pragma unroll
      for (int m = 0; m < K; ++m) {
        xp[m] = nx_[m];
        Xc[(w2 + 1) * K + m] = nx_[m];
      }
    }
  }
  __syncthreads();

  // 5. state entering this chunk, 6. homogeneous correction
  {
    double xc[K];
#pragma unroll
    for (int m = 0; m < K; ++m) xc[m] = Xc[vw * K + m];
    double st[K];
#pragma unroll
    for (int m = 0; m < K; ++m) st[m] = ex[m];
    matvec_add<K>(tab + vl * KK, xc, st);
#pragma unroll
    for (int e = 0; e < L; ++e) {
      const int j = REV ? (L - 1 - e) : e;
      double hv = 0.0;
#pragma unroll
      for (int m = 0; m < K; ++m) hv = fma(a[m], st[m], hv);
#pragma unroll
      for (int m = K - 1; m > 0; --m) st[m] = st[m - 1];
      st[0] = hv;
      x[j] = (full || e < cnt) ? x[j] + hv : x[j];
    }
  }
}

template <int L, bool REV>
__device__ __forceinline__ void recurrence_k(double (&x)[L], int cnt, int vt, int A, int T, int k,
                                             const double (&a)[KMAX], const double *tab, double *scr) {
  switch (k) {
    case 1: recurrence<L, 1, REV>(x, cnt, vt, A, T, a, tab, scr); break;
    case 2: recurrence<L, 2, REV>(x, cnt, vt, A, T, a, tab, scr); break;
    case 3: recurrence<L, 3, REV>(x, cnt, vt, A, T, a, tab, scr); break;
    default: break;
  }
}

// Operator constants held in registers for the whole launch.
struct OpRegs {
  int ncoef;
  const double *coef;  // Horner coefficients, read through the descriptor
  double top;          // coef[ncoef - 1]
  int width;  // stencil (OP_POLY_Z) or interpolation (OP_SLC) taps
  int off;    // OP_POLY_Z: st_l; OP_SLC: sl_K + sl_l
  double w[MAXTAPS];
  int has_solve, kf, kb;
  double cinv;
  double af[KMAX], ab[KMAX];
  int repeat;
};

// LDS regions of one launch.
struct Lds {
  double *vec0, *vec1;   // padded vectors (vec1 == vec0 unless double-buffered)
  double *tab_f, *tab_b; // recurrence tables
  double *scr_f, *scr_b; // recurrence scratch
  double *red;           // reduction scratch
};

// y <- T^{-1} y
template <int L>
__device__ __forceinline__ void solve(double (&y)[L], int cnt, const OpRegs &R, const Layout &lay, const Lds &S) {
  const int tid = threadIdx.x;
  const int nx = lay.nx;
  if (R.kf > 0) recurrence_k<L, false>(y, cnt, tid, lay.A, lay.T, R.kf, R.af, S.tab_f, S.scr_f);
  if (R.kb > 0) {
    if (!lay.ragged) {
      recurrence_k<L, true>(y, cnt, lay.T - 1 - tid, lay.A, lay.T, R.kb, R.ab, S.tab_b, S.scr_b);
    } else {
      // redistribute so that thread t owns indices nx-1-(tL+j), j = 0..cnt-1
      double *vec = S.vec0;
      const int base = tid * L;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (j < cnt) vec[padix(base + j)] = y[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = (j < cnt) ? vec[padix(nx - 1 - (base + j))] : 0.0;
      recurrence_k<L, false>(y, cnt, tid, lay.A, lay.T, R.kb, R.ab, S.tab_b, S.scr_b);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (j < cnt) vec[padix(nx - 1 - (base + j))] = y[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = (j < cnt) ? vec[padix(base + j)] : 0.0;
    }
  }
  const double ci = R.cinv;
#pragma unroll
  for (int j = 0; j < L; ++j) y[j] *= ci;
}

// coef[i] (uniform scalar load through the descriptor)
__device__ __forceinline__ double coef_at(const OpRegs &R, int i) { return R.coef[i]; }

// u <- Phi u  (every thread of the workgroup must call this).  buf: which
// LDS vector the next explicit stencil writes (double-buffered layouts).
template <int L, int KIND>
__device__ __forceinline__ void apply_step(double (&u)[L], int cnt, const OpRegs &R, const Layout &lay,
                                           const Lds &S, int &buf) {
  const int nx = lay.nx;
  const int base = threadIdx.x * L;
  double y[L];
  for (int rep = 0; rep < R.repeat; ++rep) {
    if (KIND == OP_SLC) {
      __syncthreads();
      chunk_to_lds<L>(S.vec0, base, cnt, u);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = 0.0;
      window_combine<L>(S.vec0, wrap_lo(base - R.off, nx), cnt, R.width, nx, R.w, y);
      if (R.has_solve) solve<L>(y, cnt, R, lay, S);
#pragma unroll
      for (int j = 0; j < L; ++j) u[j] = y[j];
    } else if (KIND == OP_POLY_Z) {
      const int start = wrap_lo(base - R.off, nx);
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = R.top * u[j];
      for (int i = R.ncoef - 2; i >= 0; --i) {
        double *v = buf ? S.vec1 : S.vec0;
        if (!lay.dbuf) __syncthreads();
        chunk_to_lds<L>(v, base, cnt, y);
        __syncthreads();
        const double ci = coef_at(R, i);
#pragma unroll
        for (int j = 0; j < L; ++j) y[j] = ci * u[j];
        window_combine<L>(v, start, cnt, R.width, nx, R.w, y);
        buf ^= lay.dbuf;
      }
#pragma unroll
      for (int j = 0; j < L; ++j) u[j] = y[j];
    } else {  // OP_POLY_W
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = R.top * u[j];
      for (int i = R.ncoef - 2; i >= 0; --i) {
        solve<L>(y, cnt, R, lay, S);
        const double ci = coef_at(R, i);
#pragma unroll
        for (int j = 0; j < L; ++j) y[j] = fma(ci, u[j], y[j]);
      }
#pragma unroll
      for (int j = 0; j < L; ++j) u[j] = y[j];
    }
  }
}

// Sum over the workgroup, deterministic order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *red) {
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

// The chain of time steps of one pass (see PassMode): load the start vector,
// advance it step by step with step(u) (all threads together), and do the
// mode's per-step and final memory work.  cnt: points of this thread.
template <int L, class Step>
__device__ __forceinline__ void run_chain(const PassArgs &pa, int nx, int cnt, double *red, Step step) {
  const int tid = threadIdx.x;
  const int base = tid * L;
  const int64_t b = blockIdx.x;
  const int64_t nxl = nx;
  const int m = pa.m;
  const int mode = pa.mode;
  double u[L];

  int nsteps;
  switch (mode) {
    case MODE_PASS_A: nsteps = m; break;
    case MODE_PASS_B: nsteps = m; break;
    case MODE_POST_F: nsteps = m - 1; break;
    case MODE_FINAL_F: nsteps = m - 1; break;
    case MODE_SEQ: nsteps = m; break;
    case MODE_APPLY: nsteps = m; break;
    default: nsteps = 1; break;  // MODE_RESID
  }
  const int64_t row0 = (mode == MODE_SEQ) ? 0 : b;
  if (pa.zero_init) {
#pragma unroll
    for (int j = 0; j < L; ++j) u[j] = 0.0;
  } else {
    load_chunk<L>(pa.cin + row0 * nxl, base, cnt, u);
  }
  if (mode == MODE_PASS_A && b == 0) store_chunk<L>(pa.cout, base, cnt, u);
  if (mode == MODE_FINAL_F) store_chunk<L>(pa.out + (b * m) * nxl, base, cnt, u);
  if (mode == MODE_SEQ && pa.out) store_chunk<L>(pa.out, base, cnt, u);
  const bool add_g = pa.g && mode != MODE_APPLY && mode != MODE_RESID && mode != MODE_FINAL_F;
  const bool add_parent = mode == MODE_POST_F || (mode == MODE_SEQ && pa.parent);
  const bool store_out = mode == MODE_FINAL_F || (mode == MODE_SEQ && pa.out);
  if (mode == MODE_POST_F) {
    double pv[L];
    load_chunk<L>(pa.parent + (b * m) * nxl, base, cnt, pv);
#pragma unroll
    for (int j = 0; j < L; ++j) pv[j] += u[j];
    store_chunk<L>(pa.parent + (b * m) * nxl, base, cnt, pv);
  }

  // the chain of time steps (single call site of the step); for short chunks
  // the rows this step adds are loaded before the step so their latency
  // overlaps it
  constexpr bool PREFETCH = L <= 16;
  for (int j = 1; j <= nsteps; ++j) {
    const int64_t n = (mode == MODE_SEQ) ? (int64_t)j : b * m + j;  // level point index
    double gv[PREFETCH ? L : 1], pv[PREFETCH ? L : 1];
    if (PREFETCH) {
      if (add_g) load_chunk<PREFETCH ? L : 1>(pa.g + (n - 1) * nxl, base, cnt, gv);
      if (add_parent) load_chunk<PREFETCH ? L : 1>(pa.parent + n * nxl, base, cnt, pv);
    }
    step(u);
    if (add_g) {
      if (PREFETCH) {
#pragma unroll
        for (int q = 0; q < (PREFETCH ? L : 1); ++q) u[q] += gv[q];
      } else {
        const double *gr = pa.g + (n - 1) * nxl + base;
#pragma unroll
        for (int q = 0; q < L; ++q)
          if (q < cnt) u[q] += gr[q];
      }
    }
    if (add_parent) {
      double *pr = pa.parent + n * nxl + base;
      if (PREFETCH) {
#pragma unroll
        for (int q = 0; q < (PREFETCH ? L : 1); ++q) pv[q] += u[q];
        store_chunk<PREFETCH ? L : 1>(pa.parent + n * nxl, base, cnt, pv);
      } else {
#pragma unroll
        for (int q = 0; q < L; ++q)
          if (q < cnt) pr[q] += u[q];
      }
    }
    if (store_out) store_chunk<L>(pa.out + n * nxl, base, cnt, u);
  }

  // post-chain actions
  if (mode == MODE_PASS_A) {
    store_chunk<L>(pa.cout + (b + 1) * nxl, base, cnt, u);
  } else if (mode == MODE_PASS_B || mode == MODE_RESID) {
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
  } else if (mode == MODE_POST_F || mode == MODE_FINAL_F) {
    if (b == pa.nint - 1) {
      load_chunk<L>(pa.cin + pa.nint * nxl, base, cnt, u);
      double *row = (mode == MODE_POST_F ? pa.parent : pa.out) + (pa.nint * m) * nxl;
      if (mode == MODE_POST_F) {
        double pv[L];
        load_chunk<L>(row, base, cnt, pv);
#pragma unroll
        for (int j = 0; j < L; ++j) u[j] += pv[j];
      }
      store_chunk<L>(row, base, cnt, u);
    }
  } else if (mode == MODE_APPLY) {
    __syncthreads();  // in-place use: every thread has read its input row
    store_chunk<L>(pa.cout + b * nxl, base, cnt, u);
  }
}

template <int L, int KIND, int MAXT>
__global__ void __launch_bounds__(MAXT) step_kernel(const LevelDesc *__restrict__ desc, PassArgs pa) {
  extern __shared__ double smem[];
  const Layout lay = desc->lay;
  const StepOp &op = desc->op;
  const int nx = lay.nx;
  const LdsOffsets lo = lds_offsets(lay, op.has_solve);
  Lds S;
  S.vec0 = smem;
  S.vec1 = smem + lo.vec1;
  S.tab_f = smem + lo.tab_f;
  S.tab_b = smem + lo.tab_b;
  S.scr_f = smem + lo.scr_f;
  S.scr_b = smem + lo.scr_b;
  S.red = smem + lo.red;

  // operator constants -> registers
  OpRegs R;
  R.repeat = op.repeat;
  R.ncoef = op.ncoef;
  R.coef = op.coef;
  R.top = op.coef[op.ncoef - 1];
  if (KIND == OP_SLC) {
    R.width = op.sl_l + op.sl_r + 1;
    R.off = op.sl_K + op.sl_l;
#pragma unroll
    for (int t = 0; t < MAXTAPS; ++t) R.w[t] = op.slw[t];
  } else {
    R.width = op.st_l + op.st_r + 1;
    R.off = op.st_l;
#pragma unroll
    for (int t = 0; t < MAXTAPS; ++t) R.w[t] = op.taps[t];
  }
  R.has_solve = op.has_solve;
  R.kf = op.fw.k;
  R.kb = op.bw.k;
  R.cinv = op.cinv;
#pragma unroll
  for (int m = 0; m < KMAX; ++m) {
    R.af[m] = op.fw.a[m];
    R.ab[m] = op.bw.a[m];
  }
  // recurrence tables -> LDS
  if (KIND != OP_POLY_Z && R.has_solve) {
    const int nf = R.kf * R.kf * RTAB, nb = R.kb * R.kb * RTAB;
    for (int i = threadIdx.x; i < nf; i += blockDim.x) S.tab_f[i] = op.fw.tab[i];
    for (int i = threadIdx.x; i < nb; i += blockDim.x) S.tab_b[i] = op.bw.tab[i];
  }
  __syncthreads();

  const int tid = threadIdx.x;
  const int cnt = min(max(nx - tid * L, 0), L);
  int buf = 0;
  run_chain<L>(pa, nx, cnt, S.red, [&](double (&u)[L]) { apply_step<L, KIND>(u, cnt, R, lay, S, buf); });
}

// ---------------------------------------------------------------------------
// Level-0 explicit relaxation, one wavefront per (CF-interval, spatial tile).
// Lane l holds the P consecutive points starting at x0 - HL + l P (periodic).
// Each application of Z = -c L_p reads SL points from the left neighbour lane
// and SR from the right one; lane 0's left and lane 63's right inputs are
// stale, which only invalidates points inside the halo.  No LDS, no barriers.
// ---------------------------------------------------------------------------
template <int P, int SL, int SR>
__global__ void __launch_bounds__(256) tile_kernel(const LevelDesc *__restrict__ desc, TileGeom tg, TileArgs ta) {
  const StepOp &op = desc->op;
  const int nx = desc->lay.nx;
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (item >= ta.nint * tg.ntiles) return;  // whole wavefront leaves together
  const int64_t b = item / tg.ntiles;
  const int tau = (int)(item - b * tg.ntiles);
  const int x0 = tau * tg.TW;
  const int tw = min(tg.TW, nx - x0);
  const int64_t nxl = nx;

  // coefficients -> registers
  const int ncoef = op.ncoef;
  double taps[SL + SR + 1];
#pragma unroll
  for (int t = 0; t <= SL + SR; ++t) taps[t] = op.taps[t];
  const double top = op.coef[ncoef - 1];

  // this lane's first global position (periodic) and its local index
  const int li0 = lane * P;              // local index of point 0 of this lane
  int g0 = x0 - tg.HL + li0;             // global position, may be outside [0, nx)
  g0 %= nx;
  if (g0 < 0) g0 += nx;

  double u[P];
  {
    const double *row = ta.cin + b * nxl;
    int g = g0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      u[k] = row[g];
      g = wrap_hi(g + 1, nx);
    }
  }
  // output window of this lane: local indices [HL, HL + tw)
  const int lo = tg.HL - li0, hi = tg.HL + tw - li0;  // k in [lo, hi) is output

  auto store_out = [&](double *row, const double (&v)[P]) {
    int g = g0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      if (k >= lo && k < hi) row[g] = v[k];
      g = wrap_hi(g + 1, nx);
    }
  };

  if (ta.mode == MODE_PASS_A && b == 0) store_out(ta.cout, u);
  if (ta.mode == MODE_FINAL_F) store_out(ta.out + (b * ta.m) * nxl, u);

  const int nsteps = (ta.mode == MODE_FINAL_F) ? ta.m - 1 : ta.m;
  for (int j = 1; j <= nsteps; ++j) {
    double y[P];
#pragma unroll
    for (int k = 0; k < P; ++k) y[k] = top * u[k];
    for (int i = ncoef - 2; i >= 0; --i) {
      double lh[SL > 0 ? SL : 1], rh[SR > 0 ? SR : 1];
#pragma unroll
      for (int q = 0; q < SL; ++q) lh[q] = __shfl(y[P - SL + q], (lane - 1) & (WAVE - 1), WAVE);
#pragma unroll
      for (int q = 0; q < SR; ++q) rh[q] = __shfl(y[q], (lane + 1) & (WAVE - 1), WAVE);
      const double ci = op.coef[i];
      double yn[P];
#pragma unroll
      for (int k = 0; k < P; ++k) {
        double acc = ci * u[k];
#pragma unroll
        for (int t = 0; t <= SL + SR; ++t) {
          const int src = k + t - SL;
          const double v = src < 0 ? lh[(src + SL) < 0 ? 0 : (src + SL)]
                                   : (src >= P ? rh[(src - P) < SR ? (src - P) : 0] : y[src < P ? src : 0]);
          acc = fma(taps[t], v, acc);
        }
        yn[k] = acc;
      }
#pragma unroll
      for (int k = 0; k < P; ++k) y[k] = yn[k];
    }
#pragma unroll
    for (int k = 0; k < P; ++k) u[k] = y[k];
    if (ta.mode == MODE_FINAL_F) store_out(ta.out + (b * ta.m + j) * nxl, u);
  }

  if (ta.mode == MODE_PASS_A) {
    store_out(ta.cout + (b + 1) * nxl, u);
  } else if (ta.mode == MODE_PASS_B) {
    const double *c1 = ta.cin + (b + 1) * nxl;
    double ss = 0.0;
    int g = g0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      if (k >= lo && k < hi) {
        const double rv = u[k] - c1[g];
        ta.r[b * nxl + g] = rv;
        ss = fma(rv, rv, ss);
      }
      g = wrap_hi(g + 1, nx);
    }
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) ss += __shfl_down(ss, d, WAVE);
    if (lane == 0) ta.normpart[item] = ss;
  } else if (ta.mode == MODE_FINAL_F && b == ta.nint - 1) {
    double c[P];
    const double *row = ta.cin + ta.nint * nxl;
    int g = g0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      c[k] = row[g];
      g = wrap_hi(g + 1, nx);
    }
    store_out(ta.out + (ta.nint * ta.m) * nxl, c);
  }
}

template <int P>
hipError_t launch_tiles_p(const LevelDesc *desc, const TileGeom &tg, const TileArgs &ta, hipStream_t stream) {
  const int64_t items = ta.nint * tg.ntiles;
  const dim3 grid((unsigned)((items + 3) / 4)), block(256);
  switch (tg.sl * 4 + tg.sr) {
    case 1 * 4 + 0: hipLaunchKernelGGL((tile_kernel<P, 1, 0>), grid, block, 0, stream, desc, tg, ta); break;
    case 2 * 4 + 0: hipLaunchKernelGGL((tile_kernel<P, 2, 0>), grid, block, 0, stream, desc, tg, ta); break;
    case 2 * 4 + 1: hipLaunchKernelGGL((tile_kernel<P, 2, 1>), grid, block, 0, stream, desc, tg, ta); break;
    case 3 * 4 + 1: hipLaunchKernelGGL((tile_kernel<P, 3, 1>), grid, block, 0, stream, desc, tg, ta); break;
    case 3 * 4 + 2: hipLaunchKernelGGL((tile_kernel<P, 3, 2>), grid, block, 0, stream, desc, tg, ta); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Coarse time step Psi = T^{-1} S on full chunks (nx = T L, T a multiple of
// 64): W interpolation taps, order-K forward and backward recurrences.  One
// barrier per recurrence: after the wavefront totals are published, every
// wavefront folds them and the periodic wrap into its own carry (the same
// short chain, computed redundantly), so no thread waits for a serial one.
// ---------------------------------------------------------------------------
// Cross-lane move of a double with a DPP row shift (bound_ctrl: lanes whose
// source lies outside their 16-lane row read 0).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffff), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffff), lane);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// One Kogge-Stone step inside 16-lane rows: take the state D lanes back in
// processing order (row_shr for the forward direction, row_shl backward).
template <int K, bool REV, int D>
__device__ __forceinline__ void row_scan_step(double (&inc)[K], const double *tab, int lr) {
  constexpr int KK = K * K;
  double o[K], t[K];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    o[m] = REV ? dpp_d<0x100 + D>(inc[m]) : dpp_d<0x110 + D>(inc[m]);
    t[m] = inc[m];
  }
  matvec_add<K>(tab + D * KK, o, t);
  const bool take = lr >= D;
#pragma unroll
  for (int m = 0; m < K; ++m) inc[m] = take ? t[m] : inc[m];
}

template <int L, int K, bool REV, class Hook>
__device__ __forceinline__ void lean_recurrence(double (&x)[L], int vt, int T, const double (&a)[K],
                                                const double *tab, double *Q, Hook pre_barrier) {
  constexpr int KK = K * K;
  constexpr int LH = L / 2;  // two interleaved sub-chains per lane
  const double *Hhalf = tab + (WAVE + 3) * KK;
  // zero-state passes of both halves (processing order: REV walks down)
  double sa[K], sb[K];
#pragma unroll
  for (int m = 0; m < K; ++m) sa[m] = sb[m] = 0.0;
#pragma unroll
  for (int e = 0; e < LH; ++e) {
    const int ja = REV ? (L - 1 - e) : e;
    const int jb = REV ? (LH - 1 - e) : (LH + e);
    double ya = x[ja], yb = x[jb];
#pragma unroll
    for (int m = 0; m < K; ++m) {
      ya = fma(a[m], sa[m], ya);
      yb = fma(a[m], sb[m], yb);
    }
#pragma unroll
    for (int m = K - 1; m > 0; --m) {
      sa[m] = sa[m - 1];
      sb[m] = sb[m - 1];
    }
    sa[0] = ya;
    sb[0] = yb;
    x[ja] = ya;
    x[jb] = yb;
  }
  // chunk total q = Hhalf sa + sb
  double q[K];
#pragma unroll
  for (int m = 0; m < K; ++m) q[m] = sb[m];
  matvec_add<K>(Hhalf, sa, q);

  // scan inside 16-lane rows (DPP), then fold the row totals (readlane)
  const int lane = threadIdx.x & (WAVE - 1);
  const int nw = T >> 6;
  const int vl = REV ? (WAVE - 1 - lane) : lane;
  const int vw = vt >> 6;
  const int lr = vl & 15, vrow = vl >> 4;
  double inc[K];
#pragma unroll
  for (int m = 0; m < K; ++m) inc[m] = q[m];
  row_scan_step<K, REV, 1>(inc, tab, lr);
  row_scan_step<K, REV, 2>(inc, tab, lr);
  row_scan_step<K, REV, 4>(inc, tab, lr);
  row_scan_step<K, REV, 8>(inc, tab, lr);
  double exr[K];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    const double o = REV ? dpp_d<0x101>(inc[m]) : dpp_d<0x111>(inc[m]);
    exr[m] = lr >= 1 ? o : 0.0;
  }
  // row carries C_r (state entering virtual row r), uniform over the wavefront
  double C1[K], C2[K], C3[K];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    C1[m] = readlane_d(inc[m], REV ? 48 : 15);
    C2[m] = readlane_d(inc[m], REV ? 32 : 31);
    C3[m] = readlane_d(inc[m], REV ? 16 : 47);
  }
  const double *H16 = tab + 16 * KK;
  matvec_add<K>(H16, C1, C2);
  matvec_add<K>(H16, C2, C3);
  double cr[K];
#pragma unroll
  for (int m = 0; m < K; ++m) cr[m] = vrow == 0 ? 0.0 : (vrow == 1 ? C1[m] : (vrow == 2 ? C2[m] : C3[m]));
  // exclusive prefix within the wavefront: ex = exr + H^lr C_row
  double ex[K];
#pragma unroll
  for (int m = 0; m < K; ++m) ex[m] = exr[m];
  matvec_add<K>(tab + lr * KK, cr, ex);

  // publish: wavefront totals q + H ex (virtual lane 63), and the last
  // chunk's exclusive value and own zero-state total
  if (vl == WAVE - 1) {
    double tot[K];
#pragma unroll
    for (int m = 0; m < K; ++m) tot[m] = q[m];
    matvec_add<K>(tab + KK, ex, tot);
#pragma unroll
    for (int m = 0; m < K; ++m) Q[vw * K + m] = tot[m];
  }
  if (vt == T - 1) {
#pragma unroll
    for (int m = 0; m < K; ++m) {
      Q[MAXWAVES * K + m] = ex[m];
      Q[(MAXWAVES + 1) * K + m] = q[m];
    }
  }
  pre_barrier();
  __syncthreads();
  const double *H64 = tab + WAVE * KK;
  const double *Hlast = tab + (WAVE + 1) * KK;
  const double *Wwrap = tab + (WAVE + 2) * KK;
  double X[K];
#pragma unroll
  for (int m = 0; m < K; ++m) X[m] = 0.0;
#pragma unroll
  for (int w2 = 0; w2 < MAXWAVES - 1; ++w2) {
    if (w2 < nw - 1) {
      double nxt[K];
#pragma unroll
      for (int m = 0; m < K; ++m) nxt[m] = Q[w2 * K + m];
      matvec_add<K>(H64, X, nxt);
#pragma unroll
      for (int m = 0; m < K; ++m) X[m] = nxt[m];
    }
  }
  double E[K], tq[K], xp[K];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    E[m] = Q[MAXWAVES * K + m];
    tq[m] = Q[(MAXWAVES + 1) * K + m];
    xp[m] = 0.0;
  }
  matvec_add<K>(tab + (WAVE - 1) * KK, X, E);
  matvec_add<K>(Hlast, E, tq);
  matvec_add<K>(Wwrap, tq, xp);
#pragma unroll
  for (int w2 = 0; w2 < MAXWAVES - 1; ++w2) {
    if (w2 < vw) {
      double nxt[K];
#pragma unroll
      for (int m = 0; m < K; ++m) nxt[m] = Q[w2 * K + m];
      matvec_add<K>(H64, xp, nxt);
#pragma unroll
      for (int m = 0; m < K; ++m) xp[m] = nxt[m];
    }
  }
  // states entering the two halves, then the homogeneous corrections
  double ta[K], tb[K];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    ta[m] = ex[m];
    tb[m] = sa[m];
  }
  matvec_add<K>(tab + vl * KK, xp, ta);
  matvec_add<K>(Hhalf, ta, tb);
#pragma unroll
  for (int e = 0; e < LH; ++e) {
    const int ja = REV ? (L - 1 - e) : e;
    const int jb = REV ? (LH - 1 - e) : (LH + e);
    double ha = 0.0, hb = 0.0;
#pragma unroll
    for (int m = 0; m < K; ++m) {
      ha = fma(a[m], ta[m], ha);
      hb = fma(a[m], tb[m], hb);
    }
#pragma unroll
    for (int m = K - 1; m > 0; --m) {
      ta[m] = ta[m - 1];
      tb[m] = tb[m - 1];
    }
    ta[0] = ha;
    tb[0] = hb;
    x[ja] += ha;
    x[jb] += hb;
  }
}

// Coalesced row segments: thread t owns the 16-byte pairs t + T q, q < L/2.
template <int L>
__device__ __forceinline__ void load_segs(const double *__restrict__ row, int T, double2 (&seg)[L / 2]) {
  const double2 *r2 = reinterpret_cast<const double2 *>(row);
#pragma unroll
  for (int q = 0; q < L / 2; ++q) seg[q] = r2[threadIdx.x + T * q];
}

template <int L, int W, int K, int MAXT>
__global__ void __launch_bounds__(MAXT) slc_kernel(const LevelDesc *__restrict__ desc, PassArgs pa) {
  extern __shared__ double smem[];
  const int nx = desc->lay.nx;
  const int T = desc->lay.T;
  const int dbuf = desc->lay.dbuf;
  const StepOp &op = desc->op;
  const LeanLds lo = lean_lds_offsets(nx, dbuf, K);
  double *vec0 = smem;
  double *vec1 = smem + lo.vec1;
  double *gbuf = smem + lo.gbuf;
  double *tab_f = smem + lo.tab_f;
  double *tab_b = smem + lo.tab_b;
  double *qf = smem + lo.qf;
  double *qb = smem + lo.qb;
  double *red = smem + lo.red;

  double w[W], af[K], ab[K];
#pragma unroll
  for (int t = 0; t < W; ++t) w[t] = op.slw[t];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    af[m] = op.fw.a[m];
    ab[m] = op.bw.a[m];
  }
  const int off = op.sl_K + op.sl_l;
  const double cinv = op.cinv;
  for (int i = threadIdx.x; i < RTAB * K * K; i += blockDim.x) {
    tab_f[i] = op.fw.tab[i];
    tab_b[i] = op.bw.tab[i];
  }
  __syncthreads();

  const int tid = threadIdx.x;
  const int base = tid * L;
  int start = base - off;
  while (start < 0) start += nx;
  const int64_t b = blockIdx.x;
  const int64_t nxl = nx;
  const int m = pa.m;
  const int mode = pa.mode;
  int nsteps;
  switch (mode) {
    case MODE_POST_F: nsteps = m - 1; break;
    default: nsteps = m; break;  // PASS_A, PASS_B, SEQ, APPLY
  }
  const int64_t row0 = (mode == MODE_SEQ) ? 0 : b;
  double u[L];
  if (pa.zero_init) {
#pragma unroll
    for (int j = 0; j < L; ++j) u[j] = 0.0;
  } else {
    load_chunk<L>(pa.cin + row0 * nxl, base, L, u);
  }
  if (mode == MODE_PASS_A && b == 0) store_chunk<L>(pa.cout, base, L, u);
  const bool add_g = pa.g && mode != MODE_APPLY;
  const bool add_parent = mode == MODE_POST_F || (mode == MODE_SEQ && pa.parent);
  if (mode == MODE_POST_F) {
    double pv[L];
    load_chunk<L>(pa.parent + (b * m) * nxl, base, L, pv);
#pragma unroll
    for (int j = 0; j < L; ++j) pv[j] += u[j];
    store_chunk<L>(pa.parent + (b * m) * nxl, base, L, pv);
  }

  // parent[row] += (vector in v), coalesced, with the row's segments in pseg
  auto parent_update = [&](const double *v, int64_t prow, const double2 (&pseg)[L / 2]) {
    double2 *p2 = reinterpret_cast<double2 *>(pa.parent + prow * nxl);
#pragma unroll
    for (int q = 0; q < L / 2; ++q) {
      const int i = 2 * (tid + T * q);
      double2 r = pseg[q];
      r.x += v[padix(i)];
      r.y += v[padix(i + 1)];
      p2[tid + T * q] = r;
    }
  };

  int buf = 0;
  int64_t pend = -1;  // parent row whose update waits for the next LDS copy
  for (int j = 1; j <= nsteps; ++j) {
    const int64_t n = (mode == MODE_SEQ) ? (int64_t)j : b * m + j;  // level point index
    double2 gseg[L / 2], pseg[L / 2];
    if (add_g) load_segs<L>(pa.g + (n - 1) * nxl, T, gseg);
    if (pend >= 0) load_segs<L>(pa.parent + pend * nxl, T, pseg);
    double *v = buf ? vec1 : vec0;
    buf ^= dbuf;
    if (!dbuf) __syncthreads();
#pragma unroll
    for (int jj = 0; jj < L; ++jj) v[padix(base + jj)] = u[jj];
    __syncthreads();
    if (pend >= 0) parent_update(v, pend, pseg);
    double y[L];
#pragma unroll
    for (int jj = 0; jj < L; ++jj) y[jj] = 0.0;
#pragma unroll
    for (int e = 0; e < L + W - 1; ++e) {
      int idx = start + e;
      idx = idx >= nx ? idx - nx : idx;
      const double val = v[padix(idx)];
#pragma unroll
      for (int t = 0; t < W; ++t) {
        const int jj = e - t;
        if (jj >= 0 && jj < L) y[jj] = fma(w[t], val, y[jj]);
      }
    }
    lean_recurrence<L, K, false>(y, tid, T, af, tab_f, qf, [] {});
    lean_recurrence<L, K, true>(y, T - 1 - tid, T, ab, tab_b, qb, [&] {
      if (add_g) {
#pragma unroll
        for (int q = 0; q < L / 2; ++q) {
          const int i = 2 * (tid + T * q);
          gbuf[padix(i)] = gseg[q].x;
          gbuf[padix(i + 1)] = gseg[q].y;
        }
      }
    });
#pragma unroll
    for (int jj = 0; jj < L; ++jj) u[jj] = y[jj] * cinv;
    if (add_g) {
#pragma unroll
      for (int jj = 0; jj < L; ++jj) u[jj] += gbuf[padix(base + jj)];
    }
    pend = add_parent ? n : -1;
  }
  if (pend >= 0) {  // the last step's parent update
    double2 pseg[L / 2];
    load_segs<L>(pa.parent + pend * nxl, T, pseg);
    double *v = buf ? vec1 : vec0;
    __syncthreads();
#pragma unroll
    for (int jj = 0; jj < L; ++jj) v[padix(base + jj)] = u[jj];
    __syncthreads();
    parent_update(v, pend, pseg);
  }

  if (mode == MODE_PASS_A) {
    store_chunk<L>(pa.cout + (b + 1) * nxl, base, L, u);
  } else if (mode == MODE_PASS_B) {
    const double *__restrict__ c1 = pa.cin + (b + 1) * nxl;
    double ss = 0.0;
#pragma unroll
    for (int jj = 0; jj < L; ++jj) {
      u[jj] -= c1[base + jj];
      ss = fma(u[jj], u[jj], ss);
    }
    store_chunk<L>(pa.r + b * nxl, base, L, u);
    const double tot = block_sum(ss, red);
    if (tid == 0) pa.normpart[b] = tot;
  } else if (mode == MODE_POST_F) {
    if (b == pa.nint - 1) {
      load_chunk<L>(pa.cin + pa.nint * nxl, base, L, u);
      double *row = pa.parent + (pa.nint * m) * nxl;
      double pv[L];
      load_chunk<L>(row, base, L, pv);
#pragma unroll
      for (int jj = 0; jj < L; ++jj) u[jj] += pv[jj];
      store_chunk<L>(row, base, L, u);
    }
  } else if (mode == MODE_APPLY) {
    __syncthreads();  // in-place use: every thread has read its input row
    store_chunk<L>(pa.cout + b * nxl, base, L, u);
  }
}

template <int L, int W, int K>
hipError_t slc_launch(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, hipStream_t stream) {
  const size_t lds = (size_t)lean_lds_offsets(lay.nx, lay.dbuf, K).total * sizeof(double);
  const dim3 grid((unsigned)pa.nint), block((unsigned)lay.T);
  if (lay.T <= 256)
    hipLaunchKernelGGL((slc_kernel<L, W, K, 256>), grid, block, lds, stream, desc, pa);
  else
    hipLaunchKernelGGL((slc_kernel<L, W, K, 1024>), grid, block, lds, stream, desc, pa);
  return hipGetLastError();
}

template <int L, int W, int K>
hipError_t slc_set_lds(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)slc_kernel<L, W, K, 256>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e) return e;
  return hipFuncSetAttribute((const void *)slc_kernel<L, W, K, 1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <int L>
hipError_t slc_launch_l(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs &pa,
                        hipStream_t stream) {
  const int W = op.sl_l + op.sl_r + 1;
  if (W == 2 && op.fw.k == 1) return slc_launch<L, 2, 1>(desc, lay, pa, stream);
  if (W == 4 && op.fw.k == 2) return slc_launch<L, 4, 2>(desc, lay, pa, stream);
  if (W == 6 && op.fw.k == 3) return slc_launch<L, 6, 3>(desc, lay, pa, stream);
  return hipErrorInvalidValue;
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
  if ((e = set_lds<2, KIND>(bytes))) return e;
  if ((e = set_lds<4, KIND>(bytes))) return e;
  if ((e = set_lds<8, KIND>(bytes))) return e;
  return set_lds<16, KIND>(bytes);
}

template <int L, int KIND>
void launch_l(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, size_t lds, hipStream_t stream) {
  const dim3 grid((unsigned)pa.nint);
  const dim3 block((unsigned)lay.T);
  if (lay.T <= 256)
    hipLaunchKernelGGL((step_kernel<L, KIND, 256>), grid, block, lds, stream, desc, pa);
  else
    hipLaunchKernelGGL((step_kernel<L, KIND, 1024>), grid, block, lds, stream, desc, pa);
}

template <int KIND>
hipError_t launch_kind(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, size_t lds,
                       hipStream_t stream) {
  if (lay.T < WAVE || lay.T > 1024 || lay.T % WAVE) return hipErrorInvalidValue;
  switch (lay.L) {
    case 2: launch_l<2, KIND>(desc, lay, pa, lds, stream); break;
    case 4: launch_l<4, KIND>(desc, lay, pa, lds, stream); break;
    case 8: launch_l<8, KIND>(desc, lay, pa, lds, stream); break;
    case 16: launch_l<16, KIND>(desc, lay, pa, lds, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

size_t lds_bytes_for(const Layout &lay, int has_solve) {
  return (size_t)lds_offsets(lay, has_solve).total * sizeof(double);
}

hipError_t configure_kernels(size_t bytes) {
  hipError_t e;
#define MGRIT_SLC_SET(L)                                        \
  if ((e = slc_set_lds<L, 2, 1>(bytes))) return e;              \
  if ((e = slc_set_lds<L, 4, 2>(bytes))) return e;              \
  if ((e = slc_set_lds<L, 6, 3>(bytes))) return e;
  MGRIT_SLC_SET(4)
  MGRIT_SLC_SET(8)
  MGRIT_SLC_SET(16)
#undef MGRIT_SLC_SET
  if ((e = set_lds_all<OP_POLY_Z>(bytes))) return e;
  if ((e = set_lds_all<OP_POLY_W>(bytes))) return e;
  return set_lds_all<OP_SLC>(bytes);
}

hipError_t launch_pass(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs &pa,
                       hipStream_t stream) {
  if (pa.nint <= 0) return hipSuccess;
  if (lean_slc_applies(op, lay)) {
    switch (lay.L) {
      case 4: return slc_launch_l<4>(desc, op, lay, pa, stream);
      case 8: return slc_launch_l<8>(desc, op, lay, pa, stream);
      case 16: return slc_launch_l<16>(desc, op, lay, pa, stream);
      default: break;
    }
  }
  const size_t lds = lds_bytes_for(lay, op.has_solve);
  switch (op.kind) {
    case OP_POLY_Z: return launch_kind<OP_POLY_Z>(desc, lay, pa, lds, stream);
    case OP_POLY_W: return launch_kind<OP_POLY_W>(desc, lay, pa, lds, stream);
    case OP_SLC: return launch_kind<OP_SLC>(desc, lay, pa, lds, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tiles(const LevelDesc *desc, const TileGeom &tg, const TileArgs &ta, hipStream_t stream) {
  if (ta.nint <= 0) return hipSuccess;
  switch (tg.P) {
    case 8: return launch_tiles_p<8>(desc, tg, ta, stream);
    case 16: return launch_tiles_p<16>(desc, tg, ta, stream);
    case 32: return launch_tiles_p<32>(desc, tg, ta, stream);
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
