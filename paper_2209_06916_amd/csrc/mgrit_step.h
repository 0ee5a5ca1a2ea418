// Generic gfx950 step kernel for MGRIT on method-of-lines advection
// (included inside namespace mgrit::{anonymous} by the per-kind
// translation units).
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
#pragma once

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
      idx = next_periodic(idx, nx);
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
  if (pa.stop && *pa.stop) return;  // the solve has already stopped
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
