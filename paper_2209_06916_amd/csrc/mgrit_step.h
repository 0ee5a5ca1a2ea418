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
// homogeneous correction pass.  The scan's matrices (powers of H, the wrap
// matrix) are read through the scalar cache from device memory where every
// lane of a wavefront reads the same one, and from a copy staged in LDS once
// per launch where the power depends on the lane; operator coefficients are
// held in registers.  No MFMA: nothing here is a dense contraction.
#pragma once

// out[j] += w[0] * v[start+j] + ... + w[width-1] * v[start+j+width-1]
// (indices periodic), reading the padded LDS copy v; 0 <= start < nx.  Each
// LDS value is read once and scattered into the outputs it feeds.  Full
// chunks whose window does not wrap take a branch-free path.
template <int L, class T>
__device__ __forceinline__ void window_combine(const T *vec, int start, int cnt, int width, int nx,
                                               const T (&w)[MAXTAPS], T (&out)[L]) {
  if (cnt == L && start + L + width - 1 <= nx) {
#pragma unroll
    for (int e = 0; e < L + MAXTAPS - 1; ++e) {
      if (e < L + width - 1) {  // uniform
        const T v = vec[padix(start + e)];
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
      const T v = vec[padix(idx)];
#pragma unroll
      for (int t = 0; t < MAXTAPS; ++t) {
        const int j = e - t;
        if (j >= 0 && j < L && t < width) out[j] = fma(w[t], v, out[j]);
      }
      idx = next_periodic(idx, nx);
    }
  }
}

template <int K, class T, class TP>
__device__ __forceinline__ void matvec_add(TP H, const T (&x)[K], T (&acc)[K]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    T s = acc[i];
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
template <class T>
using ConstPtr = const __attribute__((address_space(4))) T *;

// tab: the LDS copy of the tables (lane-dependent reads); ctab: the same
// tables in device memory, read through the scalar cache where the index is
// the same for the whole wavefront.
template <int L, int K, bool REV, class T>
__device__ __forceinline__ void recurrence(T (&x)[L], int cnt, int vt, int A, int NT, const T (&ain)[KMAX],
                                           const T *tab, ConstPtr<T> ctab, T *scr) {
  constexpr int KK = K * K;
  T a[K];
#pragma unroll
  for (int m = 0; m < K; ++m) a[m] = ain[m];

  // 1. zero-state pass over the chunk (branch-free when the chunk is full)
  const bool full = (cnt == L);
  T s[K];
#pragma unroll
  for (int m = 0; m < K; ++m) s[m] = 0.0;
#pragma unroll
  for (int e = 0; e < L; ++e) {
    const int j = REV ? (L - 1 - e) : e;
    T y = x[j];
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
  const int nw = NT >> 6;
  const int vl = REV ? (WAVE - 1 - lane) : lane;
  const int vw = REV ? (nw - 1 - wv) : wv;
  T inc[K];
#pragma unroll
  for (int m = 0; m < K; ++m) inc[m] = s[m];
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const int src = (REV ? (lane + d) : (lane - d)) & (WAVE - 1);
    T o[K];
#pragma unroll
    for (int m = 0; m < K; ++m) o[m] = __shfl(inc[m], src, WAVE);
    T t[K];
#pragma unroll
    for (int m = 0; m < K; ++m) t[m] = inc[m];
    matvec_add<K>(ctab + d * KK, o, t);
    const bool take = vl >= d;
#pragma unroll
    for (int m = 0; m < K; ++m) inc[m] = take ? t[m] : inc[m];
  }
  // exclusive value within the wavefront
  T ex[K];
  {
    const int src = (REV ? (lane + 1) : (lane - 1)) & (WAVE - 1);
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const T o = __shfl(inc[m], src, WAVE);
      ex[m] = (vl >= 1) ? o : 0.0;
    }
  }

  // 3. wavefront totals -> LDS
  T *Q = scr;
  T *Xc = scr + MAXWAVES * K;
  if (vl == WAVE - 1) {
#pragma unroll
    for (int m = 0; m < K; ++m) Q[vw * K + m] = inc[m];
  }
  __syncthreads();

  // 4. one thread: carry into its wavefront, the periodic wrap s_0, and the
  //    carries X'_w (with s_0 folded in) of every wavefront
  if (vt == A - 1) {
    const ConstPtr<T> H64 = ctab + WAVE * KK;
    const ConstPtr<T> Hlast = ctab + (WAVE + 1) * KK;
    const ConstPtr<T> Wwrap = ctab + (WAVE + 2) * KK;
    T X[K];
#pragma unroll
    for (int m = 0; m < K; ++m) X[m] = 0.0;
    for (int w2 = 0; w2 < vw; ++w2) {
      T nx_[K];
#pragma unroll
      for (int m = 0; m < K; ++m) nx_[m] = Q[w2 * K + m];
      matvec_add<K>(H64, X, nx_);
#pragma unroll
      for (int m = 0; m < K; ++m) X[m] = nx_[m];
    }
    T E[K];
#pragma unroll
    for (int m = 0; m < K; ++m) E[m] = ex[m];
    matvec_add<K>(tab + vl * KK, X, E);
    T tq[K];
#pragma unroll
    for (int m = 0; m < K; ++m) tq[m] = s[m];
    matvec_add<K>(Hlast, E, tq);
    T xp[K];
#pragma unroll
    for (int m = 0; m < K; ++m) xp[m] = 0.0;
    matvec_add<K>(Wwrap, tq, xp);  // s_0
#pragma unroll
    for (int m = 0; m < K; ++m) Xc[m] = xp[m];
    for (int w2 = 0; w2 + 1 < nw; ++w2) {
      T nx_[K];
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
    T xc[K];
#pragma unroll
    for (int m = 0; m < K; ++m) xc[m] = Xc[vw * K + m];
    T st[K];
#pragma unroll
    for (int m = 0; m < K; ++m) st[m] = ex[m];
    matvec_add<K>(tab + vl * KK, xc, st);
#pragma unroll
    for (int e = 0; e < L; ++e) {
      const int j = REV ? (L - 1 - e) : e;
      T hv = 0.0;
#pragma unroll
      for (int m = 0; m < K; ++m) hv = fma(a[m], st[m], hv);
#pragma unroll
      for (int m = K - 1; m > 0; --m) st[m] = st[m - 1];
      st[0] = hv;
      x[j] = (full || e < cnt) ? x[j] + hv : x[j];
    }
  }
}

template <int L, bool REV, class T>
__device__ __forceinline__ void recurrence_k(T (&x)[L], int cnt, int vt, int A, int NT, int k,
                                             const T (&a)[KMAX], const T *tab, ConstPtr<T> ctab, T *scr) {
  switch (k) {
    case 1: recurrence<L, 1, REV>(x, cnt, vt, A, NT, a, tab, ctab, scr); break;
    case 2: recurrence<L, 2, REV>(x, cnt, vt, A, NT, a, tab, ctab, scr); break;
    case 3: recurrence<L, 3, REV>(x, cnt, vt, A, NT, a, tab, ctab, scr); break;
    default: break;
  }
}

// Operator constants held in registers for the whole launch (in the
// kernel's precision T; the Horner coefficients are read through the
// descriptor in double and rounded at use).
template <class T>
struct OpRegs {
  int ncoef;
  const double *coef;  // Horner coefficients, read through the descriptor
  T top;               // coef[ncoef - 1]
  int width;  // stencil (OP_POLY_Z) or interpolation (OP_SLC) taps
  int off;    // OP_POLY_Z: st_l; OP_SLC: sl_K + sl_l
  T w[MAXTAPS];
  int has_solve, kf, kb;
  T cinv;
  T af[KMAX], ab[KMAX];
  int repeat;
};

// LDS regions of one launch.
template <class T>
struct Lds {
  T *vec0, *vec1;   // padded vectors (vec1 == vec0 unless double-buffered)
  T *tab_f, *tab_b; // recurrence tables
  ConstPtr<T> ctab_f, ctab_b;  // the same tables in device memory (uniform reads)
  T *scr_f, *scr_b; // recurrence scratch
  double *red;      // reduction scratch
};

// y <- T^{-1} y
template <int L, class T>
__device__ __forceinline__ void solve(T (&y)[L], int cnt, const OpRegs<T> &R, const Layout &lay, const Lds<T> &S) {
  const int tid = threadIdx.x;
  const int nx = lay.nx;
  if (R.kf > 0) recurrence_k<L, false>(y, cnt, tid, lay.A, lay.T, R.kf, R.af, S.tab_f, S.ctab_f, S.scr_f);
  if (R.kb > 0) {
    if (!lay.ragged) {
      recurrence_k<L, true>(y, cnt, lay.T - 1 - tid, lay.A, lay.T, R.kb, R.ab, S.tab_b, S.ctab_b, S.scr_b);
    } else {
      // redistribute so that thread t owns indices nx-1-(tL+j), j = 0..cnt-1
      T *vec = S.vec0;
      const int base = tid * L;
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (j < cnt) vec[padix(base + j)] = y[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = (j < cnt) ? vec[padix(nx - 1 - (base + j))] : 0.0;
      recurrence_k<L, false>(y, cnt, tid, lay.A, lay.T, R.kb, R.ab, S.tab_b, S.ctab_b, S.scr_b);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j)
        if (j < cnt) vec[padix(nx - 1 - (base + j))] = y[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < L; ++j) y[j] = (j < cnt) ? vec[padix(base + j)] : 0.0;
    }
  }
  const T ci = R.cinv;
#pragma unroll
  for (int j = 0; j < L; ++j) y[j] *= ci;
}

// coef[i] (uniform scalar load through the descriptor)
template <class T>
__device__ __forceinline__ T coef_at(const OpRegs<T> &R, int i) { return (T)R.coef[i]; }

// u <- Phi u  (every thread of the workgroup must call this).  buf: which
// LDS vector the next explicit stencil writes (double-buffered layouts).
template <int L, int KIND, class T>
__device__ __forceinline__ void apply_step(T (&u)[L], int cnt, const OpRegs<T> &R, const Layout &lay,
                                           const Lds<T> &S, int &buf) {
  const int nx = lay.nx;
  const int base = threadIdx.x * L;
  T y[L];
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
        T *v = buf ? S.vec1 : S.vec0;
        if (!lay.dbuf) __syncthreads();
        chunk_to_lds<L>(v, base, cnt, y);
        __syncthreads();
        const T ci = coef_at(R, i);
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
        const T ci = coef_at(R, i);
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
// Coalesced row walks (i = k NT + t) recompute their addresses from an
// opaque copy of the thread index in every phase: hoisted out of a step loop,
// the 2 L addresses of a walk would stay live across steps that already need
// nearly every register.
struct WalkIdx {
  int t;   // thread index
  int nt;  // threads (wave-uniform)
};
__device__ __forceinline__ WalkIdx walk_idx(const WalkIdx &w0) {
  WalkIdx w = w0;
  asm volatile("" : "+v"(w.t), "+s"(w.nt));
  return w;
}

// A row moved between global memory and the threads' chunks (L points per
// thread, nx = NT L) through an LDS staging vector padded like the
// windowed kernel's (one word after every L points), so that the global side
// is coalesced: one cache line per 16 lanes instead of one per lane.  Every
// thread must call; both end with a barrier, so the staging words are free
// again on return.
template <int L, class T>
__device__ __forceinline__ void staged_load(const T *row, T (&x)[L], T *stage, const WalkIdx &w0) {
  typedef const __attribute__((address_space(1))) T *gcT;
  __syncthreads();  // the staging words are free
  {
    const WalkIdx w = walk_idx(w0);
    const gcT g = (gcT)row;
    constexpr int H = 8;
    for (int h = 0; h < L / H; ++h) {
      T v[H];
#pragma unroll
      for (int k = 0; k < H; ++k) v[k] = g[(h * H + k) * w.nt + w.t];
#pragma unroll
      for (int k = 0; k < H; ++k) stage[(h * H + k) * w.nt + w.t + ((h * H + k) * w.nt + w.t) / L] = v[k];
    }
  }
  __syncthreads();
  const int base = (int)threadIdx.x * L;
#pragma unroll
  for (int j = 0; j < L; ++j) x[j] = stage[base + j + (base + j) / L];
  __syncthreads();
}

template <int L, class T, class U>
__device__ __forceinline__ void staged_store(U *row, const T (&x)[L], T *stage, const WalkIdx &w0) {
  typedef __attribute__((address_space(1))) U *gU;
  __syncthreads();  // the staging words are free
  const int base = (int)threadIdx.x * L;
#pragma unroll
  for (int j = 0; j < L; ++j) stage[base + j + (base + j) / L] = x[j];
  __syncthreads();
  {
    const WalkIdx w = walk_idx(w0);
    const gU g = (gU)row;
#pragma unroll 8
    for (int k = 0; k < L; ++k) {
      const int i = k * w.nt + w.t;
      g[i] = (U)stage[i + i / L];
    }
  }
  __syncthreads();
}

template <int L, class T, int PREFETCH = (L <= 16 ? 3 : 0), bool STAGED = false, class Step>
__device__ __forceinline__ void run_chain(const PassArgsT<T> &pa, int nx, int cnt, double *red, Step step,
                                          T *stage = nullptr) {
  const int tid = threadIdx.x;
  const int base = tid * L;
  const int64_t b = blockIdx.x;
  const int64_t nxl = nx;
  const int m = pa.m;
  const int mode = pa.mode;
  T u[L];
  // STAGED (nx = NT L, every chunk full): rows move through the LDS staging
  // vector, coalesced
  const WalkIdx w0{(int)threadIdx.x, STAGED ? __builtin_amdgcn_readfirstlane((int)blockDim.x) : 0};
  auto ld = [&](const T *row, T(&x)[L]) {
    if constexpr (STAGED)
      staged_load<L>(row, x, stage, w0);
    else
      load_chunk<L>(row, base, cnt, x);
  };
  auto st = [&](T *row, const T(&x)[L]) {
    if constexpr (STAGED)
      staged_store<L>(row, x, stage, w0);
    else
      store_chunk<L>(row, base, cnt, x);
  };
  auto st32 = [&](float *row, const T(&x)[L]) {  // the row rounded to float32
    if constexpr (STAGED) {
      staged_store<L>(row, x, stage, w0);
    } else {
      float xs[L];
#pragma unroll
      for (int q = 0; q < L; ++q) xs[q] = (float)x[q];
      store_chunk<L>(row, base, cnt, xs);
    }
  };

  int nsteps;
  switch (mode) {
    case MODE_PASS_A: nsteps = m; break;
    case MODE_PASS_B: nsteps = m; break;
    case MODE_POST_F: nsteps = m - 1; break;
    case MODE_FINAL_F: nsteps = m - 1; break;
    case MODE_SEQ: nsteps = m; break;
    case MODE_APPLY: nsteps = m; break;
    default: nsteps = m; break;  // MODE_RESID: m consecutive time points per workgroup
  }
  const int64_t row0 = (mode == MODE_SEQ) ? 0 : (mode == MODE_RESID ? b * m : b);
  double rss = 0.0;  // MODE_RESID: sum of squares of this workgroup's residual rows
  if (pa.zero_init) {
#pragma unroll
    for (int j = 0; j < L; ++j) u[j] = 0.0;
  } else {
    ld(pa.cin + row0 * nxl, u);
  }
  if (mode == MODE_PASS_A && b == 0) st(pa.cout, u);
  if (mode == MODE_FINAL_F) st(pa.out + (b * m) * nxl, u);
  if (mode == MODE_SEQ && pa.out) st(pa.out, u);
  const bool add_g = pa.g && mode != MODE_APPLY && mode != MODE_RESID;
  const bool add_parent = mode == MODE_POST_F || (mode == MODE_SEQ && pa.parent);
  const bool store_out = mode == MODE_FINAL_F || (mode == MODE_SEQ && pa.out);
  if (mode == MODE_POST_F) {
    T pv[L];
    load_chunk<L>(pa.parent + (b * m) * nxl, base, cnt, pv);
#pragma unroll
    for (int j = 0; j < L; ++j) pv[j] += u[j];
    store_chunk<L>(pa.parent + (b * m) * nxl, base, cnt, pv);
  }

  // the chain of time steps (single call site of the step); the rows this
  // step adds are loaded before the step so their latency overlaps it where
  // PREFETCH says so (bit 0: right-hand side, bit 1: parent; by default for
  // short chunks)
  constexpr bool PRE_G = PREFETCH & 1, PRE_P = PREFETCH & 2;
  for (int j = 1; j <= nsteps; ++j) {
    const int64_t n = (mode == MODE_SEQ) ? (int64_t)j : b * m + j;  // level point index
    T gv[PRE_G ? L : 1], pv[PRE_P ? L : 1];
    if (PRE_G && add_g) load_chunk<PRE_G ? L : 1>(pa.g + (n - 1) * nxl, base, cnt, gv);
    if (PRE_P && add_parent) load_chunk<PRE_P ? L : 1>(pa.parent + n * nxl, base, cnt, pv);
    step(u);
    if (add_g) {
      if (PRE_G) {
#pragma unroll
        for (int q = 0; q < (PRE_G ? L : 1); ++q) u[q] += gv[q];
      } else {
        const GlobalPtr<const T> gr = (GlobalPtr<const T>)(pa.g + (n - 1) * nxl + base);
#pragma unroll
        for (int q = 0; q < L; ++q)
          if (q < cnt) u[q] += gr[q];
      }
    }
    if (add_parent) {
      if (PRE_P) {
#pragma unroll
        for (int q = 0; q < (PRE_P ? L : 1); ++q) pv[q] += u[q];
        store_chunk<PRE_P ? L : 1>(pa.parent + n * nxl, base, cnt, pv);
      } else {
        const GlobalPtr<T> pr = (GlobalPtr<T>)(pa.parent + n * nxl + base);
#pragma unroll
        for (int q = 0; q < L; ++q)
          if (q < cnt) pr[q] += u[q];
      }
    }
    if (store_out) st(pa.out + n * nxl, u);
    if (mode == MODE_RESID) {
      // r_{n-1} = Phi u_{n-1} - u_n; the next step starts from u_n itself
      T c1[L];
      ld(pa.cin + n * nxl, c1);
#pragma unroll
      for (int q = 0; q < L; ++q) {
        u[q] -= c1[q];
        if (q < cnt) rss = fma((double)u[q], (double)u[q], rss);
      }
      if (pa.r) st(pa.r + (n - 1) * nxl, u);
      if (pa.r32) st32(pa.r32 + (n - 1) * nxl, u);
#pragma unroll
      for (int q = 0; q < L; ++q) u[q] = c1[q];
    }
  }

  // post-chain actions
  if (mode == MODE_PASS_A) {
    st(pa.cout + (b + 1) * nxl, u);
  } else if (mode == MODE_PASS_B) {
    double ss = 0.0;
    if constexpr (STAGED) {
      T c1[L];
      ld(pa.cin + (b + 1) * nxl, c1);
#pragma unroll
      for (int j = 0; j < L; ++j) {
        u[j] -= c1[j];
        ss = fma((double)u[j], (double)u[j], ss);
      }
    } else {
      const T *__restrict__ c1 = pa.cin + (b + 1) * nxl;
#pragma unroll
      for (int j = 0; j < L; ++j) {
        if (j < cnt) {
          u[j] -= c1[base + j];
          ss = fma((double)u[j], (double)u[j], ss);
        }
      }
    }
    if (pa.r) st(pa.r + b * nxl, u);
    const double tot = block_sum(ss, red);
    if (tid == 0) pa.normpart[b] = tot;
  } else if (mode == MODE_RESID) {
    const double tot = block_sum(rss, red);
    if (tid == 0) pa.normpart[b] = tot;
  } else if (mode == MODE_POST_F || mode == MODE_FINAL_F) {
    if (b == pa.nint - 1) {
      ld(pa.cin + pa.nint * nxl, u);
      T *row = (mode == MODE_POST_F ? pa.parent : pa.out) + (pa.nint * m) * nxl;
      if (mode == MODE_POST_F) {
        T pv[L];
        ld(row, pv);
#pragma unroll
        for (int j = 0; j < L; ++j) u[j] += pv[j];
      }
      st(row, u);
    }
  } else if (mode == MODE_APPLY) {
    __syncthreads();  // in-place use: every thread has read its input row
    st(pa.cout + b * nxl, u);
  }
}

template <int L, int KIND, int MAXT, class T>
__global__ void __launch_bounds__(MAXT) step_kernel(const LevelDesc *__restrict__ desc, PassArgsT<T> pa) {
  if (pa.stop && *pa.stop) return;  // the solve has already stopped
  // LDS is sized in doubles for either precision: the T arrays use the same
  // element offsets, and the double reduction scratch lies past all of them
  extern __shared__ double smem[];
  T *sm = reinterpret_cast<T *>(smem);
  const Layout lay = desc->lay;
  const StepOp &op = desc->op;
  const int nx = lay.nx;
  const LdsOffsets lo = lds_offsets(lay, op.has_solve);
  Lds<T> S;
  S.vec0 = sm;
  S.vec1 = sm + lo.vec1;
  S.tab_f = sm + lo.tab_f;
  S.tab_b = sm + lo.tab_b;
  S.ctab_f = (ConstPtr<T>)op.fw.tab;
  S.ctab_b = (ConstPtr<T>)op.bw.tab;
  S.scr_f = sm + lo.scr_f;
  S.scr_b = sm + lo.scr_b;
  S.red = smem + lo.red;

  // operator constants -> registers
  OpRegs<T> R;
  R.repeat = op.repeat;
  R.ncoef = op.ncoef;
  R.coef = op.coef;
  R.top = (T)op.coef[op.ncoef - 1];
  if (KIND == OP_SLC) {
    R.width = op.sl_l + op.sl_r + 1;
    R.off = op.sl_K + op.sl_l;
#pragma unroll
    for (int t = 0; t < MAXTAPS; ++t) R.w[t] = (T)op.slw[t];
  } else {
    R.width = op.st_l + op.st_r + 1;
    R.off = op.st_l;
#pragma unroll
    for (int t = 0; t < MAXTAPS; ++t) R.w[t] = (T)op.taps[t];
  }
  R.has_solve = op.has_solve;
  R.kf = op.fw.k;
  R.kb = op.bw.k;
  R.cinv = (T)op.cinv;
#pragma unroll
  for (int m = 0; m < KMAX; ++m) {
    R.af[m] = (T)op.fw.a[m];
    R.ab[m] = (T)op.bw.a[m];
  }
  // recurrence tables (stored in T by the host) -> LDS
  if (KIND != OP_POLY_Z && R.has_solve) {
    const T *tf = static_cast<const T *>(op.fw.tab), *tb = static_cast<const T *>(op.bw.tab);
    const int nf = R.kf * R.kf * RTAB, nb = R.kb * R.kb * RTAB;
    for (int i = threadIdx.x; i < nf; i += blockDim.x) S.tab_f[i] = tf[i];
    for (int i = threadIdx.x; i < nb; i += blockDim.x) S.tab_b[i] = tb[i];
  }
  __syncthreads();

  const int tid = threadIdx.x;
  const int cnt = min(max(nx - tid * L, 0), L);
  int buf = 0;
  run_chain<L, T>(pa, nx, cnt, S.red, [&](T (&u)[L]) { apply_step<L, KIND, T>(u, cnt, R, lay, S, buf); });
}

template <int L, int KIND, class T>
hipError_t set_lds(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)step_kernel<L, KIND, 256, T>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e) return e;
  return hipFuncSetAttribute((const void *)step_kernel<L, KIND, 1024, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <int KIND, class T>
hipError_t set_lds_all(size_t bytes) {
  hipError_t e;
  if ((e = set_lds<2, KIND, T>(bytes))) return e;
  if ((e = set_lds<4, KIND, T>(bytes))) return e;
  if ((e = set_lds<8, KIND, T>(bytes))) return e;
  return set_lds<16, KIND, T>(bytes);
}

template <int L, int KIND, class T>
void launch_l(const LevelDesc *desc, const Layout &lay, const PassArgsT<T> &pa, size_t lds, hipStream_t stream) {
  const dim3 grid((unsigned)pa.nint);
  const dim3 block((unsigned)lay.T);
  if (lay.T <= 256)
    hipLaunchKernelGGL((step_kernel<L, KIND, 256, T>), grid, block, lds, stream, desc, pa);
  else
    hipLaunchKernelGGL((step_kernel<L, KIND, 1024, T>), grid, block, lds, stream, desc, pa);
}

template <int KIND, class T>
hipError_t launch_kind(const LevelDesc *desc, const Layout &lay, const PassArgsT<T> &pa, size_t lds,
                       hipStream_t stream) {
  if (lay.T < WAVE || lay.T > 1024 || lay.T % WAVE) return hipErrorInvalidValue;
  switch (lay.L) {
    case 2: launch_l<2, KIND, T>(desc, lay, pa, lds, stream); break;
    case 4: launch_l<4, KIND, T>(desc, lay, pa, lds, stream); break;
    case 8: launch_l<8, KIND, T>(desc, lay, pa, lds, stream); break;
    case 16: launch_l<16, KIND, T>(desc, lay, pa, lds, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
