// Step kernel with truncated-carry periodic recurrences (included inside
// namespace mgrit::{anonymous} after mgrit_device.h and mgrit_step.h).
//
// The periodic banded solves of a step (SDIRK stages, Sec. 4.3 footnote; the
// corrected coarse operator, eq. MOL-SL-corrected) apply T^{-1} through the
// factorisation T = C * F(S^-1) * B(S), i.e. a causal recurrence
//     y_i = x_i + sum_{m=1..k} a_m y_{i-m}
// and an anti-causal one.  Every root of F lies inside the unit circle, so
// the recurrence's impulse response decays geometrically.  With chunks of L
// points per thread, the state entering chunk t is exactly
//     E_{t-1} = sum_{d >= 0} H^d Z_{t-1-d},   H = M^L,
// Z the chunks' zero-state end states and M the companion matrix; when
// ||H^D|| is below rounding (checked on the host in extended precision) the
// first D terms are the state to rounding.  A recurrence then costs a
// zero-state pass over the chunk that only keeps its end state, one
// workgroup barrier after the end states are published in LDS, the D-term
// carry (wave-uniform matrices through the scalar cache), and the pass over
// the chunk again from the exact entering state.  No wavefront scan, no
// single-thread fold, no per-point tables.  Both passes run the two halves
// of a chunk as independent chains.
//
// The layout is nx = NT * L exactly (every chunk full); thread t owns points
// [tL, tL + L).
#pragma once

template <int K, class T>
struct WinDir {
  T a[K > 0 ? K : 1];
  int D;            // predecessor chunks in the carry
  ConstPtr<T> tab;  // [D-1][K][K] H^d, d = 1..D-1, then [K][K] M^{L/2}
};

template <int K, class T>
__device__ __forceinline__ void win_dir_load(WinDir<K, T> &W, const Recurrence &rc) {
#pragma unroll
  for (int m = 0; m < (K > 0 ? K : 1); ++m) W.a[m] = (T)rc.a[m < KMAX ? m : 0];
  W.D = rc.D;
  W.tab = (ConstPtr<T>)rc.wtab;
}

// The recurrence over the two halves of a chunk at once, each from its own
// state (sa: entering the first half in processing order, sb: the second;
// s[m] is the value m+1 places back): two independent chains interleaved.
// STORE: overwrite x with the result.
template <int L, int K, bool REV, bool STORE, class T>
__device__ __forceinline__ void win_pass2(T (&x)[L], const T (&a)[K], T (&sa)[K], T (&sb)[K]) {
  constexpr int H = L / 2;
#pragma unroll
  for (int e = 0; e < H; ++e) {
    const int ja = REV ? (L - 1 - e) : e;
    const int jb = REV ? (H - 1 - e) : (H + e);
    T va = x[ja], vb = x[jb];
#pragma unroll
    for (int m = K - 1; m >= 0; --m) {
      va = fma(a[m], sa[m], va);
      vb = fma(a[m], sb[m], vb);
    }
#pragma unroll
    for (int m = K - 1; m > 0; --m) {
      sa[m] = sa[m - 1];
      sb[m] = sb[m - 1];
    }
    sa[0] = va;
    sb[0] = vb;
    if (STORE) {
      x[ja] = va;
      x[jb] = vb;
    }
  }
}

// acc += A x (A row-major K x K, wave-uniform)
template <int K, class T>
__device__ __forceinline__ void win_mv(ConstPtr<T> A, const T (&x)[K], T (&acc)[K]) {
#pragma unroll
  for (int r = 0; r < K; ++r) {
    T v = acc[r];
#pragma unroll
    for (int c = 0; c < K; ++c) v = fma(A[r * K + c], x[c], v);
    acc[r] = v;
  }
}

// One periodic recurrence over the workgroup's chunks (REV: the anti-causal
// one, processing each chunk from its last point and taking the carry from
// the following chunks).  pub: LDS words for the NT published end states.
// The halves of a chunk run as two chains: the chunk's zero-state end state
// is Z_b + G Z_a, and the state entering the second half is Z_a + G E, with
// G = M^{L/2} and Z_a, Z_b the halves' zero-state end states.
struct NoHook {
  __device__ void operator()() const {}
};

template <int L, int K, bool REV, class T, class Hook = NoHook>
__device__ __forceinline__ void win_rec(T (&y)[L], const WinDir<K, T> &W, T *pub, int tid, int NT,
                                        Hook hook = NoHook()) {
  const ConstPtr<T> G = W.tab + (W.D - 1) * K * K;
  // 1. end state of the chunk from a zero state
  T za[K], zb[K];
#pragma unroll
  for (int m = 0; m < K; ++m) za[m] = zb[m] = T(0);
  win_pass2<L, K, REV, false>(y, W.a, za, zb);
  win_mv<K>(G, za, zb);
  // 2. publish it, then sum the carry from the D chunks before this one in
  //    processing order (periodic in the thread index)
#pragma unroll
  for (int m = 0; m < K; ++m) pub[tid * K + m] = zb[m];
  __syncthreads();
  hook();  // every thread of the workgroup is past its step's gather
  int src = REV ? (tid + 1 == NT ? 0 : tid + 1) : (tid == 0 ? NT - 1 : tid - 1);
  T E[K];
#pragma unroll
  for (int m = 0; m < K; ++m) E[m] = pub[src * K + m];
  for (int d = 1; d < W.D; ++d) {
    src = REV ? (src + 1 == NT ? 0 : src + 1) : (src == 0 ? NT - 1 : src - 1);
    T z[K];
#pragma unroll
    for (int m = 0; m < K; ++m) z[m] = pub[src * K + m];
    win_mv<K>(W.tab + (d - 1) * K * K, z, E);
  }
  // 3. the chunk again from the exact entering states of its halves
  win_mv<K>(G, E, za);
  win_pass2<L, K, REV, true>(y, W.a, E, za);
}

// The padded LDS vector of OP_SLC steps: one pad word after every L points,
// so that the chunks of consecutive threads start in different banks.
template <int L>
__device__ __forceinline__ int win_pad(int i) {
  return i + i / L;
}

// out[j] += sum_{t < W} w[t] * v[start + j + t] (indices periodic,
// 0 <= start < nx) from the padded LDS vector; each value is read once and
// scattered into the outputs it feeds.
template <int L, int W, class T>
__device__ __forceinline__ void win_gather(const T *vec, int start, int nx, const T (&w)[MAXTAPS], T (&out)[L]) {
  if (start + L + W - 1 <= nx) {
#pragma unroll
    for (int e = 0; e < L + W - 1; ++e) {
      const T v = vec[win_pad<L>(start + e)];
#pragma unroll
      for (int t = 0; t < W; ++t) {
        const int j = e - t;
        if (j >= 0 && j < L) out[j] = fma(w[t], v, out[j]);
      }
    }
    return;
  }
  int idx = start;
#pragma unroll
  for (int e = 0; e < L + W - 1; ++e) {
    const T v = vec[win_pad<L>(idx)];
#pragma unroll
    for (int t = 0; t < W; ++t) {
      const int j = e - t;
      if (j >= 0 && j < L) out[j] = fma(w[t], v, out[j]);
    }
    idx = next_periodic(idx, nx);
  }
}

// The chain of OP_SLC steps of one workgroup with the state between steps
// held in the padded LDS vector instead of in the threads' chunks.  A step
// gathers from the vector and solves in the chunk layout; its result goes
// back to the vector, and every row access (the initial row, the right-hand
// side added after a step, the parent rows a post-relaxation adds into, the
// rows written out) walks the vector in the coalesced order i = k NT + t:
// consecutive lanes touch consecutive words, where the chunk layout would
// touch one cache line per lane.  Modes and row roles as in run_chain.
// p[0] += v as a device-scope atomic whose result is not returned: the add
// happens in the L2 cache, so the lane never waits for the old value.  Each
// element receives one such add per launch, so the sum is the plain
// correctly rounded a + b.
template <class T>
__device__ __forceinline__ void add_in_cache(T *p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The right-hand-side row of a step straight into the padded LDS vector, 32
// doubles per thread: wavefront w copies the 64 padded segments of 32 doubles
// its own threads own (one dword per lane per instruction, 256 bytes = one
// segment), holding no registers, so the copy runs while the step's solve
// does; after a wait for its own loads (vmcnt) each wavefront reads its
// threads' segments with no barrier.
__device__ __forceinline__ void row_to_lds_async(const double *row, double *vec) {
  const int seg0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~(WAVE - 1)));
  const unsigned *src = reinterpret_cast<const unsigned *>(row) + (threadIdx.x & (WAVE - 1));
  for (int i = 0; i < WAVE; ++i) {
    const int seg = seg0 + i;
    __builtin_amdgcn_global_load_lds(src + seg * 64, (__attribute__((address_space(3))) void *)(vec + seg * 33), 4,
                                     0, 0);
  }
}
// The float32 form: a segment is 32 floats, so one instruction per segment
// with the lower half-wavefront active (an instruction has one LDS base).
__device__ __forceinline__ void row_to_lds_async(const float *row, float *vec) {
  const int seg0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x & ~(WAVE - 1)));
  const int lane = threadIdx.x & (WAVE - 1);
  const unsigned *src = reinterpret_cast<const unsigned *>(row) + lane;
  if (lane < WAVE / 2) {
    for (int i = 0; i < WAVE; ++i) {
      const int seg = seg0 + i;
      __builtin_amdgcn_global_load_lds(src + seg * 32, (__attribute__((address_space(3))) void *)(vec + seg * 33), 4,
                                       0, 0);
    }
  }
}

template <int L, class T, class Step>
__device__ __forceinline__ void run_chain_slc(const PassArgsT<T> &pa, int nx, T *vec, double *red, bool alias,
                                              Step step) {
  typedef __attribute__((address_space(1))) T *gT;
  typedef const __attribute__((address_space(1))) T *gcT;
  // rows move in NB batches of H loads per thread issued together (larger
  // batches run out of registers at 32 points per thread)
  constexpr int H = 8, NB = L / H;
  const int64_t b = blockIdx.x;
  // the thread index and count, read once (blockDim is a memory load, and its
  // wait would also wait for every store and atomic in flight)
  const WalkIdx w0{(int)threadIdx.x, __builtin_amdgcn_readfirstlane((int)blockDim.x)};
  const int64_t nxl = nx;
  const int m = pa.m;
  const int mode = pa.mode;
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
  const bool add_g = pa.g && mode != MODE_APPLY && mode != MODE_RESID;
  const bool add_parent = mode == MODE_POST_F || (mode == MODE_SEQ && pa.parent);
  const bool store_out = mode == MODE_FINAL_F || (mode == MODE_SEQ && pa.out);

  // the initial row, and what the modes do with it
  {
    const gcT cin = (gcT)(pa.cin + row0 * nxl);
    const gT c0 = (gT)pa.cout;
    const gT o0 = (gT)(mode == MODE_FINAL_F ? pa.out + (b * m) * nxl : pa.out);
    for (int h = 0; h < NB; ++h) {
      const WalkIdx w = walk_idx(w0);
      const int tid = w.t, NT = w.nt;
      T x[H];
#pragma unroll
      for (int k = 0; k < H; ++k) x[k] = pa.zero_init ? T(0) : cin[(h * H + k) * NT + tid];
#pragma unroll
      for (int k = 0; k < H; ++k) vec[win_pad<L>((h * H + k) * NT + tid)] = x[k];
      if (mode == MODE_PASS_A && b == 0) {
#pragma unroll
        for (int k = 0; k < H; ++k) c0[(h * H + k) * NT + tid] = x[k];
      }
      if (mode == MODE_FINAL_F || (mode == MODE_SEQ && pa.out)) {
#pragma unroll
        for (int k = 0; k < H; ++k) o0[(h * H + k) * NT + tid] = x[k];
      }
      if (mode == MODE_POST_F) {
#pragma unroll
        for (int k = 0; k < H; ++k) add_in_cache(pa.parent + (b * m) * nxl + (h * H + k) * NT + tid, x[k]);
      }
    }
  }
  __syncthreads();

  // 32 points per thread with separate published states: the right-hand
  // side goes straight into the vector while the solve runs (issued once
  // every thread is past its gather, added to the result after the solve)
  const bool direct_g = L == 32 && !alias && add_g;
  for (int j = 1; j <= nsteps; ++j) {
    const int64_t n = (mode == MODE_SEQ) ? (int64_t)j : b * m + j;  // level point index
    {
      T y[L];
      step(y, [&] {  // every thread is past its gather: the vector's words are free
        if constexpr (L == 32) {
          if (direct_g) row_to_lds_async(pa.g + (n - 1) * nxl, vec);
        }
      });
      const int base = (int)threadIdx.x * L;
      if (direct_g) {
        __builtin_amdgcn_s_waitcnt(0);  // this wavefront's segments of the right-hand side have landed
#pragma unroll
        for (int q = 0; q < L; ++q) {
          const int pq = win_pad<L>(base + q);
          vec[pq] = y[q] + vec[pq];
        }
      } else {
        // every thread is past its gather (the first recurrence's barrier);
        // aliased, the solve's published states must be read first
        if (alias) __syncthreads();
#pragma unroll
        for (int q = 0; q < L; ++q) vec[win_pad<L>(base + q)] = y[q];
      }
    }
    __syncthreads();
    if (direct_g) {
      if (add_parent || store_out) {
        const WalkIdx w = walk_idx(w0);
        const gT o = (gT)(pa.out + n * nxl);
        for (int h = 0; h < NB; ++h) {
          T x[H];
#pragma unroll
          for (int k = 0; k < H; ++k) x[k] = vec[win_pad<L>((h * H + k) * w.nt + w.t)];
          if (add_parent) {
#pragma unroll
            for (int k = 0; k < H; ++k) add_in_cache(pa.parent + n * nxl + (h * H + k) * w.nt + w.t, x[k]);
          }
          if (store_out) {
#pragma unroll
            for (int k = 0; k < H; ++k) o[(h * H + k) * w.nt + w.t] = x[k];
          }
        }
      }
      continue;
    }
    if (add_g || add_parent || store_out) {
      const gcT g = (gcT)(pa.g + (n - 1) * nxl);
      const gT o = (gT)(pa.out + n * nxl);
      for (int h = 0; h < NB; ++h) {
        const WalkIdx w = walk_idx(w0);
        const int tid = w.t, NT = w.nt;
        T x[H];
#pragma unroll
        for (int k = 0; k < H; ++k) x[k] = vec[win_pad<L>((h * H + k) * NT + tid)];
        if (add_g) {
          T gv[H];
#pragma unroll
          for (int k = 0; k < H; ++k) gv[k] = g[(h * H + k) * NT + tid];
#pragma unroll
          for (int k = 0; k < H; ++k) {
            x[k] += gv[k];
            vec[win_pad<L>((h * H + k) * NT + tid)] = x[k];
          }
        }
        if (add_parent) {
#pragma unroll
          for (int k = 0; k < H; ++k) add_in_cache(pa.parent + n * nxl + (h * H + k) * NT + tid, x[k]);
        }
        if (store_out) {
#pragma unroll
          for (int k = 0; k < H; ++k) o[(h * H + k) * NT + tid] = x[k];
        }
      }
      if (add_g) __syncthreads();
    }
  }

  // post-chain actions (the vector holds the chain's last point)
  if (mode == MODE_PASS_A || mode == MODE_APPLY) {
    const WalkIdx w = walk_idx(w0);
    const int tid = w.t, NT = w.nt;
    const gT c1 = (gT)(pa.cout + (mode == MODE_PASS_A ? b + 1 : b) * nxl);
#pragma unroll
    for (int k = 0; k < L; ++k) c1[k * NT + tid] = vec[win_pad<L>(k * NT + tid)];
  } else if (mode == MODE_PASS_B || mode == MODE_RESID) {
    const gcT c1 = (gcT)(pa.cin + (b + 1) * nxl);
    const gT r = (gT)(pa.r + b * nxl);
    double ss = 0.0;
    for (int h = 0; h < NB; ++h) {
      const WalkIdx w = walk_idx(w0);
      const int tid = w.t, NT = w.nt;
      T x[H];
#pragma unroll
      for (int k = 0; k < H; ++k) x[k] = c1[(h * H + k) * NT + tid];
#pragma unroll
      for (int k = 0; k < H; ++k) {
        x[k] = vec[win_pad<L>((h * H + k) * NT + tid)] - x[k];
        ss = fma((double)x[k], (double)x[k], ss);
      }
      if (pa.r) {
#pragma unroll
        for (int k = 0; k < H; ++k) r[(h * H + k) * NT + tid] = x[k];
      }
    }
    const double tot = block_sum(ss, red);
    if (threadIdx.x == 0) pa.normpart[b] = tot;
  } else if (mode == MODE_POST_F || mode == MODE_FINAL_F) {
    if (b == pa.nint - 1) {
      const gcT cl = (gcT)(pa.cin + pa.nint * nxl);
      const gT row = (gT)((mode == MODE_POST_F ? pa.parent : pa.out) + (pa.nint * m) * nxl);
      for (int h = 0; h < NB; ++h) {
        const WalkIdx w = walk_idx(w0);
        const int tid = w.t, NT = w.nt;
        T x[H];
#pragma unroll
        for (int k = 0; k < H; ++k) x[k] = cl[(h * H + k) * NT + tid];
        if (mode == MODE_POST_F) {
#pragma unroll
          for (int k = 0; k < H; ++k)
            add_in_cache(pa.parent + (pa.nint * m) * nxl + (h * H + k) * NT + tid, x[k]);
        } else {
#pragma unroll
          for (int k = 0; k < H; ++k) row[(h * H + k) * NT + tid] = x[k];
        }
      }
    }
  }
}

// Operator constants of the windowed kernel.
template <int KF, int KB, class T>
struct WinOp {
  int repeat;
  int ncoef;
  const double *coef;  // OP_POLY_W: Horner coefficients in B^{-1} F^{-1} (1/C folded in)
  T top;
  int off;             // OP_SLC: start offset of the interpolation taps
  T w[MAXTAPS];        // OP_SLC: interpolation weights (1/C folded in)
  WinDir<KF, T> f;
  WinDir<KB, T> b;
};

// y <- B^{-1} F^{-1} y.  pub0/pub1: the published-state areas.  With no
// anti-causal factor the causal recurrence alternates between them (flip), so
// that a recurrence never overwrites words another thread has yet to read.
// hook: run once by every thread right after the first recurrence's barrier
// (every thread is then past the gather that preceded the solve).
template <int L, int KF, int KB, class T, class Hook = NoHook>
__device__ __forceinline__ void win_solve(T (&y)[L], const WinOp<KF, KB, T> &R, T *pub0, T *pub1, int &flip,
                                          int tid, int NT, Hook hook = NoHook()) {
  if constexpr (KF > 0) {
    win_rec<L, KF, false>(y, R.f, flip ? pub1 : pub0, tid, NT, hook);
    if constexpr (KB == 0) flip ^= 1;
  }
  if constexpr (KB > 0) {
    if constexpr (KF > 0)
      win_rec<L, KB, true>(y, R.b, pub1, tid, NT);
    else
      win_rec<L, KB, true>(y, R.b, pub1, tid, NT, hook);
  }
}

template <int L, int KIND, int KF, int KB, int MAXT, class T>
__global__ void __launch_bounds__(MAXT) wstep_kernel(const LevelDesc *__restrict__ desc, PassArgsT<T> pa) {
  if (pa.stop && *pa.stop) return;  // the solve has already stopped
  constexpr int KW = (KF > KB ? KF : KB) > 0 ? (KF > KB ? KF : KB) : 1;
  extern __shared__ double smem[];
  const StepOp &op = desc->op;
  const int nx = desc->lay.nx;
  const int NT = blockDim.x;
  const int tid = threadIdx.x;
  const WinLds lo = win_lds(KIND, nx, NT, KW, (int)sizeof(T), L);
  T *sm = reinterpret_cast<T *>(smem);
  T *vec = sm;  // the padded vector (OP_SLC: the gather's; OP_POLY_W: row staging)
  T *pub0 = sm + lo.pub0, *pub1 = sm + lo.pub1;
  double *red = smem + lo.red;

  WinOp<KF, KB, T> R;
  R.repeat = op.repeat;
  R.ncoef = op.ncoef;
  R.coef = op.wcoef;
  R.top = KIND == OP_POLY_W ? (T)op.wcoef[op.ncoef - 1] : T(0);
  if (KIND == OP_SLC) {
    R.off = op.sl_K + op.sl_l;
#pragma unroll
    for (int t = 0; t < MAXTAPS; ++t) R.w[t] = (T)(op.slw[t] * op.cinv);
  }
  win_dir_load<KF, T>(R.f, op.fw);
  win_dir_load<KB, T>(R.b, op.bw);

  int flip = 0;
  // OP_SLC with the chain state in LDS; with 1024 threads (128 registers per
  // thread) the coalesced batches do not fit, and the state stays in the chunks
  if constexpr (KIND == OP_SLC && MAXT <= 512) {
    const int base = tid * L;
    // y = Psi^repeat of the vector; the vector holds the input on entry
    run_chain_slc<L, T>(pa, nx, vec, red, lo.alias != 0, [&](T (&y)[L], auto after_gather) {
      for (int rep = 0; rep < R.repeat; ++rep) {
        if (rep > 0) {
          __syncthreads();  // every thread has finished the previous gather
#pragma unroll
          for (int j = 0; j < L; ++j) vec[win_pad<L>(base + j)] = y[j];
          __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < L; ++j) y[j] = T(0);
        win_gather<L, 2 * KF>(vec, wrap_lo(base - R.off, nx), nx, R.w, y);
        if (lo.alias) __syncthreads();  // the published states reuse the vector's words
        const bool last = rep + 1 == R.repeat;
        win_solve<L, KF, KB>(y, R, pub0, pub1, flip, tid, NT, [&] {
          if (last) after_gather();
        });
      }
    });
    return;
  }
  // OP_POLY_W: rows move through the padded LDS vector (coalesced); the rows
  // a step adds are read after the step: loading them before it (into
  // registers) measured slower at 32 points per thread
  run_chain<L, T, 0, KIND == OP_POLY_W>(pa, nx, L, red, [&](T (&u)[L]) {
    const int base = tid * L;
    for (int rep = 0; rep < R.repeat; ++rep) {
      T y[L];
      if constexpr (KIND == OP_SLC) {
        __syncthreads();  // every thread has finished the previous gather
#pragma unroll
        for (int j = 0; j < L; ++j) vec[win_pad<L>(base + j)] = u[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < L; ++j) y[j] = T(0);
        win_gather<L, 2 * KF>(vec, wrap_lo(base - R.off, nx), nx, R.w, y);
        if (lo.alias) __syncthreads();  // the published states reuse the vector's words
        win_solve<L, KF, KB>(y, R, pub0, pub1, flip, tid, NT);
      } else {  // OP_POLY_W: Phi u = sum_i wcoef[i] (B^{-1} F^{-1})^i u by Horner
#pragma unroll
        for (int j = 0; j < L; ++j) y[j] = R.top * u[j];
        for (int i = R.ncoef - 2; i >= 0; --i) {
          win_solve<L, KF, KB>(y, R, pub0, pub1, flip, tid, NT);
          const T ci = (T)R.coef[i];
#pragma unroll
          for (int j = 0; j < L; ++j) y[j] = fma(ci, u[j], y[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < L; ++j) u[j] = y[j];
    }
  }, vec);
}
