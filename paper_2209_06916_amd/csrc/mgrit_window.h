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
// zero-state pass over the chunk, one workgroup barrier after the end states
// are published in LDS, the D-term carry and a correction over the first hc
// points of the chunk (the homogeneous response, row 0 of M^{e+1} times the
// carry, through the scalar cache).  No wavefront scan and no single-thread
// fold; the carry and correction matrices are wave-uniform.
//
// The layout is nx = NT * L exactly (every chunk full); thread t owns points
// [tL, tL + L).
#pragma once

template <int K, class T>
struct WinDir {
  T a[K > 0 ? K : 1];
  int D;            // predecessor chunks in the carry
  int hc;           // corrected points per chunk
  ConstPtr<T> tab;  // [D-1][K][K] H^d, d = 1..D-1, then [L][K] row 0 of M^{e+1}
};

template <int K, class T>
__device__ __forceinline__ void win_dir_load(WinDir<K, T> &W, const Recurrence &rc) {
#pragma unroll
  for (int m = 0; m < (K > 0 ? K : 1); ++m) W.a[m] = (T)rc.a[m < KMAX ? m : 0];
  W.D = rc.D;
  W.hc = rc.hc;
  W.tab = (ConstPtr<T>)rc.wtab;
}

// One periodic recurrence over the workgroup's chunks (REV: the anti-causal
// one, processing each chunk from its last point and taking the carry from
// the following chunks).  pub: LDS words for the NT published end states.
template <int L, int K, bool REV, class T>
__device__ __forceinline__ void win_rec(T (&y)[L], const WinDir<K, T> &W, T *pub, int tid, int NT) {
  // 1. zero-state pass; s[m] = y of the point m+1 places back in processing order
  T s[K];
#pragma unroll
  for (int m = 0; m < K; ++m) s[m] = T(0);
#pragma unroll
  for (int e = 0; e < L; ++e) {
    const int j = REV ? (L - 1 - e) : e;
    T v = y[j];
#pragma unroll
    for (int m = K - 1; m >= 0; --m) v = fma(W.a[m], s[m], v);
#pragma unroll
    for (int m = K - 1; m > 0; --m) s[m] = s[m - 1];
    s[0] = v;
    y[j] = v;
  }
  // 2. publish the end state, then gather the carry from the D chunks before
  //    this one in processing order (periodic in the thread index)
#pragma unroll
  for (int m = 0; m < K; ++m) pub[tid * K + m] = s[m];
  __syncthreads();
  int src = REV ? (tid + 1 == NT ? 0 : tid + 1) : (tid == 0 ? NT - 1 : tid - 1);
  T E[K];
#pragma unroll
  for (int m = 0; m < K; ++m) E[m] = pub[src * K + m];
  for (int d = 1; d < W.D; ++d) {
    src = REV ? (src + 1 == NT ? 0 : src + 1) : (src == 0 ? NT - 1 : src - 1);
    T z[K];
#pragma unroll
    for (int m = 0; m < K; ++m) z[m] = pub[src * K + m];
    const ConstPtr<T> Hd = W.tab + (d - 1) * K * K;
#pragma unroll
    for (int r = 0; r < K; ++r) {
      T acc = E[r];
#pragma unroll
      for (int c = 0; c < K; ++c) acc = fma(Hd[r * K + c], z[c], acc);
      E[r] = acc;
    }
  }
  // 3. homogeneous correction of the first hc points
  const ConstPtr<T> C = W.tab + (W.D - 1) * K * K;
#pragma unroll
  for (int e = 0; e < L; ++e) {
    if (e < W.hc) {  // uniform
      const int j = REV ? (L - 1 - e) : e;
      T v = y[j];
#pragma unroll
      for (int m = 0; m < K; ++m) v = fma(C[e * K + m], E[m], v);
      y[j] = v;
    }
  }
}

// Operator constants of the windowed kernel.
template <int KF, int KB, class T>
struct WinOp {
  int repeat;
  int ncoef;
  const double *coef;  // OP_POLY_W: Horner coefficients in G = B^{-1} F^{-1} (1/C folded in)
  T top;
  int width, off;      // OP_SLC: interpolation taps (1/C folded in) and their start offset
  T w[MAXTAPS];
  WinDir<KF, T> f;
  WinDir<KB, T> b;
};

// y <- G y = B^{-1} F^{-1} y.  pub0/pub1: the published-state areas.  With no
// anti-causal factor the causal recurrence alternates between them (flip), so
// that a recurrence never overwrites words another thread has yet to read.
template <int L, int KF, int KB, class T>
__device__ __forceinline__ void win_solve(T (&y)[L], const WinOp<KF, KB, T> &R, T *pub0, T *pub1, int &flip,
                                          int tid, int NT) {
  if constexpr (KF > 0) {
    win_rec<L, KF, false>(y, R.f, flip ? pub1 : pub0, tid, NT);
    if constexpr (KB == 0) flip ^= 1;
  }
  if constexpr (KB > 0) win_rec<L, KB, true>(y, R.b, pub1, tid, NT);
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
  const WinLds lo = win_lds(KIND, nx, NT, KW, (int)sizeof(T));
  T *sm = reinterpret_cast<T *>(smem);
  T *vec = sm;  // OP_SLC: the padded vector
  T *pub0 = sm + lo.pub0, *pub1 = sm + lo.pub1;
  double *red = smem + lo.red;

  WinOp<KF, KB, T> R;
  R.repeat = op.repeat;
  R.ncoef = op.ncoef;
  R.coef = op.wcoef;
  R.top = KIND == OP_POLY_W ? (T)op.wcoef[op.ncoef - 1] : T(0);
  if (KIND == OP_SLC) {
    R.width = op.sl_l + op.sl_r + 1;
    R.off = op.sl_K + op.sl_l;
#pragma unroll
    for (int t = 0; t < MAXTAPS; ++t) R.w[t] = (T)(op.slw[t] * op.cinv);
  }
  win_dir_load<KF, T>(R.f, op.fw);
  win_dir_load<KB, T>(R.b, op.bw);

  int flip = 0;
  run_chain<L, T>(pa, nx, L, red, [&](T (&u)[L]) {
    const int base = tid * L;
    for (int rep = 0; rep < R.repeat; ++rep) {
      T y[L];
      if (KIND == OP_SLC) {
        __syncthreads();  // every thread has finished the previous gather
        chunk_to_lds<L>(vec, base, L, u);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < L; ++j) y[j] = T(0);
        window_combine<L>(vec, wrap_lo(base - R.off, nx), L, R.width, nx, R.w, y);
        if (lo.alias) __syncthreads();  // the published states reuse the vector's words
        win_solve<L, KF, KB>(y, R, pub0, pub1, flip, tid, NT);
      } else {  // OP_POLY_W: Phi u = sum_i wcoef[i] G^i u by Horner
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
  });
}
