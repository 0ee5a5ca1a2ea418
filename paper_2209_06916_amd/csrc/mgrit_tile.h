// Level-0 explicit relaxation with wavefront tiles (included inside
// namespace mgrit::{anonymous} by the per-width translation units).
#pragma once

// ---------------------------------------------------------------------------
// Level-0 explicit relaxation, one wavefront per (CF-interval, spatial tile).
// Lane l holds the P consecutive points starting at x0 - HL + l P (periodic).
// Each application of Z = -c L_p reads SL points from the left neighbour lane
// and SR from the right one, moved by whole-wavefront DPP shifts; lane 0's
// left and lane 63's right inputs are zero, which only invalidates points
// inside the halo.  No LDS, no barriers.
// ---------------------------------------------------------------------------
// Whole-wavefront shift of a double by one lane: WAVE_SHR1 (0x138) gives lane
// l the value of lane l-1, WAVE_SHL1 (0x130) that of lane l+1; the lane
// without a source reads 0.
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffff), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
template <int CTRL>
__device__ __forceinline__ float wave_shift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// 16 bytes of consecutive elements
template <class T>
struct Vec16 {
  typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
  static constexpr int N = 16 / (int)sizeof(T);
};

// x[0..P) = row[g .. g+P) (periodic); 16-byte loads when the run is
// contiguous and aligned.
template <int P, class T>
__device__ __forceinline__ void load_run(const T *__restrict__ row, int g, int nx, T (&x)[P]) {
  const T *p = row + g;
  constexpr int N = Vec16<T>::N;
  if (P % N == 0 && g + P <= nx && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
    const typename Vec16<T>::type *pv = reinterpret_cast<const typename Vec16<T>::type *>(p);
#pragma unroll
    for (int k = 0; k < P / N; ++k) {
      const typename Vec16<T>::type t = pv[k];
#pragma unroll
      for (int e = 0; e < N; ++e) x[N * k + e] = t[e];
    }
  } else {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      x[k] = row[g];
      g = next_periodic(g, nx);
    }
  }
}
// COMP: every step is one application of the explicit step written out as a
// single stencil, u_k <- sum_t ctaps[t] u_{k+t-SL} (SL, SR: its extents);
// otherwise R(Z) u by Horner, (ncoef - 1) applications of Z (extents SL, SR).
template <int P, int SL, int SR, bool COMP, class T>
__global__ void __launch_bounds__(256) tile_kernel(const LevelDesc *__restrict__ desc, TileGeom tg, TileArgsT<T> ta) {
  static_assert(!COMP || (SL <= P && SR <= P && SL + SR + 1 <= MAXCTAPS), "written-out step wider than a lane pair");
  if (ta.stop && *ta.stop) return;  // the solve has already stopped
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

  // coefficients -> registers (the Horner loop below is unrolled over the
  // largest stage count with uniform guards, so no stage reloads them)
  const int ncoef = op.ncoef;
  T taps[SL + SR + 1];
#pragma unroll
  for (int t = 0; t <= SL + SR; ++t) taps[t] = (T)(COMP ? op.ctaps[t] : op.taps[t]);
  T cf[MAXCOEF];
#pragma unroll
  for (int i = 0; i < MAXCOEF; ++i) cf[i] = (T)op.coef[i];
  const T top = (T)op.coef[ncoef - 1];

  // this lane's first global position (periodic) and its local index
  const int li0 = lane * P;              // local index of point 0 of this lane
  int g0 = x0 - tg.HL + li0;             // global position, may be outside [0, nx)
  g0 %= nx;
  if (g0 < 0) g0 += nx;

  T u[P];
  load_run<P>(ta.cin + b * nxl, g0, nx, u);
  // output window of this lane: local indices [HL, HL + tw)
  const int lo = tg.HL - li0, hi = tg.HL + tw - li0;  // k in [lo, hi) is output
  const bool whole = lo <= 0 && hi >= P && g0 + P <= nx;  // all P points are output, no wrap

  auto store_out = [&](T *row, const T (&v)[P]) {
    T *p = row + g0;
    constexpr int N = Vec16<T>::N;
    if (P % N == 0 && whole && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
      typename Vec16<T>::type *pv = reinterpret_cast<typename Vec16<T>::type *>(p);
#pragma unroll
      for (int k = 0; k < P / N; ++k) {
        typename Vec16<T>::type t;
#pragma unroll
        for (int e = 0; e < N; ++e) t[e] = v[N * k + e];
        pv[k] = t;
      }
      return;
    }
    int g = g0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      if (k >= lo && k < hi) row[g] = v[k];
      g = next_periodic(g, nx);
    }
  };

  if (ta.mode == MODE_PASS_A && b == 0) store_out(ta.cout, u);
  if (ta.mode == MODE_FINAL_F) store_out(ta.out + (b * ta.m) * nxl, u);

  // FINAL_F computes the m-1 F-points (the C-point comes from the iterate);
  // SEQ advances one block of m steps of sequential time-stepping (nint = 1)
  // and writes every step.
  const int nsteps = (ta.mode == MODE_FINAL_F) ? ta.m - 1 : ta.m;
  const bool store_steps = ta.mode == MODE_FINAL_F || ta.mode == MODE_SEQ;
  // one step u <- R(Z) u
  auto advance = [&]() {
    if constexpr (COMP) {
      T lh[SL > 0 ? SL : 1], rh[SR > 0 ? SR : 1];
#pragma unroll
      for (int q = 0; q < SL; ++q) lh[q] = wave_shift<0x138>(u[P - SL + q]);
#pragma unroll
      for (int q = 0; q < SR; ++q) rh[q] = wave_shift<0x130>(u[q]);
      T yn[P];
#pragma unroll
      for (int k = 0; k < P; ++k) {
        T acc = T(0);
#pragma unroll
        for (int t = 0; t <= SL + SR; ++t) {
          const int src = k + t - SL;
          const T v = src < 0 ? lh[(src + SL) < 0 ? 0 : (src + SL)]
                              : (src >= P ? rh[(src - P) < SR ? (src - P) : 0] : u[src < P ? src : 0]);
          acc = t == 0 ? taps[0] * v : fma(taps[t], v, acc);
        }
        yn[k] = acc;
      }
#pragma unroll
      for (int k = 0; k < P; ++k) u[k] = yn[k];
    } else {
      T y[P];
#pragma unroll
      for (int k = 0; k < P; ++k) y[k] = top * u[k];
#pragma unroll
      for (int i = MAXCOEF - 2; i >= 0; --i) {
        if (i > ncoef - 2) continue;  // uniform
        T lh[SL > 0 ? SL : 1], rh[SR > 0 ? SR : 1];
#pragma unroll
        for (int q = 0; q < SL; ++q) lh[q] = wave_shift<0x138>(y[P - SL + q]);
#pragma unroll
        for (int q = 0; q < SR; ++q) rh[q] = wave_shift<0x130>(y[q]);
        const T ci = cf[i];
        T yn[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
          T acc = ci * u[k];
#pragma unroll
          for (int t = 0; t <= SL + SR; ++t) {
            const int src = k + t - SL;
            const T v = src < 0 ? lh[(src + SL) < 0 ? 0 : (src + SL)]
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
    }
  };
  // u += g_{n-1} at level point n (every point of the tile, halo included)
  auto add_rhs = [&](int j) {
    if (ta.g) {
      T gv[P];
      load_run<P>(ta.g + (b * ta.m + j - 1) * nxl, g0, nx, gv);
#pragma unroll
      for (int k = 0; k < P; ++k) u[k] += gv[k];
    }
  };
  for (int j = 1; j < nsteps; ++j) {
    advance();
    add_rhs(j);
    if (store_steps) store_out(ta.out + (b * ta.m + j) * nxl, u);
  }
  // the last step; pass B first requests the next C-point, whose load then
  // overlaps the step
  T cn[P];
  if (ta.mode == MODE_PASS_B) load_run<P>(ta.cin + (b + 1) * nxl, g0, nx, cn);
  if (nsteps > 0) {
    advance();
    add_rhs(nsteps);
    if (store_steps) store_out(ta.out + (b * ta.m + nsteps) * nxl, u);
  }

  if (ta.mode == MODE_PASS_A) {
    store_out(ta.cout + (b + 1) * nxl, u);
  } else if (ta.mode == MODE_PASS_B) {
    T rv[P];
    double ss = 0.0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      rv[k] = u[k] - cn[k];
      if (k >= lo && k < hi) ss = fma((double)rv[k], (double)rv[k], ss);
    }
    store_out(ta.r + b * nxl, rv);
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) ss += __shfl_down(ss, d, WAVE);
    if (lane == 0) ta.normpart[item] = ss;
  } else if (ta.mode == MODE_FINAL_F && b == ta.nint - 1) {
    T c[P];
    load_run<P>(ta.cin + ta.nint * nxl, g0, nx, c);
    store_out(ta.out + (ta.nint * ta.m) * nxl, c);
  }
}

template <int P, class T>
hipError_t launch_tiles_p(const LevelDesc *desc, const TileGeom &tg, const TileArgsT<T> &ta, hipStream_t stream) {
  const int64_t items = ta.nint * tg.ntiles;
  const dim3 grid((unsigned)((items + 3) / 4)), block(256);
  if (tg.comp) {
    // written-out explicit steps: ERK3 + U3 (3 stages x (2, 1))
    if constexpr (P >= 8) {
      if (tg.sl == 6 && tg.sr == 3) {
        hipLaunchKernelGGL((tile_kernel<P, 6, 3, true, T>), grid, block, 0, stream, desc, tg, ta);
        return hipGetLastError();
      }
    }
    return hipErrorInvalidValue;
  }
  switch (tg.sl * 4 + tg.sr) {
    case 1 * 4 + 0: hipLaunchKernelGGL((tile_kernel<P, 1, 0, false, T>), grid, block, 0, stream, desc, tg, ta); break;
    case 2 * 4 + 0: hipLaunchKernelGGL((tile_kernel<P, 2, 0, false, T>), grid, block, 0, stream, desc, tg, ta); break;
    case 2 * 4 + 1: hipLaunchKernelGGL((tile_kernel<P, 2, 1, false, T>), grid, block, 0, stream, desc, tg, ta); break;
    case 3 * 4 + 1: hipLaunchKernelGGL((tile_kernel<P, 3, 1, false, T>), grid, block, 0, stream, desc, tg, ta); break;
    case 3 * 4 + 2: hipLaunchKernelGGL((tile_kernel<P, 3, 2, false, T>), grid, block, 0, stream, desc, tg, ta); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
