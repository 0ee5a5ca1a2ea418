// gfx950 kernel for the coarse-level time step of MGRIT (Sec. 2.2 with the
// corrected semi-Lagrangian operator, eqs. MOL-SL-corrected and
// MOL-SL-corrected-multilevel) on vectors of 64 L NW points: L = 16 or 8
// with NW = 1, 2, 4, 8 wavefronts, and one wavefront with L = 4; in float64,
// and in float32 for the inner solves of mixed precision.
#include "mgrit_internal.h"

namespace mgrit {

namespace {

#include "mgrit_device.h"

// ---------------------------------------------------------------------------
// Coarse time step Psi = T^{-1} S (eq. MOL-SL-corrected-multilevel) for
// nx = 64 L NW: L points per lane, NW full wavefronts, W interpolation taps,
// order-K forward and backward recurrences.  Per step: one barrier after the
// vector is written to LDS, one per recurrence.  After a recurrence's
// wavefront totals are published, every wavefront folds them and the
// periodic wrap into its own carry (a short chain computed redundantly), so
// no thread waits for a serial one.  The scan's lane-dependent matrix powers
// are loaded into registers once per launch for K <= 2; the matrices every
// lane of a wavefront shares are read through the scalar cache from device
// memory, which keeps them out of LDS and out of vector registers.
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

// The same moves for either precision (a float is one 32-bit move).
template <int CTRL>
__device__ __forceinline__ double dpp_t(double v) {
  return dpp_d<CTRL>(v);
}
template <int CTRL>
__device__ __forceinline__ float dpp_t(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ double readlane_t(double v, int lane) { return readlane_d(v, lane); }
__device__ __forceinline__ float readlane_t(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

template <int K, class TP, class E>
__device__ __forceinline__ void ld_mat(TP p, E (&M)[K * K]) {
#pragma unroll
  for (int i = 0; i < K * K; ++i) M[i] = p[i];
}

// acc += M x (M row-major K x K)
template <int K, class E>
__device__ __forceinline__ void mv_acc(const E (&M)[K * K], const E (&x)[K], E (&acc)[K]) {
#pragma unroll
  for (int r = 0; r < K; ++r) {
    E s = acc[r];
#pragma unroll
    for (int c = 0; c < K; ++c) s = fma(M[r * K + c], x[c], s);
    acc[r] = s;
  }
}

// Lane-dependent matrices of one recurrence direction: H^{lr} (lr = position
// in the 16-lane row, processing order), H^{vl} (position in the wavefront)
// and H^{64 vw} (vw = wavefront position).  HOIST keeps them in registers;
// otherwise they are read from the LDS table where used.
template <int K, bool HOIST, class E>
struct LaneMats {
  static constexpr int N = HOIST ? K * K : 1;
  E lr_[N], vl_[N], vw_[N];
  const E *tab;
  int lr, vl, vw;
  // t: the LDS copy of the table (read in the loop when not hoisted); src:
  // the same table in device memory (hoisted values are loaded from there, so
  // they do not wait for the LDS copy)
  __device__ __forceinline__ void init(const E *t, const E *src, int lr0, int vl0, int vw0) {
    tab = t;
    lr = lr0;
    vl = vl0;
    vw = vw0;
    if constexpr (HOIST) {
      ld_mat<K>(src + lr * K * K, lr_);
      ld_mat<K>(src + vl * K * K, vl_);
      ld_mat<K>(src + (TAB_HWAVE + vw) * K * K, vw_);
    }
  }
  __device__ __forceinline__ void get(int which, E (&M)[K * K]) const {
    if constexpr (HOIST) {
      const E *src = which == 0 ? lr_ : (which == 1 ? vl_ : vw_);
#pragma unroll
      for (int i = 0; i < K * K; ++i) M[i] = src[i];
    } else {
      const int idx = which == 0 ? lr : (which == 1 ? vl : TAB_HWAVE + vw);
      ld_mat<K>(tab + idx * K * K, M);
    }
  }
};

// One Kogge-Stone step inside 16-lane rows: add H^D times the state D lanes
// back in processing order (row_shr forward, row_shl backward; lanes without
// such a neighbour receive 0 and keep their value).
template <int K, bool REV, int D, class E>
__device__ __forceinline__ void row_step(E (&inc)[K], const E (&M)[K * K]) {
  E o[K];
#pragma unroll
  for (int m = 0; m < K; ++m) o[m] = REV ? dpp_t<0x100 + D>(inc[m]) : dpp_t<0x110 + D>(inc[m]);
  mv_acc<K>(M, o, inc);
}

// The wave-uniform matrices of one direction's in-row scan: M^{L/2} and the
// chunk transfer powers H, H^2, H^4, H^8, H^16.  The caller requests them
// well ahead of the scan (their scalar loads then arrive while other work
// runs) and passes them in.
template <int K, class E>
struct ScanMats {
  E h[K * K], m1[K * K], m2[K * K], m4[K * K], m8[K * K], m16[K * K];
  template <class TP>
  __device__ __forceinline__ void load(TP tab) {
    ld_mat<K>(tab + TAB_HHALF * K * K, h);
    ld_mat<K>(tab + K * K, m1);
    ld_mat<K>(tab + 2 * K * K, m2);
    ld_mat<K>(tab + 4 * K * K, m4);
    ld_mat<K>(tab + 8 * K * K, m8);
    ld_mat<K>(tab + 16 * K * K, m16);
  }
};

// Periodic recurrence x_i += sum_m a[m] x_{i-1-m} (REV: x_{i+1+m}) over the
// workgroup's 16-point chunks; pre_barrier() runs just before the barrier,
// post_barrier() right after it, pre_corr() once the carries are folded
// (after the last LDS read of the published totals).
template <int L, int K, int NW, bool REV, bool HOIST, class E, class TP, class Hook, class PostHook, class CorrHook>
__device__ __forceinline__ void lean_rec(E (&x)[L], const E (&a)[K], TP tab,
                                         const LaneMats<K, HOIST, E> &lm, const ScanMats<K, E> &sm, E *Q,
                                         Hook pre_barrier, PostHook post_barrier, CorrHook pre_corr) {
  constexpr int KK = K * K;
  constexpr int LH = L / 2;  // two interleaved sub-chains per lane
  const int vl = lm.vl, vw = lm.vw, vrow = vl >> 4;
  const auto &Mh = sm.h, &M1 = sm.m1, &M2 = sm.m2, &M4 = sm.m4, &M8 = sm.m8, &M16 = sm.m16;
  // zero-state passes of both halves (processing order: REV walks down)
  E sa[K], sb[K];
#pragma unroll
  for (int m = 0; m < K; ++m) sa[m] = sb[m] = E(0);
#pragma unroll
  for (int e = 0; e < LH; ++e) {
    const int ja = REV ? (L - 1 - e) : e;
    const int jb = REV ? (LH - 1 - e) : (LH + e);
    E ya = x[ja], yb = x[jb];
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
  E q[K];
#pragma unroll
  for (int m = 0; m < K; ++m) q[m] = sb[m];
  mv_acc<K>(Mh, sa, q);

  // inclusive scan inside 16-lane rows
  E inc[K];
#pragma unroll
  for (int m = 0; m < K; ++m) inc[m] = q[m];
  row_step<K, REV, 1>(inc, M1);
  row_step<K, REV, 2>(inc, M2);
  row_step<K, REV, 4>(inc, M4);
  row_step<K, REV, 8>(inc, M8);
  // exclusive value in the row, then the row carries (uniform over the
  // wavefront): ex = ex_row + H^{lr} C_row
  E ex[K], C1[K], C2[K], C3[K];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    ex[m] = REV ? dpp_t<0x101>(inc[m]) : dpp_t<0x111>(inc[m]);
    C1[m] = readlane_t(inc[m], REV ? 48 : 15);
    C2[m] = readlane_t(inc[m], REV ? 32 : 31);
    C3[m] = readlane_t(inc[m], REV ? 16 : 47);
  }
  mv_acc<K>(M16, C1, C2);
  mv_acc<K>(M16, C2, C3);
  // the carry into this lane's row (zero in row 0), selected with 0/1
  // weights: a data-dependent select here would be lowered to branches
  const E s1 = vrow == 1 ? E(1) : E(0), s2 = vrow == 2 ? E(1) : E(0), s3 = vrow == 3 ? E(1) : E(0);
  E cr[K];
#pragma unroll
  for (int m = 0; m < K; ++m) cr[m] = fma(s3, C3[m], fma(s2, C2[m], s1 * C1[m]));
  E P[KK];
  lm.get(0, P);
  mv_acc<K>(P, cr, ex);

  // publish the wavefront total (last lane: q + H ex) and, from the last
  // chunk of the vector, its exclusive state and zero-state total
  if (vl == WAVE - 1) {
    E tot[K];
#pragma unroll
    for (int m = 0; m < K; ++m) tot[m] = q[m];
    mv_acc<K>(M1, ex, tot);
#pragma unroll
    for (int m = 0; m < K; ++m) Q[vw * K + m] = tot[m];
    if (vw == NW - 1) {
#pragma unroll
      for (int m = 0; m < K; ++m) {
        Q[NW * K + m] = ex[m];
        Q[(NW + 1) * K + m] = q[m];
      }
    }
  }
  // the fold's matrices, requested before the barrier so that they arrive
  // while it waits
  E Mw[KK], Mw1[KK], Mlast[KK], Mwrap[KK];
  ld_mat<K>(tab + WAVE * KK, Mw);
  ld_mat<K>(tab + (WAVE - 1) * KK, Mw1);
  ld_mat<K>(tab + TAB_HLAST * KK, Mlast);
  ld_mat<K>(tab + TAB_WWRAP * KK, Mwrap);
  pre_barrier();
  __syncthreads();
  post_barrier();

  // zero-start carries X_w entering each wavefront; keep X_vw and X_{NW-1}
  E X[K], Xv[K];
#pragma unroll
  for (int m = 0; m < K; ++m) X[m] = Xv[m] = E(0);
#pragma unroll
  for (int w2 = 0; w2 < NW - 1; ++w2) {
    E nxt[K];
#pragma unroll
    for (int m = 0; m < K; ++m) nxt[m] = Q[w2 * K + m];
    mv_acc<K>(Mw, X, nxt);
#pragma unroll
    for (int m = 0; m < K; ++m) {
      X[m] = nxt[m];
      Xv[m] = (vw == w2 + 1) ? nxt[m] : Xv[m];
    }
  }
  // periodic wrap: state entering point 0, s0 = Wwrap (Hlast Ex + q_last),
  // Ex the last chunk's exclusive state
  E Ex[K], tq[K], s0[K];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    Ex[m] = Q[NW * K + m];
    tq[m] = Q[(NW + 1) * K + m];
    s0[m] = E(0);
  }
  mv_acc<K>(Mw1, X, Ex);
  mv_acc<K>(Mlast, Ex, tq);
  mv_acc<K>(Mwrap, tq, s0);
  // carry into this wavefront, this lane, and both halves of its chunk
  lm.get(2, P);
  mv_acc<K>(P, s0, Xv);
  E ta[K], tb[K];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    ta[m] = ex[m];
    tb[m] = sa[m];
  }
  lm.get(1, P);
  mv_acc<K>(P, Xv, ta);
  mv_acc<K>(Mh, ta, tb);
  pre_corr();
  // homogeneous corrections
#pragma unroll
  for (int e = 0; e < LH; ++e) {
    const int ja = REV ? (L - 1 - e) : e;
    const int jb = REV ? (LH - 1 - e) : (LH + e);
    E ha = E(0), hb = E(0);
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

// Coalesced row segments of 16 bytes (SEG_N elements): thread t of NTH owns
// the segments t + NTH q, q < L / SEG_N.
template <class E>
struct alignas(16) Seg {
  E e[16 / sizeof(E)];
};
template <class E>
constexpr int SEG_N = 16 / sizeof(E);
template <int L, int NTH, class E>
__device__ __forceinline__ void load_segs(const E *__restrict__ row, Seg<E> (&seg)[L / SEG_N<E>]) {
  const Seg<E> *r = reinterpret_cast<const Seg<E> *>(row);
#pragma unroll
  for (int q = 0; q < L / SEG_N<E>; ++q) seg[q] = r[threadIdx.x + NTH * q];
}

// One pass (PassMode) of one CF-interval b with the coarse step of `op`.
// LDS: v the padded vector, tab_f / tab_b the scan tables, qf / qb the
// wavefront totals, red the reduction scratch.  hsrc_f / hsrc_b: where the
// lane-dependent powers are loaded from.
// prologue() runs once the first loads are in flight; false ends the pass.
template <int W, int K, int L, int NW, class E, class Prologue>
__device__ __forceinline__ void lean_pass(const StepOp &op, const PassArgsT<E> &pa, int64_t b, E *v, E *tab_f,
                                          E *tab_b, const E *hsrc_f, const E *hsrc_b, E *qf, E *qb, double *red,
                                          Prologue prologue) {
  constexpr int NTH = WAVE * NW;
  constexpr int NX = L * NTH;
  constexpr bool HOIST = K <= 2;
  constexpr int SN = SEG_N<E>;

  // interpolation weights with the 1/C of the factorisation folded in
  E w[W], af[K], ab[K];
  const double cinv = op.cinv;
#pragma unroll
  for (int t = 0; t < W; ++t) w[t] = (E)(op.slw[t] * cinv);
#pragma unroll
  for (int m = 0; m < K; ++m) {
    af[m] = (E)op.fw.a[m];
    ab[m] = (E)op.bw.a[m];
  }
  const int tid = threadIdx.x;
  const int base = tid * L;
  const int64_t nxl = NX;
  const int m = pa.m;
  const int mode = pa.mode;
  const int nsteps = (mode == MODE_POST_F) ? m - 1 : m;  // PASS_A, PASS_B, SEQ, APPLY: m
  const int64_t row0 = (mode == MODE_SEQ) ? 0 : b;
  // start vector (loads issued before the table copy so their latencies overlap)
  E u[L];
  if (pa.zero_init) {
#pragma unroll
    for (int j = 0; j < L; ++j) u[j] = E(0);
  } else {
    load_chunk<L>(pa.cin + row0 * nxl, base, L, u);
  }
  const int lane = tid & (WAVE - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // the wave-uniform scan matrices are read through the scalar cache from
  // the device copy of the tables (constant address space)
  typedef const __attribute__((address_space(4))) E *ConstTab;
  const ConstTab ctf = (ConstTab)op.fw.tab, ctb = (ConstTab)op.bw.tab;
  LaneMats<K, HOIST, E> lmf, lmb;
  lmf.init(tab_f, hsrc_f, lane & 15, lane, wave);
  lmb.init(tab_b, hsrc_b, (WAVE - 1 - lane) & 15, WAVE - 1 - lane, NW - 1 - wave);
  if (!prologue()) return;

  int start = base - (op.sl_K + op.sl_l) % NX;
  if (start < 0) start += NX;
  if (mode == MODE_PASS_A && b == 0) store_chunk<L>(pa.cout, base, L, u);
  const bool add_g = pa.g && mode != MODE_APPLY;
  const E gsc = add_g ? E(1) : E(0);
  // read the right-hand-side chunk right after the backward barrier (its
  // latency then overlaps the fold); at 8 wavefronts the registers it holds
  // meanwhile would spill, so it is read at the end there
  constexpr bool EARLY_G = NW < 8;
  const bool add_parent = mode == MODE_POST_F || (mode == MODE_SEQ && pa.parent);
  if (mode == MODE_POST_F) {
    E pv[L];
    load_chunk<L>(pa.parent + (b * m) * nxl, base, L, pv);
#pragma unroll
    for (int j = 0; j < L; ++j) pv[j] += u[j];
    store_chunk<L>(pa.parent + (b * m) * nxl, base, L, pv);
  }

  // parent[prow] += the vector in v, coalesced, with the row's segments in pseg
  auto parent_update = [&](int64_t prow, const Seg<E> (&pseg)[L / SN]) {
    Seg<E> *p2 = reinterpret_cast<Seg<E> *>(pa.parent + prow * nxl);
#pragma unroll
    for (int q = 0; q < L / SN; ++q) {
      const int i = SN * (tid + NTH * q);
      Seg<E> r = pseg[q];
#pragma unroll
      for (int c = 0; c < SN; ++c) r.e[c] += v[padix(i + c)];
      p2[tid + NTH * q] = r;
    }
  };

  // One LDS vector serves every step.  Each thread writes only its own chunk
  // of it at the start of a step and reads only its own chunk at the end; the
  // cross-thread reads (gather, parent update) precede the forward
  // recurrence's barrier and the cross-thread writes (right-hand side, in the
  // backward recurrence's pre-barrier hook) follow it.  Each thread reads its
  // chunk of the right-hand side back right after the backward recurrence's
  // barrier, so those reads overlap the carry fold and the corrections.
  // pseg: the pending parent row's segments; in the last step it is refilled
  // with what the epilogue needs (the next parent row, or pass B's C'_{k+1})
  // so that load overlaps the step.
  // gseg: the right-hand-side row of the coming step, loaded a whole step
  // ahead (right after the previous row is consumed) so its latency is hidden.
  int64_t pend = -1;  // parent row whose update waits for the next LDS copy
  Seg<E> pseg[L / SN], gseg[L / SN];
  const unsigned long long ctf_bits = (unsigned long long)ctf, ctb_bits = (unsigned long long)ctb;
  const unsigned tf_lo = __builtin_amdgcn_readfirstlane((unsigned)ctf_bits);
  const unsigned tf_hi = __builtin_amdgcn_readfirstlane((unsigned)(ctf_bits >> 32));
  const unsigned tb_lo = __builtin_amdgcn_readfirstlane((unsigned)ctb_bits);
  const unsigned tb_hi = __builtin_amdgcn_readfirstlane((unsigned)(ctb_bits >> 32));
  if (mode == MODE_PASS_B && nsteps == 0) load_segs<L, NTH>(pa.cin + (b + 1) * nxl, pseg);
  if (add_g && nsteps >= 1) load_segs<L, NTH>(pa.g + ((mode == MODE_SEQ) ? 0 : b * m) * nxl, gseg);
  for (int j = 1; j <= nsteps; ++j) {
    const int64_t n = (mode == MODE_SEQ) ? (int64_t)j : b * m + j;  // level point index
    // The scan matrices are read afresh in every step: an opaque copy of the
    // table pointers keeps their scalar loads inside the step, where they are
    // short-lived, instead of being hoisted out of the loop and spilled.
    unsigned tfl = tf_lo, tfh = tf_hi, tbl = tb_lo, tbh = tb_hi;
    asm volatile("" : "+s"(tfl), "+s"(tfh), "+s"(tbl), "+s"(tbh));
    const ConstTab tf = (ConstTab)(((unsigned long long)tfh << 32) | tfl);
    const ConstTab tb = (ConstTab)(((unsigned long long)tbh << 32) | tbl);
    if (pend >= 0) load_segs<L, NTH>(pa.parent + pend * nxl, pseg);
    if (mode == MODE_PASS_B && j == nsteps) load_segs<L, NTH>(pa.cin + (b + 1) * nxl, pseg);
    ScanMats<K, E> smf, smb;
    smf.load(tf);  // arrives while the vector is written and the barrier waits
#pragma unroll
    for (int jj = 0; jj < L; ++jj) v[padix(base + jj)] = u[jj];
    __syncthreads();
    if (pend >= 0) parent_update(pend, pseg);
    if (add_parent && j == nsteps) load_segs<L, NTH>(pa.parent + n * nxl, pseg);
    E y[L];
#pragma unroll
    for (int jj = 0; jj < L; ++jj) y[jj] = E(0);
#pragma unroll
    for (int e = 0; e < L + W - 1; ++e) {
      int idx = start + e;
      idx = idx >= NX ? idx - NX : idx;
      const E val = v[padix(idx)];
#pragma unroll
      for (int t = 0; t < W; ++t) {
        const int jj = e - t;
        if (jj >= 0 && jj < L) y[jj] = fma(w[t], val, y[jj]);
      }
    }
    E gch[L];
    lean_rec<L, K, NW, false>(y, af, tf, lmf, smf, qf, [] {}, [] {}, [&] {
      // the backward scan's matrices: issued here (the scheduling barrier
      // keeps the compiler from sinking them to their use), they arrive
      // during the corrections and the backward zero-state pass
      smb.load(tb);
      __builtin_amdgcn_sched_barrier(0);
    });
    lean_rec<L, K, NW, true>(
        y, ab, tb, lmb, smb, qb,
        [&] {
          if (add_g) {  // g_n -> v in coalesced segments, then fetch the next step's row
#pragma unroll
            for (int q = 0; q < L / SN; ++q) {
              const int i = SN * (tid + NTH * q);
#pragma unroll
              for (int c = 0; c < SN; ++c) v[padix(i + c)] = gseg[q].e[c];
            }
            if (j < nsteps) load_segs<L, NTH>(pa.g + n * nxl, gseg);
          }
        },
        [&] {  // this thread's chunk of g_n (the vector itself without a right-hand side)
          if constexpr (EARLY_G) {
#pragma unroll
            for (int jj = 0; jj < L; ++jj) gch[jj] = v[padix(base + jj)];
          }
        },
        [] {});
    if constexpr (!EARLY_G) {
#pragma unroll
      for (int jj = 0; jj < L; ++jj) gch[jj] = v[padix(base + jj)];
    }
    // u = y + g, or y: fma with a 0/1 weight is exact either way (the chunk
    // read is finite), and no branch lets the reads sink past the corrections
#pragma unroll
    for (int jj = 0; jj < L; ++jj) u[jj] = fma(gsc, gch[jj], y[jj]);
    pend = add_parent ? n : -1;
  }
  if (pend >= 0) {  // the last step's parent update (row prefetched into pseg)
#pragma unroll
    for (int jj = 0; jj < L; ++jj) v[padix(base + jj)] = u[jj];
    __syncthreads();
    parent_update(pend, pseg);
  }

  if (mode == MODE_PASS_A) {
    store_chunk<L>(pa.cout + (b + 1) * nxl, base, L, u);
  } else if (mode == MODE_PASS_B) {
    // r = u - C'_{k+1} (C'_{k+1} prefetched into pseg), in coalesced segments
#pragma unroll
    for (int jj = 0; jj < L; ++jj) v[padix(base + jj)] = u[jj];
    __syncthreads();
    Seg<E> *r2 = reinterpret_cast<Seg<E> *>(pa.r + b * nxl);
    double ss = 0.0;  // the partial norms are float64 in both precisions
#pragma unroll
    for (int q = 0; q < L / SN; ++q) {
      const int i = SN * (tid + NTH * q);
      Seg<E> rr;
#pragma unroll
      for (int c = 0; c < SN; ++c) {
        rr.e[c] = v[padix(i + c)] - pseg[q].e[c];
        ss = fma((double)rr.e[c], (double)rr.e[c], ss);
      }
      r2[tid + NTH * q] = rr;
    }
    const double tot = block_sum(ss, red);
    if (tid == 0) pa.normpart[b] = tot;
  } else if (mode == MODE_POST_F) {
    if (b == pa.nint - 1) {
      load_chunk<L>(pa.cin + pa.nint * nxl, base, L, u);
      E *row = pa.parent + (pa.nint * m) * nxl;
      E pv[L];
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

// One launch per pass (float64, or float32 for the inner solves of mixed
// precision).  The LDS holds the elements at the offsets of lean_lds_offsets
// counted in E and the float64 reduction scratch at its float64 offset,
// which lies past the float32 data.
template <int W, int K, int L, int NW, class E>
__global__ void __launch_bounds__(WAVE * NW) slc_kernel(const LevelDesc *__restrict__ desc, PassArgsT<E> pa) {
  extern __shared__ double smem[];
  constexpr LeanLds lo = lean_lds_offsets(L * WAVE * NW, K);
  const StepOp &op = desc->op;
  E *sm = reinterpret_cast<E *>(smem);
  E *tab_f = sm + lo.tab_f;
  E *tab_b = sm + lo.tab_b;
  const E *gtab_f = static_cast<const E *>(op.fw.tab), *gtab_b = static_cast<const E *>(op.bw.tab);
  lean_pass<W, K, L, NW>(op, pa, blockIdx.x, sm, tab_f, tab_b, gtab_f, gtab_b, sm + lo.qf, sm + lo.qb,
                      smem + lo.red, [&] {
                        // Scan tables to LDS.  No barrier here: the first step's
                        // barrier (after the vector is written to LDS) comes
                        // before any read of them.
                        for (int i = threadIdx.x; i < RTAB_ALL * K * K; i += WAVE * NW) {
                          tab_f[i] = gtab_f[i];
                          tab_b[i] = gtab_b[i];
                        }
                        return !(pa.stop && *pa.stop);  // the solve has already stopped (uniform)
                      });
}

// ---------------------------------------------------------------------------
// Persistent coarse V-cycle.  Every workgroup of the launch is resident (the
// host checks the grid against the occupancy limit, and the launch follows
// the previous kernel on the stream), so a workgroup may wait for the others.
// Each wait is bounded in real time (GRID_WAIT_TICKS of the 100 MHz counter,
// 0.1 s, far above any phase the host lets through, at most 256 steps): past
// it, or on seeing another workgroup's failure, a workgroup sets the failure
// flag and the kernel returns, so the grid always drains.
// ---------------------------------------------------------------------------
constexpr unsigned long long GRID_WAIT_TICKS = 10000000ull;

__device__ __forceinline__ bool wait_expired(unsigned long long t0, const GridSync *gs) {
  return __builtin_amdgcn_s_memrealtime() - t0 > GRID_WAIT_TICKS ||
         __hip_atomic_load(&gs->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Grid barrier: every workgroup publishes its arrival in its own word, the
// first wavefront of workgroup 0 polls all of them and releases the new
// generation, everyone waits for that release.  Every wavefront first waits
// until its own global stores have completed (reached the L2 of its XCD;
// the workgroup barrier alone only waits for LDS), then after the workgroup
// barrier thread 0's device-scope release writes that L2 back before the
// arrival word: one device-scope release (a cache write-back) per workgroup
// instead of one per wavefront.  After the release thread 0 only acquires
// (invalidates), since its workgroup's writes went out on arrival.
__device__ __forceinline__ bool grid_barrier(GridSync *gs, unsigned &gen, int *ok_lds) {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0) (expcnt, lgkmcnt unconstrained)
  __syncthreads();
  const unsigned target = gen + 1;
  int ok = 1;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0x0F70);  // the write-back has completed before the arrival word
    __hip_atomic_store(&gs->arrive[blockIdx.x], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (blockIdx.x == 0 && threadIdx.x < WAVE) {
    const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
      bool done = true;
      for (unsigned b = threadIdx.x; b < gridDim.x; b += WAVE)
        done = done && __hip_atomic_load(&gs->arrive[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == target;
      if (__all(done)) break;
      if (wait_expired(t0, gs)) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    if (threadIdx.x == 0 && ok) {
      __threadfence();
      __hip_atomic_store(&gs->rel, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (threadIdx.x == 0) {
    if (ok) {
      const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
      while (__hip_atomic_load(&gs->rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != target) {
        if (wait_expired(t0, gs)) {
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (!ok) atomicExch(&gs->err, 1);
    // acquire only: this workgroup's own writes were released on arrival
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *ok_lds = ok;
  }
  gen = target;
  __syncthreads();
  return *ok_lds != 0;
}

template <int W, int K, int L, int NW>
__global__ void __launch_bounds__(WAVE * NW) coarse_vcycle_kernel(CoarsePlan plan, GridSync *gs, const int *stop) {
  extern __shared__ double smem[];
  __shared__ int ok;
  constexpr int T = WAVE * NW;
  constexpr int NX = L * T;
  constexpr int KK = K * K;
  constexpr int TABSZ = RTAB_ALL * KK;
  if (stop && *stop) return;  // the solve has already stopped (uniform)
  if (__hip_atomic_load(&gs->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  unsigned gen = __hip_atomic_load(&gs->rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double *v = smem;
  double *tabs = smem + NX + (NX >> 4) + 1;
  double *qf = tabs + plan.nlevels * 2 * TABSZ;
  double *qb = qf + (MAXWAVES + 2) * K;
  double *red = qb + (MAXWAVES + 2) * K;
  for (int l = 0; l < plan.nlevels; ++l) {
    const StepOp &op = plan.desc[l]->op;
    double *tf = tabs + 2 * l * TABSZ;
    for (int i = threadIdx.x; i < TABSZ; i += T) {
      tf[i] = static_cast<const double *>(op.fw.tab)[i];
      tf[TABSZ + i] = static_cast<const double *>(op.bw.tab)[i];
    }
  }
  __syncthreads();
  for (int ph = 0; ph < plan.nphases; ++ph) {
    const CoarsePhase &P = plan.ph[ph];
    if (P.kind == CP_FILL) {
      for (int64_t i = (int64_t)blockIdx.x * T + threadIdx.x; i < P.pa.nint; i += (int64_t)gridDim.x * T)
        P.pa.cout[i] = 0.0;
    } else if ((int64_t)blockIdx.x < P.pa.nint) {
      const StepOp &op = plan.desc[P.level]->op;
      double *tf = tabs + 2 * P.level * TABSZ;
      lean_pass<W, K, L, NW>(op, P.pa, blockIdx.x, v, tf, tf + TABSZ, tf, tf + TABSZ, qf, qb, red,
                          [] { return true; });
    }
    if (ph + 1 < plan.nphases && !grid_barrier(gs, gen, &ok)) return;
  }
}

template <int W, int K, int L, int NW>
hipError_t coarse_vcycle_launch(const CoarsePlan &plan, int64_t grid, size_t lds, GridSync *gs, const int *stop,
                                hipStream_t stream) {
  hipLaunchKernelGGL((coarse_vcycle_kernel<W, K, L, NW>), dim3((unsigned)grid), dim3(WAVE * NW), lds, stream, plan, gs,
                     stop);
  return hipGetLastError();
}

template <int W, int K, int L, int NW>
int coarse_vcycle_grid(size_t lds) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)coarse_vcycle_kernel<W, K, L, NW>, WAVE * NW,
                                                   lds) != hipSuccess)
    return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

template <int W, int K, int L, int NW, class E>
hipError_t slc_launch(const LevelDesc *desc, const PassArgsT<E> &pa, hipStream_t stream) {
  constexpr size_t lds = (size_t)lean_lds_offsets(L * WAVE * NW, K).total * sizeof(double);
  hipLaunchKernelGGL((slc_kernel<W, K, L, NW, E>), dim3((unsigned)pa.nint), dim3(WAVE * NW), lds, stream, desc, pa);
  return hipGetLastError();
}

// The (L, NW) shapes: nx = 64 L NW.
#define MGRIT_LEAN_SHAPES(X, W, K)                                                                 \
  X(W, K, 16, 1) X(W, K, 16, 2) X(W, K, 16, 4) X(W, K, 16, 8) X(W, K, 8, 1) X(W, K, 8, 2) X(W, K, 8, 4) \
  X(W, K, 8, 8) X(W, K, 4, 1)

template <class E>
hipError_t slc_launch_any(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgsT<E> &pa,
                          hipStream_t stream) {
  const int W = op.sl_l + op.sl_r + 1;
  const int key = lean_key(W, op.fw.k, lay.L, lay.nx / (WAVE * lay.L));
#define MGRIT_SLC_CASE(Wv, Kv, Lv, NWv) \
  case lean_key(Wv, Kv, Lv, NWv): return slc_launch<Wv, Kv, Lv, NWv, E>(desc, pa, stream);
  switch (key) {
    MGRIT_LEAN_SHAPES(MGRIT_SLC_CASE, 2, 1)
    MGRIT_LEAN_SHAPES(MGRIT_SLC_CASE, 4, 2)
    MGRIT_LEAN_SHAPES(MGRIT_SLC_CASE, 6, 3)
    default: return hipErrorInvalidValue;
  }
#undef MGRIT_SLC_CASE
}

hipError_t slc_set_lds(size_t bytes) {
  hipError_t e = hipSuccess;
#define MGRIT_SLC_LDS(Wv, Kv, Lv, NWv)                                                                    \
  if (e == hipSuccess)                                                                                   \
    e = hipFuncSetAttribute((const void *)slc_kernel<Wv, Kv, Lv, NWv, double>,                             \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);                       \
  if (e == hipSuccess)                                                                                   \
    e = hipFuncSetAttribute((const void *)slc_kernel<Wv, Kv, Lv, NWv, float>,                              \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  MGRIT_LEAN_SHAPES(MGRIT_SLC_LDS, 2, 1)
  MGRIT_LEAN_SHAPES(MGRIT_SLC_LDS, 4, 2)
  MGRIT_LEAN_SHAPES(MGRIT_SLC_LDS, 6, 3)
#undef MGRIT_SLC_LDS
  // The persistent coarse cycle's instances get the same process-wide limit
  // (less their static LDS) here, once, so that no later setup changes it
  // while launches are in flight.
#define MGRIT_CV_LDS(Wv, Kv, Lv, NWv)                                                                       \
  if (e == hipSuccess) {                                                                                   \
    hipFuncAttributes fa{};                                                                                \
    e = hipFuncGetAttributes(&fa, (const void *)coarse_vcycle_kernel<Wv, Kv, Lv, NWv>);                    \
    if (e == hipSuccess)                                                                                   \
      e = hipFuncSetAttribute((const void *)coarse_vcycle_kernel<Wv, Kv, Lv, NWv>,                         \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)(bytes - fa.sharedSizeBytes)); \
  }
  MGRIT_LEAN_SHAPES(MGRIT_CV_LDS, 2, 1)
  MGRIT_LEAN_SHAPES(MGRIT_CV_LDS, 4, 2)
  MGRIT_LEAN_SHAPES(MGRIT_CV_LDS, 6, 3)
#undef MGRIT_CV_LDS
  return e;
}

}  // namespace

hipError_t launch_lean(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs &pa,
                       hipStream_t stream) {
  return slc_launch_any(desc, op, lay, pa, stream);
}

hipError_t launch_lean32(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs32 &pa,
                         hipStream_t stream) {
  return slc_launch_any(desc, op, lay, pa, stream);
}

hipError_t configure_lean_kernels(size_t bytes) { return slc_set_lds(bytes); }

size_t coarse_vcycle_lds(const StepOp &op, const Layout &lay, int nlevels) {
  if (!lean_slc_applies(op, lay) || nlevels < 1 || nlevels > MAX_COARSE_LEVELS) return 0;
  const int K = op.fw.k;
  const size_t n = (size_t)lay.nx + (lay.nx >> 4) + 1 + (size_t)nlevels * 2 * RTAB_ALL * K * K +
                   2 * (MAXWAVES + 2) * K + MAXWAVES;
  const size_t bytes = n * sizeof(double);
  return bytes + 256 <= 160 * 1024 ? bytes : 0;  // 256: the kernel's static LDS
}

// (W, K, L, NW) of the persistent launch from the operator and the layout.
#define MGRIT_CV_SWITCH(CASE, FAIL)                                                 \
  do {                                                                              \
    switch (lean_key(op.sl_l + op.sl_r + 1, op.fw.k, lay.L, lay.nx / (WAVE * lay.L))) { \
      MGRIT_LEAN_SHAPES(CASE, 2, 1)                                                 \
      MGRIT_LEAN_SHAPES(CASE, 4, 2)                                                 \
      MGRIT_LEAN_SHAPES(CASE, 6, 3)                                                 \
      default: return FAIL;                                                         \
    }                                                                               \
  } while (0)

// Occupancy query only: the LDS attribute was raised to the device limit once,
// before any launch (configure_lean_kernels).
int coarse_vcycle_max_grid(const StepOp &op, const Layout &lay, size_t lds) {
  if (!lean_slc_applies(op, lay)) return 0;
#define MGRIT_CV_GRID(Wv, Kv, Lv, NWv) \
  case lean_key(Wv, Kv, Lv, NWv): return coarse_vcycle_grid<Wv, Kv, Lv, NWv>(lds);
  MGRIT_CV_SWITCH(MGRIT_CV_GRID, 0);
#undef MGRIT_CV_GRID
}

hipError_t launch_coarse_vcycle(const CoarsePlan &plan, const StepOp &op, const Layout &lay, int64_t grid,
                                size_t lds, GridSync *gs, const int *stop, hipStream_t stream) {
  if (!lean_slc_applies(op, lay)) return hipErrorInvalidValue;
#define MGRIT_CV_LAUNCH(Wv, Kv, Lv, NWv) \
  case lean_key(Wv, Kv, Lv, NWv): return coarse_vcycle_launch<Wv, Kv, Lv, NWv>(plan, grid, lds, gs, stop, stream);
  MGRIT_CV_SWITCH(MGRIT_CV_LAUNCH, hipErrorInvalidValue);
#undef MGRIT_CV_LAUNCH
}

#undef MGRIT_CV_SWITCH
#undef MGRIT_LEAN_SHAPES

}  // namespace mgrit
