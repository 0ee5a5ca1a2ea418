// Internal types shared by the host driver (mgrit_host.cpp) and the gfx950
// kernels (mgrit_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mgrit {

constexpr int KMAX = 3;       // max order of one periodic recurrence
constexpr int MAXTAPS = 8;    // max stencil / interpolation taps
constexpr int MAXCOEF = 8;    // max Horner coefficients (degree + 1)
constexpr int MAXCTAPS = 16;  // max taps of an explicit step written out as one stencil
constexpr int MAXWAVES = 16;  // 1024 threads / 64
constexpr int WAVE = 64;

// How one time step Phi acts on a spatial vector u.
//  OP_POLY_Z: Phi u = sum_i coef[i] Z^i u,  Z = stencil (taps) = -c L_p.
//             Explicit RK: R(z) is a polynomial (Sec. 4.2).
//  OP_POLY_W: Phi u = sum_i coef[i] W^i u,  W = (I + gamma c L_p)^{-1} = T^{-1}.
//             SDIRK: R(z) = P(z)/(1 - gamma z)^s is a polynomial in
//             w = 1/(1 - gamma z) (every stage solves with the same matrix).
//  OP_SLC:    Phi u = T^{-1} S u, S the semi-Lagrangian interpolation and
//             T = I - phi_p D^(p+1) - phi_q D^(q+1)  (eq. MOL-SL-corrected).
// T^{-1} is applied through the factorisation T = C * F(S^-1) * B(S) into a
// causal and an anti-causal banded factor; each factor's inverse is a linear
// recurrence on the periodic mesh (see the kernels).
enum OpKind : int { OP_POLY_Z = 0, OP_POLY_W = 1, OP_SLC = 2 };

// One periodic linear recurrence y_i = x_i + sum_{m=1..k} a[m-1] y_{i-m}
// (forward) or y_{i+m} (backward), run over T threads that each own a chunk
// of L consecutive points.  tab holds RTAB_ALL matrices of k*k doubles, for
// this chunk layout (M the companion matrix, H = M^L, A threads own points):
//   Hpow[t] = H^t, t = 0..64, then Hlast = M^{Llast},
//   then Wwrap = (I - Hlast * H^{A-1})^{-1}, then Hhalf = M^{L/2},
//   then Hwave[w] = H^{64 w}, w = 0..MAXWAVES-1.
// The generic step kernel stages the first RTAB of them in LDS, the lean
// coarse-step kernel all RTAB_ALL.
constexpr int RTAB = WAVE + 4;
constexpr int TAB_HLAST = WAVE + 1, TAB_WWRAP = WAVE + 2, TAB_HHALF = WAVE + 3, TAB_HWAVE = WAVE + 4;
constexpr int RTAB_ALL = RTAB + MAXWAVES;
struct Recurrence {
  int k;
  double a[KMAX];
  const void *tab;  // the tables in the precision of the kernels that read them
  // Truncated-carry evaluation (the windowed step kernel, mgrit_window.h):
  // the state entering a chunk is the sum over the D chunks before it of
  // H^d (their zero-state end states), H = M^{win_L}.  wtab: [D-1][k][k] H^d
  // (d = 1..D-1), then M^{win_L/2}, in the kernels' precision.
  int D;
  const void *wtab;
};
constexpr int WIN_DMAX = 12;  // longest carry the windowed kernel accepts

struct StepOp {
  int kind;
  int repeat;             // apply the whole operator `repeat` times per step
  int ncoef;              // Horner: coef[0..ncoef-1]
  double coef[MAXCOEF];
  int st_l, st_r;         // OP_POLY_Z stencil offsets -st_l..st_r
  double taps[MAXTAPS];   // taps[j + st_l]
  int ct_l, ct_r;         // the whole explicit step R(Z) as one stencil, offsets -ct_l..ct_r
  double ctaps[MAXCTAPS]; // ctaps[j + ct_l] (level-0 tiles only)
  int sl_l, sl_r;         // OP_SLC interpolation nodes -sl_l..sl_r around i-K
  int sl_K;               // floor(shift) mod nx
  double slw[MAXTAPS];    // slw[j + sl_l]
  int has_solve;          // T != I
  double cinv;            // 1/C of the factorisation
  Recurrence fw, bw;
  // windowed step kernel (0: not available): points per thread, nx = threads
  // * win_L; OP_POLY_W takes Horner coefficients in G = B^{-1} F^{-1}
  // (wcoef[i] = coef[i] / C^i), OP_SLC folds 1/C into the interpolation weights
  int win_L;
  double wcoef[MAXCOEF];
  // OP_SLC with GMRES coarse solves (gmres_max > 0): T itself as a symmetric
  // stencil ttaps[d + t_k], d = -t_k..t_k, and per-workgroup Krylov storage
  // krylov + b (gmres_max + 1) nx for workgroup b < krylov_cap
  int gmres_max;
  double gmres_rtol;
  int no_lean;  // OP_SLC: keep this operator off the lean kernel (setup's choice)
  int t_k;
  double ttaps[MAXTAPS];
  double *krylov;
  int64_t krylov_cap;
};
constexpr int GMRES_MAX = 32;

// Work distribution of one nx-vector over a workgroup.
struct Layout {
  int nx;
  int L;      // points per thread (template parameter of the kernels)
  int A;      // threads that own points: ceil(nx / L)
  int T;      // workgroup size, multiple of 64, >= A
  int Llast;  // points of thread A-1
  int ragged; // 0: nx == A*L and A == T (backward recurrence runs in reversed
              //    thread order); 1: redistribute through LDS instead
  int dbuf;   // explicit stencils alternate between two LDS vectors
};

// LDS layout of one launch (in doubles): padded vector(s), the forward and
// backward recurrence tables, their scan scratch, and the reduction scratch.
struct LdsOffsets {
  int vec1, tab_f, tab_b, scr_f, scr_b, red, total;
};

__host__ __device__ inline LdsOffsets lds_offsets(const Layout &lay, int has_solve) {
  LdsOffsets o;
  const int pv = lay.nx + (lay.nx >> 4) + 1;
  int off = pv;
  o.vec1 = lay.dbuf ? off : 0;
  if (lay.dbuf) off += pv;
  const int tabsz = has_solve ? RTAB * KMAX * KMAX : 0;
  o.tab_f = off;
  off += tabsz;
  o.tab_b = off;
  off += tabsz;
  o.scr_f = off;
  off += 2 * MAXWAVES * KMAX;
  o.scr_b = off;
  off += 2 * MAXWAVES * KMAX;
  o.red = off;
  off += MAXWAVES;
  o.total = off;
  return o;
}

// Per-level descriptor, uploaded once to device memory; kernels read it
// through a pointer so every field is a uniform (scalar) load.
struct LevelDesc {
  StepOp op;
  Layout lay;
};

// The lean coarse-step kernel: L points per lane and NW full wavefronts,
// nx = 64 L NW, for L = 16 or 8 with NW = 1, 2, 4, 8 (nx = 512 ... 8192) and
// for L = 4 with one wavefront (nx = 256).  At 16 wavefronts the
// 128-register budget of a 1024-thread workgroup would spill.
constexpr __host__ __device__ inline bool lean_shape(int L, int nw) {
  return ((L == 16 || L == 8) && (nw == 1 || nw == 2 || nw == 4 || nw == 8)) || (L == 4 && nw == 1);
}
constexpr __host__ __device__ inline int lean_key(int W, int K, int L, int nw) {
  return ((W * 4 + K) * 32 + L) * 16 + nw;
}

// LDS layout of the lean coarse-step kernel (in doubles): one padded vector,
// the forward and backward tables, the two wavefront-total arrays, and the
// reduction scratch.
struct LeanLds {
  int tab_f, tab_b, qf, qb, red, total;
};

constexpr __host__ __device__ inline LeanLds lean_lds_offsets(int nx, int K) {
  LeanLds o{};
  int off = nx + (nx >> 4) + 1;
  o.tab_f = off;
  off += RTAB_ALL * K * K;
  o.tab_b = off;
  off += RTAB_ALL * K * K;
  o.qf = off;
  off += (MAXWAVES + 2) * K;
  o.qb = off;
  off += (MAXWAVES + 2) * K;
  o.red = off;
  off += MAXWAVES;
  o.total = off;
  return o;
}

// The lean kernel takes semi-Lagrangian steps with a solve: W = 2K
// interpolation taps (odd p, K = (p+1)/2 for the single-term correction),
// equal forward/backward orders, no repetition, and recurrence tables built
// for 16-point chunks that cover nx exactly.
inline bool lean_slc_applies(const StepOp &op, const Layout &lay) {
  if (op.gmres_max > 0 || op.no_lean) return false;
  const int W = op.sl_l + op.sl_r + 1;
  const int nw = lay.L > 0 ? lay.nx / (WAVE * lay.L) : 0;
  return op.kind == OP_SLC && op.has_solve && op.repeat == 1 && !lay.ragged && lay.A == lay.T &&
         lay.nx == nw * WAVE * lay.L && lean_shape(lay.L, nw) &&
         op.fw.k == op.bw.k && op.fw.k >= 1 && W == 2 * op.fw.k &&
         lean_lds_offsets(lay.nx, op.fw.k).total * sizeof(double) <= 160 * 1024;
}

enum PassMode : int {
  MODE_PASS_A = 0,   // F-relaxation then C-relaxation of every CF-interval
  MODE_PASS_B = 1,   // F-relaxation then the C-point residual (+ norm partials)
  MODE_POST_F = 2,   // F-relaxation, every point added into the parent level
  MODE_FINAL_F = 3,  // F-relaxation writing every time point to the output
  MODE_SEQ = 4,      // sequential stepping over all steps (one workgroup)
  MODE_APPLY = 5,    // independent vectors, nsteps applications each
  MODE_RESID = 6     // space-time residual: m consecutive time points per workgroup, one step each
};

template <class T>
struct PassArgsT {
  int mode;
  int m;              // steps per interval (MODE_SEQ: total steps; APPLY: nsteps)
  int zero_init;      // start every interval from 0 instead of cin
  int64_t nint;       // intervals / vectors / time points = gridDim.x
  const T *cin;       // [nint+1][nx] C-points (APPLY/RESID: [nint(+1)][nx])
  T *cout;            // PASS_A: [nint+1][nx]; APPLY: [nint][nx]
  const T *g;         // right-hand side rows, g[n-1] for level point n; NULL = 0
  T *r;               // PASS_B: [nint][nx] residual; RESID: [nint][nx] or NULL
  float *r32;         // RESID (float64 kernels): the residual rounded to float32, or NULL
  T *parent;          // POST_F / SEQ: parent C-point rows to add into
  T *out;             // FINAL_F / SEQ: output rows
  double *normpart;   // PASS_B / RESID: per-workgroup partial sum of squares
  const int *stop;    // non-NULL: the launch does nothing once *stop != 0
};
using PassArgs = PassArgsT<double>;   // every kernel
using PassArgs32 = PassArgsT<float>;  // the generic step kernel in FP32 (inner solves of mixed precision)

// Iteration state of one solve, kept in device memory: the kernel that
// reduces the residual norm also takes the stopping decision, so the passes
// queued behind it (the coarse-grid correction) can skip themselves without
// the host waiting in between.
enum StopCode : int {
  STOP_NONE = 0,
  STOP_CONVERGED = 1,
  STOP_MAX_ITER = 2,
  STOP_NONFINITE = 3,
  STOP_DIVERGED = 4,
  STOP_DEVICE = 5,  // a persistent launch gave up at a grid barrier
  STOP_STALLED = 6,  // the residual fell by less than StopRule::stall in one iteration
  STOP_OUTER = 7     // an inner solve queued behind an outer stop: skipped
};
struct SolveCtl {
  double res0;  // ||r_0||
  double rho;   // the latest ||r_it||
  int it;       // coarse-grid corrections performed so far
  int stop;     // StopCode
};
static_assert(sizeof(SolveCtl) <= 128, "the pinned host words hold SolveCtl in 128 bytes");
struct StopRule {
  double rtol;
  double diverge_factor;  // <= 0: no growth test
  int max_iter;
  double stall;           // > 0: stop once ||r_it|| > stall ||r_{it-1}|| (float32 inner solves)
};

// Level-0 explicit relaxation with wavefront tiles (temporal blocking): one
// wavefront owns the output range [x0, x0 + TW) of one CF-interval plus a halo
// of HL points on the left and HR on the right, P points per lane (64 P =
// TW + HL + HR), and advances all steps of the interval in registers; the
// halo shrinks by the stencil extent at every stencil application.
struct TileGeom {
  int P;       // points per lane (kernel template parameter)
  int HL, HR;  // halo widths: steps * (Horner depth) * stencil extent
  int TW;      // output points per tile (last tile may have fewer)
  int ntiles;  // tiles per interval
  int sl, sr;  // stencil extents (kernel template parameters)
  int comp;    // 1: one application of the written-out step (ct_l, ct_r), else Horner
};

template <class T>
struct TileArgsT {
  int mode;           // MODE_PASS_A, MODE_PASS_B, MODE_FINAL_F or MODE_SEQ (one block
                      // of m sequential steps: nint = 1, cin = out = the block's first row)
  int m;              // steps per interval
  int64_t nint;       // intervals
  const T *cin;       // [nint+1][nx]
  T *cout;            // PASS_A: [nint+1][nx]
  T *r;               // PASS_B: [nint][nx]
  T *out;             // FINAL_F: [nint*m+1][nx]
  const T *g;         // right-hand side rows, g[n-1] added after the step to level point n; NULL = 0
  double *normpart;   // PASS_B: [nint*ntiles]
  const int *stop;    // non-NULL: the launch does nothing once *stop != 0
};
using TileArgs = TileArgsT<double>;
using TileArgs32 = TileArgsT<float>;  // the float32 inner passes of mixed precision

hipError_t launch_tiles(const LevelDesc *desc, const TileGeom &tg, const TileArgs &ta, hipStream_t stream);
hipError_t launch_tiles_4(const LevelDesc *desc, const TileGeom &tg, const TileArgs &ta, hipStream_t stream);
hipError_t launch_tiles_8(const LevelDesc *desc, const TileGeom &tg, const TileArgs &ta, hipStream_t stream);
hipError_t launch_tiles_16(const LevelDesc *desc, const TileGeom &tg, const TileArgs &ta, hipStream_t stream);
hipError_t launch_tiles32(const LevelDesc *desc, const TileGeom &tg, const TileArgs32 &ta, hipStream_t stream);
hipError_t launch_tiles_4(const LevelDesc *desc, const TileGeom &tg, const TileArgs32 &ta, hipStream_t stream);
hipError_t launch_tiles_8(const LevelDesc *desc, const TileGeom &tg, const TileArgs32 &ta, hipStream_t stream);
hipError_t launch_tiles_16(const LevelDesc *desc, const TileGeom &tg, const TileArgs32 &ta, hipStream_t stream);

// 2D extension (mgrit_2d.hip).  One explicit Runge-Kutta step of the
// dimension-split operator on a batch of nb [ny][nx] slabs: dst = Phi(src)
// (+ g).  The Horner coefficients and the x / y stencil taps (-c_x w,
// -c_y w, offsets -sl..sr) are passed by value.
template <class T>
struct Step2dArgsT {
  const T *src;
  int64_t src_stride;
  T *dst;
  int64_t dst_stride;
  const T *g;  // NULL: no right-hand side
  int64_t g_stride;
  double g_scale;  // dst = Phi(src) + g_scale g
  int64_t nb;
  int nx, ny;
  int ncoef;
  double coef[MAXCOEF];
  int sl, sr;
  double tx[MAXTAPS], ty[MAXTAPS];
  int use_reg;  // the register-tile kernel where it has an instance (else LDS tiles)
};
using Step2dArgs = Step2dArgsT<double>;
using Step2dArgs32 = Step2dArgsT<float>;
size_t step2d_lds_bytes(int ncoef, int sl, int sr);
hipError_t configure_2d_kernels(size_t bytes);
template <class T>
hipError_t launch_step2d(const Step2dArgsT<T> &a, hipStream_t stream);
// dst slab b = transpose(src slab b) (+ g slab b), src slabs [rows][cols]
template <class T>
hipError_t launch_transpose(const T *src, int64_t src_stride, T *dst, int64_t dst_stride, const T *g, int64_t g_stride,
                            int64_t nb, int rows, int cols, hipStream_t stream);
// dst slab b = (dst slab b +) src slab b, n points per slab
template <class T>
hipError_t launch_slab_axpy(T *dst, int64_t dst_stride, const T *src, int64_t src_stride, int64_t nb, int64_t n,
                            bool accumulate, hipStream_t stream);
// r = a - c over nb contiguous slabs of n points (r may be NULL); part gets
// blocks_per_slab partial sums of squares per slab (float64)
template <class T>
hipError_t launch_slab_resid(const T *a, const T *c, T *r, int64_t nb, int64_t n, int blocks_per_slab, double *part,
                             hipStream_t stream);
// partial sums of squares of nb contiguous float64 slabs (as launch_slab_resid with c = 0)
hipError_t launch_slab_norm(const double *a, int64_t nb, int64_t n, int blocks_per_slab, double *part,
                            hipStream_t stream);

// Launch the step kernel for one pass (mgrit_kernels.hip).  lds_bytes is
// computed by the launcher.  Returns the HIP error of the launch.
// `desc` is the device copy of (op, lay); op.kind and lay are read on the host
// to select the kernel instance and launch shape.
hipError_t launch_pass(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs &pa,
                       hipStream_t stream);
// Deterministic reduction of n partial sums into out[0] (sum) on the device.
hipError_t launch_reduce(const double *part, int64_t n, double *out, hipStream_t stream);
// dst rows k = src rows k*stride (k = 0..rows-1), row length nx.
hipError_t launch_gather_rows(const double *src, int64_t stride, double *dst, int64_t rows, int nx,
                              hipStream_t stream);
hipError_t launch_fill(double *dst, int64_t n, double value, hipStream_t stream, const int *stop = nullptr);
// rows r = 0..rows-1 of dst: time points n0 + r dn of the seeded U[0,1)
// initial iterate (SplitMix64 output (n-1) nx + i at point (n, i))
hipError_t launch_splitmix_rows(double *dst, int64_t rows, int64_t n0, int64_t dn, int nx, uint64_t seed,
                                hipStream_t stream);
// Float32 passes of the generic step kernel (mixed precision).
hipError_t launch_pass32(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs32 &pa,
                         hipStream_t stream);
hipError_t launch_fill32(float *dst, int64_t n, hipStream_t stream, const int *stop = nullptr);
// dst[i] = (float) src[i] (nothing once *stop != 0, when stop is given)
hipError_t launch_round32(const double *src, float *dst, int64_t n, hipStream_t stream, const int *stop = nullptr);
// u[i] += (double) e[i] (nothing once *stop != 0, when stop is given)
hipError_t launch_add32(double *u, const float *e, int64_t n, hipStream_t stream, const int *stop = nullptr);
// *ctl = zero state, stopped with STOP_OUTER when gate && *gate
hipError_t launch_ctl_reset(SolveCtl *ctl, const int *gate, hipStream_t stream);
// Sum the n norm partials in a fixed order, set ctl->rho = sqrt(sum) and take
// the stopping decision of iteration ctl->it (ctl zeroed before the first
// call of a solve; a state that has stopped stays as it is); the state is
// also written to ctl_host (pinned host memory) when it is not NULL.
struct GridSync;
hipError_t launch_solve_ctl(const double *part, int64_t n, SolveCtl *ctl, SolveCtl *ctl_host, const GridSync *gs,
                            StopRule rule, hipStream_t stream);
// The coarse part of one V-cycle (every pass on levels >= 1, in order) as
// one persistent launch: the workgroups run each phase on the intervals they
// own and meet at a grid-wide barrier between phases.
enum CoarsePhaseKind : int { CP_PASS = 0, CP_FILL = 1 };
constexpr int MAX_COARSE_PHASES = 24;
constexpr int MAX_COARSE_LEVELS = 15;
struct CoarsePhase {
  int kind;     // CP_PASS: PassArgs pa on level `level`; CP_FILL: zero pa.nint doubles at pa.cout
  int level;    // index into CoarsePlan::desc
  PassArgs pa;  // pa.stop is not used (the launch checks its stop flag once)
};
struct CoarsePlan {
  int nphases;
  int nlevels;
  const LevelDesc *desc[MAX_COARSE_LEVELS];
  CoarsePhase ph[MAX_COARSE_PHASES];
};
// Grid-barrier state in device memory (zeroed at setup): the generation
// released by workgroup 0, a failure flag set by a workgroup that gave up
// waiting (the launch then ends early and the solve reports MGRIT_EDEVICE),
// and one arrival word per workgroup.
constexpr int MAX_PERSISTENT_GRID = 1024;
struct GridSync {
  unsigned rel;
  int err;
  unsigned pad[30];  // rel and err on their own 128-byte line
  unsigned arrive[MAX_PERSISTENT_GRID];
};
// Dynamic LDS bytes of the persistent launch, 0 if it cannot run (the lean
// kernel does not apply, or LDS or co-residency limits).
size_t coarse_vcycle_lds(const StepOp &op, const Layout &lay, int nlevels);
// Largest grid the persistent launch can keep resident (0 on error).
int coarse_vcycle_max_grid(const StepOp &op, const Layout &lay, size_t lds);
hipError_t launch_coarse_vcycle(const CoarsePlan &plan, const StepOp &op, const Layout &lay, int64_t grid,
                                size_t lds, GridSync *gs, const int *stop, hipStream_t stream);

// LDS of the windowed step kernel (in elements of the kernel's precision;
// red in doubles): OP_SLC's padded vector, two areas of published
// recurrence states and the reduction scratch.  When they do not fit beside
// the vector (nx = 16384 in float64) the states reuse the vector's words.
struct WinLds {
  int pub0, pub1, red, bytes, alias;
};
constexpr __host__ __device__ inline WinLds win_lds(int kind, int nx, int nt, int kw, int wsize, int L) {
  WinLds o{};
  const int pv = nx + nx / L + 1;  // the padded vector (OP_SLC: gather; OP_POLY_W: row staging)
  const int pubn = nt * kw;
  int end = pv + 2 * pubn;
  if ((size_t)(end * wsize + 8) / 8 * 8 + MAXWAVES * 8 > 160 * 1024) {
    o.alias = 1;
    end = pv;
    o.pub0 = 0;
    o.pub1 = pubn;
  } else {
    o.pub0 = pv;
    o.pub1 = pv + pubn;
  }
  o.red = (end * wsize + 7) / 8;  // in doubles
  o.bytes = (o.red + MAXWAVES) * 8;
  return o;
}

// The windowed step kernel (mgrit_window.h): OP_POLY_W and OP_SLC operators
// whose recurrences have a truncated-carry plan (op.win_L > 0).
// Instances: SDIRK stage matrices of the odd upwind orders (recurrence orders
// (1,0), (2,1), (3,2)), symmetric coarse operators (k, k), k = 1..3; 16 or
// 32 points per thread.
inline bool window_instance(int kind, int kf, int kb, int L) {
  const bool orders = kind == OP_POLY_W ? (kf >= 1 && kf <= 3 && kb == kf - 1)
                                        : (kind == OP_SLC && kf >= 1 && kf <= 3 && kb == kf);
  return orders && (L == 16 || L == 32);
}
inline bool window_applies(const StepOp &op, const Layout &lay) {
  if (op.gmres_max > 0 || op.win_L <= 0 || !op.has_solve || !window_instance(op.kind, op.fw.k, op.bw.k, op.win_L)) return false;
  if (op.kind == OP_SLC && op.sl_l + op.sl_r + 1 != 2 * op.fw.k) return false;  // the gather has 2k taps
  const int nt = lay.nx / op.win_L;
  return lay.nx == nt * op.win_L && nt % WAVE == 0 && nt <= 1024 && (op.win_L == 16 || nt <= 512);
}
hipError_t launch_window(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs &pa,
                         hipStream_t stream);
hipError_t launch_window32(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs32 &pa,
                           hipStream_t stream);
hipError_t configure_window_kernels64(size_t bytes);
// Corrected SL steps with GMRES solves (mgrit_gmres.hip), float64.
hipError_t launch_gmres(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs &pa,
                        hipStream_t stream);
hipError_t configure_gmres_kernels(size_t bytes);
size_t gmres_lds_bytes(const Layout &lay, int kmax);
hipError_t configure_window_kernels32(size_t bytes);

// The lean coarse-step kernel (mgrit_lean.hip) for layouts where
// lean_slc_applies() holds, and its LDS attribute.
hipError_t launch_lean(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs &pa,
                       hipStream_t stream);
// The same kernel in float32 (one launch per pass) for the inner solves of
// mixed precision; desc holds the float32 copy of the tables.
hipError_t launch_lean32(const LevelDesc *desc, const StepOp &op, const Layout &lay, const PassArgs32 &pa,
                         hipStream_t stream);
hipError_t configure_lean_kernels(size_t bytes);
// The generic step kernel, one translation unit per operator kind.
hipError_t launch_step_poly_z(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, size_t lds,
                              hipStream_t stream);
hipError_t launch_step_poly_w(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, size_t lds,
                              hipStream_t stream);
hipError_t launch_step_slc(const LevelDesc *desc, const Layout &lay, const PassArgs &pa, size_t lds,
                           hipStream_t stream);
hipError_t configure_step_poly_z(size_t bytes);
// Float32 instances (mgrit_step32_*.hip); the level descriptor's tables are float32.
hipError_t launch_step32_poly_z(const LevelDesc *desc, const Layout &lay, const PassArgs32 &pa, size_t lds,
                                hipStream_t stream);
hipError_t launch_step32_poly_w(const LevelDesc *desc, const Layout &lay, const PassArgs32 &pa, size_t lds,
                                hipStream_t stream);
hipError_t launch_step32_slc(const LevelDesc *desc, const Layout &lay, const PassArgs32 &pa, size_t lds,
                             hipStream_t stream);
hipError_t configure_step32_poly_z(size_t bytes);
hipError_t configure_step32_poly_w(size_t bytes);
hipError_t configure_step32_slc(size_t bytes);
hipError_t configure_step_poly_w(size_t bytes);
hipError_t configure_step_slc(size_t bytes);
// Allow the step kernels to use up to `bytes` of dynamic LDS.
hipError_t configure_kernels(size_t bytes);
size_t lds_bytes_for(const Layout &lay, int has_solve);

}  // namespace mgrit
