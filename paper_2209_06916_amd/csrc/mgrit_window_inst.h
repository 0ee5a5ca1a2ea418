// Launch and attribute functions of the windowed step kernel for one
// precision (included by mgrit_window.hip and mgrit_window32.hip with
// MGRIT_WIN_T, MGRIT_WIN_ARGS, MGRIT_WIN_LAUNCH and MGRIT_WIN_CONFIGURE set).
// Instances: SDIRK steps (OP_POLY_W) with U1, U3, U5 stage matrices
// (recurrence orders (1,0), (2,1), (3,2)), corrected semi-Lagrangian steps
// (OP_SLC) with symmetric factors of order 1, 2, 3; 16 or 32 points per
// thread; workgroups of up to 256, 512 or 1024 threads.

#define MGRIT_WIN_SHAPES(X, KIND, KF, KB) \
  X(16, KIND, KF, KB, 256) X(16, KIND, KF, KB, 512) X(16, KIND, KF, KB, 1024) X(32, KIND, KF, KB, 256) \
  X(32, KIND, KF, KB, 512)
#define MGRIT_WIN_ALL(X)                                                                              \
  MGRIT_WIN_SHAPES(X, OP_POLY_W, 1, 0) MGRIT_WIN_SHAPES(X, OP_POLY_W, 2, 1) MGRIT_WIN_SHAPES(X, OP_POLY_W, 3, 2) \
  MGRIT_WIN_SHAPES(X, OP_SLC, 1, 1) MGRIT_WIN_SHAPES(X, OP_SLC, 2, 2) MGRIT_WIN_SHAPES(X, OP_SLC, 3, 3)

namespace {
constexpr int win_key(int L, int kind, int kf, int kb, int maxt) {
  return (((L * 4 + kind) * 4 + kf) * 4 + kb) * 2048 + maxt;
}
}  // namespace

hipError_t MGRIT_WIN_LAUNCH(const LevelDesc *desc, const StepOp &op, const Layout &lay, const MGRIT_WIN_ARGS &pa,
                            hipStream_t stream) {
  if (pa.nint <= 0) return hipSuccess;
  if (!window_applies(op, lay)) return hipErrorInvalidValue;
  const int L = op.win_L;
  const int nt = lay.nx / L;
  const int maxt = nt <= 256 ? 256 : (nt <= 512 ? 512 : 1024);
  const int kw = op.fw.k > op.bw.k ? op.fw.k : (op.bw.k > 0 ? op.bw.k : 1);
  const WinLds lo = win_lds(op.kind, lay.nx, nt, kw, (int)sizeof(MGRIT_WIN_T), L);
  const size_t lds = (size_t)lo.bytes;
#define MGRIT_WIN_CASE(Lv, KINDv, KFv, KBv, MAXTv)                                                              \
  case win_key(Lv, KINDv, KFv, KBv, MAXTv):                                                                     \
    hipLaunchKernelGGL((wstep_kernel<Lv, KINDv, KFv, KBv, MAXTv, MGRIT_WIN_T>), dim3((unsigned)pa.nint), dim3(nt), \
                       lds, stream, desc, pa);                                                                  \
    return hipGetLastError();
  switch (win_key(L, op.kind, op.fw.k, op.bw.k, maxt)) {
    MGRIT_WIN_ALL(MGRIT_WIN_CASE)
    default: return hipErrorInvalidValue;
  }
#undef MGRIT_WIN_CASE
}

hipError_t MGRIT_WIN_CONFIGURE(size_t bytes) {
  hipError_t e = hipSuccess;
#define MGRIT_WIN_ATTR(Lv, KINDv, KFv, KBv, MAXTv)                                                            \
  if (e == hipSuccess)                                                                                        \
    e = hipFuncSetAttribute((const void *)wstep_kernel<Lv, KINDv, KFv, KBv, MAXTv, MGRIT_WIN_T>,                \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  MGRIT_WIN_ALL(MGRIT_WIN_ATTR)
#undef MGRIT_WIN_ATTR
  return e;
}

#undef MGRIT_WIN_ALL
#undef MGRIT_WIN_SHAPES
