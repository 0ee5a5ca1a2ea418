"""Thin ctypes binding of libmgrit.so (include/mgrit.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Device arrays are torch float64 CUDA tensors (contiguous); torch provides the
device memory and the stream, nothing else.  If the library has not been
built, every entry point raises instead of falling back to anything else.
"""
import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmgrit.so")
_lib = None

MAX_LEVELS = 16
MAX_NX = 16384

OK, ENOTCONVERGED, EINVAL, EUNSTABLE, ENOMEM, EDEVICE, EDIVERGED = 0, 1, -1, -2, -3, -4, -5
ERK, SDIRK = 0, 1
CG_SL_CORRECTED, CG_IDEAL, CG_SL_PLAIN, CG_REDISC = 0, 1, 2, 3
PREC_FP64, PREC_MIXED = 0, 1


class MgritError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"mgrit status {status}: {message}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("velocity", ctypes.c_double), ("x_lo", ctypes.c_double), ("x_hi", ctypes.c_double),
                ("nx", ctypes.c_int64), ("nt", ctypes.c_int64), ("cfl", ctypes.c_double),
                ("upwind_order", ctypes.c_int32), ("rk_kind", ctypes.c_int32), ("rk_order", ctypes.c_int32),
                ("rk_stages", ctypes.c_int32), ("rk_A", ctypes.POINTER(ctypes.c_double)),
                ("rk_b", ctypes.POINTER(ctypes.c_double))]


class Options(ctypes.Structure):
    _fields_ = [("max_levels", ctypes.c_int32), ("m", ctypes.c_int32 * (MAX_LEVELS - 1)),
                ("min_coarse_nt", ctypes.c_int32), ("nu", ctypes.c_int32), ("cg_kind", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("diverge_factor", ctypes.c_double),
                ("coarse_launch", ctypes.c_int32), ("precision", ctypes.c_int32), ("inner_rtol", ctypes.c_double),
                ("inner_max_iter", ctypes.c_int32), ("tile_tune", ctypes.c_int32), ("init_seed", ctypes.c_uint64),
                ("coarse_solve", ctypes.c_int32), ("gmres_rtol", ctypes.c_double), ("gmres_max_iter", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("res0", ctypes.c_double), ("res_final", ctypes.c_double),
                ("conv_factor", ctypes.c_double), ("res_history", ctypes.POINTER(ctypes.c_double)),
                ("res_history_cap", ctypes.c_int32), ("res_history_len", ctypes.c_int32),
                ("t_solve_s", ctypes.c_double), ("inner_iterations", ctypes.c_int32)]


class Problem2D(ctypes.Structure):
    _fields_ = [("velocity_x", ctypes.c_double), ("velocity_y", ctypes.c_double), ("x_lo", ctypes.c_double),
                ("x_hi", ctypes.c_double), ("y_lo", ctypes.c_double), ("y_hi", ctypes.c_double),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nt", ctypes.c_int64), ("dt", ctypes.c_double),
                ("upwind_order", ctypes.c_int32), ("rk_order", ctypes.c_int32)]


class LevelDesc(ctypes.Structure):
    _fields_ = [("nt", ctypes.c_int64), ("m", ctypes.c_int32), ("shift", ctypes.c_double),
                ("K", ctypes.c_int64), ("eps", ctypes.c_double), ("phi_p", ctypes.c_double),
                ("phi_q", ctypes.c_double), ("tile_p", ctypes.c_int32), ("win_L", ctypes.c_int32),
                ("win_D", ctypes.c_int32 * 2), ("gmres_max_iter", ctypes.c_int32)]


PROF_PHASES = ["fine_relax", "coarse", "final", "sequential", "residual", "other"]


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * len(PROF_PHASES)), ("total_ms", ctypes.c_double * len(PROF_PHASES))]


EXPORTED = ["mgrit_setup", "mgrit_setup_ws", "mgrit_solve", "mgrit_solve_noalloc", "mgrit_solve_start", "mgrit_solve_advance", "mgrit_solve_finish",
            "mgrit_workspace_bytes", "mgrit_residual", "mgrit_sequential", "mgrit_apply_step",
            "mgrit_num_levels", "mgrit_level_info", "mgrit_lfa_rho", "mgrit_profile_enable",
            "mgrit_profile_read", "mgrit_status_string", "mgrit_last_error", "mgrit_destroy",
            "mgrit2d_setup", "mgrit2d_solve", "mgrit2d_sequential", "mgrit2d_apply_step", "mgrit2d_num_levels",
            "mgrit2d_last_error", "mgrit2d_destroy"]


def library_path():
    return _LIB_PATH


def lib():
    """Load libmgrit.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2209_06916_amd.build")
        L = ctypes.CDLL(_LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.mgrit_setup.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options), vp, ctypes.POINTER(vp)]
        L.mgrit_setup_ws.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options), vp, vp, ctypes.c_uint64,
                                     ctypes.POINTER(vp)]
        L.mgrit_solve.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(Stats)]
        L.mgrit_solve_noalloc.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options), vp, vp, vp, vp, vp,
                                          ctypes.POINTER(Stats)]
        L.mgrit_solve_start.argtypes = [vp, vp, vp, vp, vp]
        L.mgrit_solve_advance.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.mgrit_solve_finish.argtypes = [vp, ctypes.POINTER(Stats)]
        L.mgrit_workspace_bytes.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                            ctypes.POINTER(ctypes.c_uint64)]
        L.mgrit_residual.argtypes = [vp, vp, vp, dp]
        L.mgrit_sequential.argtypes = [vp, vp, vp]
        L.mgrit_apply_step.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int64, ctypes.c_int32]
        L.mgrit_num_levels.argtypes = [vp]
        L.mgrit_num_levels.restype = ctypes.c_int32
        L.mgrit_level_info.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(LevelDesc)]
        L.mgrit_lfa_rho.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options), dp]
        L.mgrit_profile_enable.argtypes = [vp, ctypes.c_uint32]
        L.mgrit_profile_read.argtypes = [vp, ctypes.POINTER(Profile), ctypes.c_int32]
        L.mgrit_status_string.argtypes = [ctypes.c_int]
        L.mgrit_status_string.restype = ctypes.c_char_p
        L.mgrit_last_error.argtypes = [vp]
        L.mgrit_last_error.restype = ctypes.c_char_p
        L.mgrit_destroy.argtypes = [vp]
        L.mgrit_destroy.restype = None
        L.mgrit2d_setup.argtypes = [ctypes.POINTER(Problem2D), ctypes.POINTER(Options), vp, ctypes.POINTER(vp)]
        L.mgrit2d_solve.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(Stats)]
        L.mgrit2d_sequential.argtypes = [vp, vp, vp]
        L.mgrit2d_apply_step.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int64]
        L.mgrit2d_num_levels.argtypes = [vp]
        L.mgrit2d_num_levels.restype = ctypes.c_int32
        L.mgrit2d_last_error.argtypes = [vp]
        L.mgrit2d_last_error.restype = ctypes.c_char_p
        L.mgrit2d_destroy.argtypes = [vp]
        L.mgrit2d_destroy.restype = None
        for name in ("mgrit2d_setup", "mgrit2d_solve", "mgrit2d_sequential", "mgrit2d_apply_step"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("mgrit_setup", "mgrit_setup_ws", "mgrit_solve", "mgrit_solve_noalloc", "mgrit_solve_start", "mgrit_solve_advance", "mgrit_solve_finish",
                     "mgrit_workspace_bytes", "mgrit_residual", "mgrit_sequential", "mgrit_apply_step",
                     "mgrit_level_info", "mgrit_lfa_rho", "mgrit_profile_enable", "mgrit_profile_read"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def make_problem(nx, nt, cfl, p, kind="erk", q=None, velocity=1.0, x_lo=-1.0, x_hi=1.0, tableau=None):
    """tableau: optional (A, b) Butcher tableau of `kind` (q is then the
    order it claims); None selects the built-in tableau of (kind, q)."""
    q = p if q is None else q
    pr = Problem(velocity, x_lo, x_hi, nx, nt, cfl, p, ERK if kind == "erk" else SDIRK, q)
    if tableau is not None:
        A = [float(x) for row in tableau[0] for x in row]
        b = [float(x) for x in tableau[1]]
        pr._arrays = ((ctypes.c_double * len(A))(*A), (ctypes.c_double * len(b))(*b))  # kept alive with pr
        pr.rk_stages = len(b)
        pr.rk_A = ctypes.cast(pr._arrays[0], ctypes.POINTER(ctypes.c_double))
        pr.rk_b = ctypes.cast(pr._arrays[1], ctypes.POINTER(ctypes.c_double))
    return pr


def make_options(m, max_levels=2, min_coarse_nt=0, nu=1, coarse="sl_corrected", rtol=1e-10, max_iter=30,
                 diverge_factor=1e8, coarse_launch=0, precision="fp64", inner_rtol=1e-5, inner_max_iter=30,
                 tile_tune=0, init_seed=0, gmres=None):
    """gmres: (rtol, max_iter) to solve the corrected coarse operators'
    periodic systems approximately by GMRES (Sec. 6.3); None: exactly."""
    o = Options()
    o.max_levels = max_levels
    ms = list(m) if isinstance(m, (list, tuple)) else [m]
    for i, v in enumerate(ms[:MAX_LEVELS - 1]):
        o.m[i] = v
    o.min_coarse_nt = min_coarse_nt
    o.nu = nu
    o.cg_kind = {"sl_corrected": CG_SL_CORRECTED, "ideal": CG_IDEAL, "sl_plain": CG_SL_PLAIN, "redisc": CG_REDISC}[coarse]
    o.rtol = rtol
    o.max_iter = max_iter
    o.diverge_factor = diverge_factor
    o.coarse_launch = coarse_launch
    o.precision = {"fp64": PREC_FP64, "mixed": PREC_MIXED}[precision]
    o.inner_rtol = inner_rtol
    o.inner_max_iter = inner_max_iter
    o.tile_tune = tile_tune
    o.init_seed = init_seed
    if gmres is not None:
        o.coarse_solve, o.gmres_rtol, o.gmres_max_iter = 1, gmres[0], gmres[1]
    return o


def solve_noalloc(problem, options, u0, v_init=None, u_out=None, u_final=None, stream=None, history_cap=128,
                  allow=(OK, ENOTCONVERGED)):
    """mgrit_solve_noalloc: the float64 solve in one call that allocates no
    device memory (its workspace is the library's per-device static array)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    nx, nt = problem.nx, problem.nt
    hist = (ctypes.c_double * history_cap)()
    stats = Stats()
    stats.res_history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    stats.res_history_cap = history_cap
    st = lib().mgrit_solve_noalloc(ctypes.byref(problem), ctypes.byref(options), ctypes.c_void_p(stream.cuda_stream),
                                   _ptr(u0, (nx,)), _ptr(v_init, (nt + 1, nx)), _ptr(u_out, (nt + 1, nx)),
                                   _ptr(u_final, (nx,)), ctypes.byref(stats))
    if st not in allow:
        raise MgritError(st, lib().mgrit_last_error(None).decode())
    return dict(status=st, iterations=stats.iterations, res0=stats.res0, res_final=stats.res_final,
                conv_factor=stats.conv_factor, res_history=list(hist[:stats.res_history_len]))


def workspace_bytes(problem, options):
    """Device memory a handle of (problem, options) allocates (host-only query)."""
    n = ctypes.c_uint64()
    st = lib().mgrit_workspace_bytes(ctypes.byref(problem), ctypes.byref(options), ctypes.byref(n))
    if st != OK:
        raise MgritError(st, "workspace_bytes")
    return n.value


def lfa_rho(problem, options):
    rho = ctypes.c_double()
    st = lib().mgrit_lfa_rho(ctypes.byref(problem), ctypes.byref(options), ctypes.byref(rho))
    if st != OK:
        raise MgritError(st, "lfa")
    return rho.value


def _ptr(t, shape=None):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One mgrit_handle: a problem + options set up on the current device."""

    def __init__(self, problem, options, stream=None, workspace=None):
        """workspace: None (the handle allocates its own device memory) or a
        device tensor of at least workspace_bytes(problem, options) bytes,
        256-byte aligned, that the handle uses until close()."""
        self.problem, self.options = problem, options
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        sp = ctypes.c_void_p(stream.cuda_stream)
        if workspace is None:
            st = lib().mgrit_setup(ctypes.byref(problem), ctypes.byref(options), sp, ctypes.byref(h))
        else:
            nbytes = workspace.numel() * workspace.element_size()
            st = lib().mgrit_setup_ws(ctypes.byref(problem), ctypes.byref(options), sp,
                                      ctypes.c_void_p(workspace.data_ptr()), nbytes, ctypes.byref(h))
        self.workspace = workspace
        if st != OK:
            raise MgritError(st, lib().mgrit_last_error(None).decode())
        self.h = h
        self.nx, self.nt = problem.nx, problem.nt

    def _check(self, st, allow=(OK,)):
        if st not in allow:
            raise MgritError(st, lib().mgrit_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            lib().mgrit_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_levels(self):
        return lib().mgrit_num_levels(self.h)

    def level_info(self, level):
        d = LevelDesc()
        self._check(lib().mgrit_level_info(self.h, level, ctypes.byref(d)))
        return dict(nt=d.nt, m=d.m, shift=d.shift, K=d.K, eps=d.eps, phi_p=d.phi_p, phi_q=d.phi_q, tile_p=d.tile_p,
                    win_L=d.win_L, win_D=(d.win_D[0], d.win_D[1]), gmres_max_iter=d.gmres_max_iter)

    def solve(self, u0, v_init=None, u_out=None, u_final=None, history_cap=128,
              allow=(OK, ENOTCONVERGED)):
        nx, nt = self.nx, self.nt
        hist = (ctypes.c_double * history_cap)()
        stats = Stats()
        stats.res_history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        stats.res_history_cap = history_cap
        st = lib().mgrit_solve(self.h, _ptr(u0, (nx,)), _ptr(v_init, (nt + 1, nx)), _ptr(u_out, (nt + 1, nx)),
                               _ptr(u_final, (nx,)), ctypes.byref(stats))
        self._check(st, allow)
        return dict(status=st, iterations=stats.iterations, res0=stats.res0, res_final=stats.res_final,
                    conv_factor=stats.conv_factor, res_history=list(hist[:stats.res_history_len]),
                    t_solve_s=stats.t_solve_s, inner_iterations=stats.inner_iterations)

    # the same solve in steps (mgrit_solve_start / _advance / _finish)
    def solve_start(self, u0, v_init=None, u_out=None, u_final=None):
        nx, nt = self.nx, self.nt
        self._keep = (u0, v_init, u_out, u_final)  # the device buffers must outlive the solve
        self._check(lib().mgrit_solve_start(self.h, _ptr(u0, (nx,)), _ptr(v_init, (nt + 1, nx)),
                                            _ptr(u_out, (nt + 1, nx)), _ptr(u_final, (nx,))))

    def solve_advance(self):
        done = ctypes.c_int32()
        self._check(lib().mgrit_solve_advance(self.h, ctypes.byref(done)))
        return bool(done.value)

    def solve_finish(self, history_cap=128, allow=(OK, ENOTCONVERGED)):
        hist = (ctypes.c_double * history_cap)()
        stats = Stats()
        stats.res_history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        stats.res_history_cap = history_cap
        st = lib().mgrit_solve_finish(self.h, ctypes.byref(stats))
        self._keep = None
        self._check(st, allow)
        return dict(status=st, iterations=stats.iterations, res0=stats.res0, res_final=stats.res_final,
                    conv_factor=stats.conv_factor, res_history=list(hist[:stats.res_history_len]),
                    t_solve_s=stats.t_solve_s, inner_iterations=stats.inner_iterations)

    def residual(self, u, r=None):
        n = ctypes.c_double()
        self._check(lib().mgrit_residual(self.h, _ptr(u, (self.nt + 1, self.nx)), _ptr(r, (self.nt, self.nx)),
                                         ctypes.byref(n)))
        return n.value

    def sequential(self, u0, u_out):
        self._check(lib().mgrit_sequential(self.h, _ptr(u0, (self.nx,)), _ptr(u_out, (self.nt + 1, self.nx))))

    def profile_enable(self, phases):
        mask = 0
        for ph in phases:
            mask |= 1 << PROF_PHASES.index(ph)
        self._check(lib().mgrit_profile_enable(self.h, mask))

    def profile_read(self, reset=True):
        p = Profile()
        self._check(lib().mgrit_profile_read(self.h, ctypes.byref(p), 1 if reset else 0))
        return {ph: dict(launches=p.launches[i], total_ms=p.total_ms[i]) for i, ph in enumerate(PROF_PHASES)}

    def apply_step(self, level, v_in, v_out, nsteps=1):
        count = v_in.shape[0]
        self._check(lib().mgrit_apply_step(self.h, level, _ptr(v_in, (count, self.nx)),
                                           _ptr(v_out, (count, self.nx)), count, nsteps))


def make_problem_2d(nx, ny, nt, dt_over_h, p, q=None, ax=0.85, ay=1.0, lo=-1.0, hi=1.0):
    """u_t + a_x u_x + a_y u_y = 0 on [lo, hi)^2 with nx x ny points and
    dt = dt_over_h * h, h the smaller of the two mesh widths; ERKq (q
    defaults to p) + Up."""
    pr = Problem2D()
    pr.velocity_x, pr.velocity_y = ax, ay
    pr.x_lo, pr.x_hi, pr.y_lo, pr.y_hi = lo, hi, lo, hi
    pr.nx, pr.ny, pr.nt = nx, ny, nt
    pr.dt = dt_over_h * (hi - lo) / max(nx, ny)
    pr.upwind_order = p
    pr.rk_order = p if q is None else q
    return pr


class Solver2D:
    """One mgrit2d_handle (the dimension-split 2D extension)."""

    def __init__(self, problem, options, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.problem, self.options = problem, options
        h = ctypes.c_void_p()
        st = lib().mgrit2d_setup(ctypes.byref(problem), ctypes.byref(options), ctypes.c_void_p(stream.cuda_stream),
                                 ctypes.byref(h))
        if st != OK:
            raise MgritError(st, lib().mgrit2d_last_error(None).decode())
        self.h = h
        self.nx, self.ny, self.nt = problem.nx, problem.ny, problem.nt

    def _check(self, st, allow=(OK,)):
        if st not in allow:
            raise MgritError(st, lib().mgrit2d_last_error(self.h).decode())
        return st

    @property
    def num_levels(self):
        return lib().mgrit2d_num_levels(self.h)

    def solve(self, u0, v_init=None, u_out=None, u_final=None, history_cap=128, allow=(OK, ENOTCONVERGED)):
        sl = (self.ny, self.nx)
        hist = (ctypes.c_double * history_cap)()
        stats = Stats()
        stats.res_history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        stats.res_history_cap = history_cap
        st = lib().mgrit2d_solve(self.h, _ptr(u0, sl), _ptr(v_init, (self.nt + 1,) + sl),
                                 _ptr(u_out, (self.nt + 1,) + sl), _ptr(u_final, sl), ctypes.byref(stats))
        self._check(st, allow)
        return dict(status=st, iterations=stats.iterations, res0=stats.res0, res_final=stats.res_final,
                    conv_factor=stats.conv_factor, res_history=list(hist[:stats.res_history_len]),
                    t_solve_s=stats.t_solve_s, inner_iterations=stats.inner_iterations)

    def sequential(self, u0, u_out):
        sl = (self.ny, self.nx)
        self._check(lib().mgrit2d_sequential(self.h, _ptr(u0, sl), _ptr(u_out, (self.nt + 1,) + sl)))

    def apply_step(self, level, v_in, v_out):
        count = v_in.shape[0]
        sl = (self.ny, self.nx)
        self._check(lib().mgrit2d_apply_step(self.h, level, _ptr(v_in, (count,) + sl), _ptr(v_out, (count,) + sl),
                                             count))

    def close(self):
        if getattr(self, "h", None):
            lib().mgrit2d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
