"""Sequential time-stepping and linear MGRIT (oracle; test infrastructure only).

Follows Sec. 2.2 of the paper (and eq. one-step-coarse-general): on each level
the unknowns are v_0..v_nt with equations v_0 = b_0 and
v_n - Phi v_{n-1} = g_n; C-points are every m-th point; a CF-interval is a
C-point and the m-1 F-points after it.

Schedule (identical on the GPU side):
  level-0 iteration it = 0, 1, ...:
    F-relaxation, then nu sweeps of (C-relaxation, F-relaxation)
    C-point residual r_k = g_{km} - v_{km} + Phi v_{km-1}, rho_it = ||r||_2
    stop if rho_it <= rtol * rho_0 or it == max_iter
    otherwise coarse-grid correction: solve e_k = Psi e_{k-1} + r_k, e_0 = 0
    (sequentially on the coarsest level, by recursion otherwise), add e to the
    C-points; the F-relaxation that follows the correction (post-relaxation) is
    the first step of the next iteration.
  coarse level (V-cycle, recursive): start from v = 0, same pre-relaxation and
    residual, recurse, correct the C-points, then post F-relaxation.
The reported iteration count is the number of coarse-grid corrections done.
Arrays hold every time point of a level ([nt+1, nx], or [nt+1, ny, nx] for
the 2D hierarchy of oracle.advection2d); F-relaxation advances all
CF-intervals at once (they are independent by definition).
"""
import numpy as np

from . import discretization as disc


# ---------------------------------------------------------------------------
# Level hierarchy
# ---------------------------------------------------------------------------

class Hierarchy:
    """Time-steppers and sizes of every level.

    ``tab``: an optional Butcher tableau (A, b) in place of the built-in
    one of (kind, q).  ``gmres``: (rtol, maxit) to apply the corrected
    coarse operators' periodic solves approximately by GMRES (Sec. 6.3)
    instead of exactly.  ``coarse`` selects the coarse operator: "sl_corrected" (the paper's
    eq. MOL-SL-corrected-multilevel), "sl_plain" (phi = 0), "ideal"
    (Psi = Phi^m; only meaningful for two levels) or "redisc" (the fine
    Runge-Kutta + upwind step taken with the level's step, i.e. at CFL number
    c m_0 ... m_{l-1}: the rediscretisation of Sec. 5 and Theorem 1).
    """

    def __init__(self, nx, nt, p, kind, q, c, ms, coarse="sl_corrected", tab=None, gmres=None):
        self.nx, self.nt = nx, nt
        self.space = (nx,)  # shape of one time point's vector
        self.p, self.kind, self.q, self.c = p, kind, q, float(c)
        self.ms = list(ms)
        self.nts = [nt]
        for m in self.ms:
            if self.nts[-1] % m != 0:
                raise ValueError("nt must be divisible by the product of the coarsening factors")
            self.nts.append(self.nts[-1] // m)
        fine = disc.MOLStep(p, kind, q, c, tab)
        self.steps = [fine]
        self.coeffs = []
        if coarse == "ideal":
            if len(self.ms) != 1:
                raise ValueError("ideal coarse operator only for two levels")
            self.steps.append(disc.RepeatedStep(fine, self.ms[0]))
        elif coarse == "redisc":
            prod = 1
            for m in self.ms:
                prod *= m
                self.steps.append(disc.MOLStep(p, kind, q, self.c * prod, tab))
        else:
            self.coeffs = disc.correction_coefficients(p, kind, q, c, self.ms, tab)
            for rec in self.coeffs:
                if coarse == "sl_plain":
                    st = disc.CorrectedSLStep(p, q, rec["shift"], 0.0, 0.0)
                elif coarse == "sl_corrected":
                    st = disc.CorrectedSLStep(p, q, rec["shift"], rec["phi_p"], rec["phi_q"], gmres=gmres)
                else:
                    raise ValueError(coarse)
                self.steps.append(st)

    @property
    def nlevels(self):
        return len(self.steps)


def coarsening_schedule(nt, m, min_coarse_nt, max_levels=32):
    """Uniform coarsening factors: keep coarsening level l by m while
    nt_l > min_coarse_nt and m divides nt_l (so the coarsest level has at most
    ``min_coarse_nt`` steps)."""
    ms = []
    cur = nt
    while cur > min_coarse_nt and cur % m == 0 and len(ms) + 1 < max_levels:
        ms.append(m)
        cur //= m
    return ms


# ---------------------------------------------------------------------------
# Sequential stepping (eq. one-step-general) and the space-time residual
# ---------------------------------------------------------------------------

def sequential(step, u0, nt):
    """u_{n+1} = Phi u_n, n = 0..nt-1; returns [nt+1, nx] ([nt+1, ny, nx] in 2D)."""
    u0 = np.asarray(u0, dtype=float)
    u = np.empty((nt + 1,) + u0.shape)
    u[0] = u0
    for n in range(nt):
        u[n + 1] = step(u[n])
    return u


def spacetime_residual(step, u):
    """r_n = Phi u_{n-1} - u_n, n = 1..nt (rows 0..nt-1 of the result)."""
    return step(u[:-1]) - u[1:]


# ---------------------------------------------------------------------------
# Relaxation and residual on one level
# ---------------------------------------------------------------------------

def f_relax(v, g, step, m):
    """v_{km+j} = Phi v_{km+j-1} + g_{km+j}, j = 1..m-1, every interval k."""
    nt = v.shape[0] - 1
    starts = np.arange(0, nt, m)
    for j in range(1, m):
        idx = starts + j
        v[idx] = step(v[idx - 1]) + (g[idx] if g is not None else 0.0)


def c_relax(v, g, step, m):
    """v_{km} = Phi v_{km-1} + g_{km}, every C-point k >= 1."""
    nt = v.shape[0] - 1
    idx = np.arange(m, nt + 1, m)
    v[idx] = step(v[idx - 1]) + (g[idx] if g is not None else 0.0)


def c_residual(v, g, step, m):
    """r_k = g_{km} - v_{km} + Phi v_{km-1}, k = 1..nt/m (eq. 3's right side)."""
    nt = v.shape[0] - 1
    idx = np.arange(m, nt + 1, m)
    r = step(v[idx - 1]) - v[idx]
    if g is not None:
        r = r + g[idx]
    return r


def _pre_relax(v, g, step, m, nu):
    f_relax(v, g, step, m)
    for _ in range(nu):
        c_relax(v, g, step, m)
        f_relax(v, g, step, m)


def vcycle(H, lev, g, nu):
    """Approximate solve of the level-``lev`` system (lev >= 1) with zero
    initial guess and right-hand side g (array [nt_lev+1, nx], g[0] unused).
    Returns the full level iterate [nt_lev+1, nx]."""
    nt = H.nts[lev]
    step = H.steps[lev]
    v = np.zeros((nt + 1,) + H.space)
    if lev == H.nlevels - 1:
        for n in range(1, nt + 1):
            v[n] = step(v[n - 1]) + g[n]
        return v
    m = H.ms[lev]
    _pre_relax(v, g, step, m, nu)
    r = c_residual(v, g, step, m)
    gc = np.zeros((nt // m + 1,) + H.space)
    gc[1:] = r
    e = vcycle(H, lev + 1, gc, nu)
    v[0::m] += e
    f_relax(v, g, step, m)
    return v


def solve(H, u0, v_init, rtol=1e-10, max_iter=30, nu=1, record=False):
    """Linear MGRIT on the level-0 system u_0 = u0, u_n = Phi u_{n-1}.

    ``v_init`` is the initial iterate [nt+1, nx] (only its C-points matter,
    since the first operation is an F-relaxation); row 0 is replaced by u0.
    Returns (u, info) with u the final iterate (F-points relaxed from the final
    C-points) and info = dict(iterations, res_history, conv_factor[, iterates]).
    """
    nt = H.nt
    m = H.ms[0]
    step = H.steps[0]
    v = np.array(v_init, dtype=float, copy=True)
    v[0] = u0
    hist = []
    iterates = []
    it = 0
    while True:
        _pre_relax(v, None, step, m, nu)
        r = c_residual(v, None, step, m)
        rho = float(np.sqrt(np.sum(r * r)))
        hist.append(rho)
        if record:
            iterates.append(v[0::m].copy())
        if not np.isfinite(rho):
            raise FloatingPointError("MGRIT diverged (non-finite residual)")
        if rho <= rtol * hist[0] or it == max_iter:
            break
        gc = np.zeros((nt // m + 1,) + H.space)
        gc[1:] = r
        e = vcycle(H, 1, gc, nu)
        v[0::m] += e
        it += 1
    # the iterate's F-points are consistent with its C-points already (the
    # last operation was an F-relaxation): this is the returned solution
    conv = hist[-1] / hist[-2] if len(hist) >= 2 else float("nan")
    info = dict(iterations=it, res_history=hist, conv_factor=conv)
    if record:
        info["iterates"] = iterates
    return v, info
