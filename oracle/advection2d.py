"""2D periodic advection u_t + a_x u_x + a_y u_y = 0 (oracle; test
infrastructure only).

The paper is one-dimensional.  Its 2D extension follows one reading:
  * the semi-discretisation is dimension-split: L = c_x L_p^(x) + c_y L_p^(y),
    the 1D p-th order upwind stencil of Sec. 4.1 along each axis, with
    c_x = a_x dt / h_x and c_y = a_y dt / h_y, inside every Runge-Kutta stage
    (the fine step is R(-L) of the 2D operator, not a product of 1D steps);
  * the coarse step is dimension-split too: the 1D corrected semi-Lagrangian
    step of eq. (MOL-SL-corrected-multilevel) along x with the 1D
    coefficients for c_x, then the same along y for c_y,
        Psi = (I - phi_y D_y)^{-1} S_y (I - phi_x D_x)^{-1} S_x,
    i.e. a tensor-product semi-Lagrangian step and one periodic banded solve
    per grid line in each direction.
Arrays are [..., ny, nx]: x is the last axis, y the one before it.  The
MGRIT iteration itself is oracle.mgrit's, on [nt+1, ny, nx] arrays.
"""
import numpy as np

from . import discretization as disc
from . import lfa


def _along_y(f, v):
    return np.swapaxes(f(np.swapaxes(v, -1, -2)), -1, -2)


class MOLStep2D:
    """One explicit Runge-Kutta step (Butcher stage form, Sec. 4.3) of
    dv/dt = -(c_x L_p^(x) + c_y L_p^(y)) v in units of dt."""

    def __init__(self, p, q, cx, cy):
        self.p, self.q, self.cx, self.cy = p, q, float(cx), float(cy)
        self.w = disc.upwind_weights(p)
        self.A, self.b = disc.tableau("erk", q)

    def rhs(self, v):
        lx = disc.apply_stencil(v, self.w)
        ly = _along_y(lambda a: disc.apply_stencil(a, self.w), v)
        return -(self.cx * lx + self.cy * ly)

    def __call__(self, u):
        u = np.asarray(u, dtype=float)
        A, b = self.A, self.b
        K = []
        for i in range(len(b)):
            arg = u.copy()
            for j in range(i):
                if A[i, j] != 0.0:
                    arg = arg + A[i, j] * K[j]
            K.append(self.rhs(arg))
        out = u.copy()
        for i in range(len(b)):
            out = out + b[i] * K[i]
        return out

    def symbol(self, wx, wy):
        """R(-(c_x Lhat(w_x) + c_y Lhat(w_y))) for the mode e^{i(w_x j + w_y k)}."""
        z = -(self.cx * disc.stencil_symbol(self.w, wx) + self.cy * disc.stencil_symbol(self.w, wy))
        return disc.stability_function(self.A, self.b, z)


class CorrectedSLStep2D:
    """The dimension-split coarse step: the 1D corrected semi-Lagrangian step
    along x (shift and coefficients of c_x), then along y (of c_y)."""

    def __init__(self, p, q, rec_x, rec_y):
        self.sx = disc.CorrectedSLStep(p, q, rec_x["shift"], rec_x["phi_p"], rec_x["phi_q"])
        self.sy = disc.CorrectedSLStep(p, q, rec_y["shift"], rec_y["phi_p"], rec_y["phi_q"])

    def __call__(self, v):
        return _along_y(self.sy, self.sx(np.asarray(v, dtype=float)))

    def symbol(self, wx, wy):
        return self.sx.symbol(wx) * self.sy.symbol(wy)


class Hierarchy2D:
    """Levels of 2D MGRIT (same interface as oracle.mgrit.Hierarchy)."""

    def __init__(self, nx, ny, nt, p, q, cx, cy, ms):
        self.nx, self.ny, self.nt = nx, ny, nt
        self.space = (ny, nx)
        self.ms = list(ms)
        self.nts = [nt]
        for m in self.ms:
            if self.nts[-1] % m != 0:
                raise ValueError("nt must be divisible by the product of the coarsening factors")
            self.nts.append(self.nts[-1] // m)
        self.steps = [MOLStep2D(p, q, cx, cy)]
        self.coeffs_x = disc.correction_coefficients(p, "erk", q, cx, self.ms)
        self.coeffs_y = disc.correction_coefficients(p, "erk", q, cy, self.ms)
        for rx, ry in zip(self.coeffs_x, self.coeffs_y):
            self.steps.append(CorrectedSLStep2D(p, q, rx, ry))

    @property
    def nlevels(self):
        return len(self.steps)


def rho_two_level_2d(p, q, cx, cy, m, nu=1, n=1 << 8, drop=1):
    """Two-level LFA (eq. rho-asym) over an n x n grid of (w_x, w_y), without
    the samples within ``drop`` grid steps of the origin in both directions."""
    om = -np.pi + 2.0 * np.pi * np.arange(n) / n
    wx, wy = np.meshgrid(om, om, indexing="xy")
    near = (np.abs(wx) <= drop * 2 * np.pi / n + 1e-15) & (np.abs(wy) <= drop * 2 * np.pi / n + 1e-15)
    fine = MOLStep2D(p, q, cx, cy)
    rx = disc.correction_coefficients(p, "erk", q, cx, [m])[0]
    ry = disc.correction_coefficients(p, "erk", q, cy, [m])[0]
    coarse = CorrectedSLStep2D(p, q, rx, ry)
    lam = fine.symbol(wx[~near], wy[~near])
    mu = coarse.symbol(wx[~near], wy[~near])
    return lfa.rho_two_level(lam, mu, m, nu)
