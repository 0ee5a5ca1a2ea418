"""Discretization pieces of the oracle (test infrastructure only, see package doc).

Conventions (Sec. 2.1): periodic mesh x_i = x_lo + i*h, i = 0..nx-1 (the paper
counts from 1), h = (x_hi - x_lo)/nx, CFL number c = alpha*dt/h.  Vectors are
numpy arrays whose LAST axis is space; leading axes are batches (e.g. several
CF-intervals advanced at once, which is how MGRIT's F-relaxation is defined:
every interval independently).
"""
from fractions import Fraction
from math import factorial, comb

import numpy as np


# ---------------------------------------------------------------------------
# Upwind finite differences L_p (Sec. 4.1, Lemma 2, Table 1 left)
# ---------------------------------------------------------------------------

def upwind_extent(p):
    """Stencil extent (l, r) of the p-th order upwind rule (Sec. 4.1).

    Odd p: one-point bias, l = (p+1)/2, r = l-1.  Even p: two-point bias,
    l = p/2 + 1, r = l-2.  The stencil is {x_i + j h : j = -l..r}.
    """
    if p < 1:
        raise ValueError("upwind order p must be >= 1")
    if p % 2 == 1:
        l = (p + 1) // 2
        return l, l - 1
    l = p // 2 + 1
    return l, l - 2


def _lagrange_derivative_at_zero(nodes, j):
    """d/dx of the Lagrange basis polynomial of node j (nodes in units of h), at x=0."""
    total = Fraction(0)
    for m in nodes:
        if m == j:
            continue
        term = Fraction(1, j - m)
        for k in nodes:
            if k in (j, m):
                continue
            term *= Fraction(0 - k, j - k)
        total += term
    return total


def upwind_weights_exact(p):
    """Exact rational weights {j: w_j} of L_p: (L_p v)_i = sum_j w_j v_{i+j}.

    L_p/h differentiates the degree-p interpolant through the p+1 stencil
    points and evaluates it at x_i (Sec. 4.1).
    """
    l, r = upwind_extent(p)
    nodes = list(range(-l, r + 1))
    return {j: _lagrange_derivative_at_zero(nodes, j) for j in nodes}


def upwind_weights(p):
    return {j: float(w) for j, w in upwind_weights_exact(p).items()}


def e_fd_closed_form(p):
    """Error constant of L_p, eq. (e_FD_def): (-1)^r l! r! / (p+1)!."""
    l, r = upwind_extent(p)
    return (-1) ** r * factorial(l) * factorial(r) / factorial(p + 1)


def apply_stencil(v, weights):
    """sum_j w_j v_{i+j} on the periodic mesh (last axis)."""
    out = np.zeros_like(v)
    for j, w in weights.items():
        out += w * np.roll(v, -j, axis=-1)
    return out


def stencil_symbol(weights, omega):
    """Fourier symbol sum_j w_j e^{i j omega} of a periodic stencil."""
    omega = np.asarray(omega, dtype=float)
    return sum(w * np.exp(1j * j * omega) for j, w in weights.items())


# ---------------------------------------------------------------------------
# Runge-Kutta methods (Sec. 4.2, Table 1 right, Table 2)
# ---------------------------------------------------------------------------

def _sdirk3_gamma():
    """Root in (0.4, 0.5) of 6 g^3 - 18 g^2 + 9 g - 1 = 0 (bisection)."""
    f = lambda g: ((6.0 * g - 18.0) * g + 9.0) * g - 1.0
    lo, hi = 0.4, 0.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(lo) * f(mid) <= 0.0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


def erk_tableau(q):
    """Butcher tableau (A, b) of the order-q explicit method ERKq.

    The paper takes its tableaux from an earlier work that is not part of the
    text; only the error constants (Table 1) and CFL limits (Table 2) are
    printed.  For this linear problem the step equals R(z) u for the method's
    stability polynomial R (eq. MOL_M_def), so any tableau with the same R is
    equivalent.  Choices: q=1 forward Euler; q=2 Heun; q=3 the three-stage
    strong-stability-preserving method; q=4 the classical method.  All have
    R = sum_{j<=q} z^j/j!, hence e_RK = -1/(q+1)! (Table 1).

    q=5: Table 1's e_RK = -6.0764e-4 fixes beta_6 = 1/1280; we use the six-stage
    method whose only nonzero coupling is the sub-diagonal (3/32, 1/5, 1/4, 1/3,
    1/2) with b = e_6, i.e. R = T_5(z) + z^6/1280.  Its CFL limit with U5 is
    1.9399, not Table 2's 1.96583: the two tables are not consistent with any
    six-stage polynomial, so ERK5's CFL limit is parity unpinned.
    """
    if q == 1:
        return np.array([[0.0]]), np.array([1.0])
    if q == 2:
        return np.array([[0.0, 0.0], [1.0, 0.0]]), np.array([0.5, 0.5])
    if q == 3:
        A = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.25, 0.25, 0.0]])
        return A, np.array([1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0])
    if q == 4:
        A = np.zeros((4, 4))
        A[1, 0] = 0.5
        A[2, 1] = 0.5
        A[3, 2] = 1.0
        return A, np.array([1.0, 2.0, 2.0, 1.0]) / 6.0
    if q == 5:
        A = np.zeros((6, 6))
        for i, a in enumerate([3.0 / 32.0, 0.2, 0.25, 1.0 / 3.0, 0.5]):
            A[i + 1, i] = a
        b = np.zeros(6)
        b[5] = 1.0
        return A, b
    raise ValueError(f"no ERK tableau of order {q}")


def sdirk_tableau(q):
    """Butcher tableau (A, b) of the order-q singly diagonally implicit method.

    q=1 backward Euler; q=2 the two-stage L-stable method with
    gamma = 1 - 1/sqrt(2); q=3 the three-stage L-stable method whose diagonal
    gamma solves 6g^3 - 18g^2 + 9g - 1 = 0 and whose last row of A equals b.
    The paper's fourth/fifth-order SDIRK tableaux come from references outside
    its text and are not provided.
    """
    if q == 1:
        return np.array([[1.0]]), np.array([1.0])
    if q == 2:
        g = 1.0 - 1.0 / np.sqrt(2.0)
        return np.array([[g, 0.0], [1.0 - g, g]]), np.array([1.0 - g, g])
    if q == 3:
        g = _sdirk3_gamma()
        b1 = -(6.0 * g * g - 16.0 * g + 1.0) / 4.0
        b2 = (6.0 * g * g - 20.0 * g + 5.0) / 4.0
        A = np.array([[g, 0.0, 0.0],
                      [(1.0 - g) / 2.0, g, 0.0],
                      [b1, b2, g]])
        return A, np.array([b1, b2, g])
    raise ValueError(f"no SDIRK tableau of order {q}")


def tableau(kind, q):
    if kind == "erk":
        return erk_tableau(q)
    if kind == "sdirk":
        return sdirk_tableau(q)
    raise ValueError(kind)


def stability_function(A, b, z):
    """R(z) = 1 + z b^T (I - zA)^{-1} 1 for complex z (elementwise)."""
    z = np.atleast_1d(np.asarray(z, dtype=complex))
    s = len(b)
    out = np.empty(z.shape, dtype=complex)
    one = np.ones(s)
    for idx, zz in np.ndenumerate(z):
        out[idx] = 1.0 + zz * (b @ np.linalg.solve(np.eye(s) - zz * A, one))
    return out


def e_rk(A, b, q):
    """Error constant of eq. (e_RK_def): beta_{q+1} - 1/(q+1)!, with
    beta_{q+1} = b^T A^q 1 the z^{q+1} Taylor coefficient of R."""
    beta = b @ np.linalg.matrix_power(A, q) @ np.ones(len(b))
    return beta - 1.0 / factorial(q + 1)


def cfl_limit(p, q=None, n_omega=1 << 14, tol=1e-12):
    """c_max of ERKq+Up (Table 2): the largest c with max_omega |R(-c Lhat(omega))| <= 1.

    Bisection on c with omega sampled densely on (0, pi] (the symbol is
    conjugate-symmetric) plus a local refinement of the maximising omega.
    """
    q = p if q is None else q
    A, b = erk_tableau(q)
    w = upwind_weights(p)
    omega = np.linspace(0.0, np.pi, n_omega + 1)[1:]
    lhat = stencil_symbol(w, omega)
    # R is a polynomial for explicit methods: coefficients b^T A^{j-1} 1
    coeffs = [1.0] + [b @ np.linalg.matrix_power(A, j - 1) @ np.ones(len(b))
                      for j in range(1, len(b) + 1)]

    def maxabs(c):
        z = -c * lhat
        val = np.zeros_like(z)
        for a in reversed(coeffs):
            val = val * z + a
        k = int(np.argmax(np.abs(val)))
        # refine around the sampled maximum
        lo = omega[max(k - 1, 0)]
        hi = omega[min(k + 1, len(omega) - 1)]
        om = np.linspace(lo, hi, 2001)
        zz = -c * stencil_symbol(w, om)
        v2 = np.zeros_like(zz)
        for a in reversed(coeffs):
            v2 = v2 * zz + a
        return max(np.abs(val).max(), np.abs(v2).max())

    lo, hi = 1e-3, 4.0
    assert maxabs(lo) <= 1.0 + tol and maxabs(hi) > 1.0 + tol
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if maxabs(mid) <= 1.0 + tol:
            lo = mid
        else:
            hi = mid
    return lo


# ---------------------------------------------------------------------------
# Fine time-stepper: method-of-lines step (eq. MOL_M_def)
# ---------------------------------------------------------------------------

def circulant_solve(rhs, weights, diag_shift, scale):
    """Solve (diag_shift*I + scale*W) y = rhs exactly, W the periodic stencil
    ``weights``, by diagonalising the circulant matrix with the FFT.

    numpy's forward FFT uses e^{-2 pi i k n/N}, so the multiplier of
    (W v)_n = sum_j w_j v_{n+j} is sum_j w_j e^{+2 pi i j k/N}.
    """
    nx = rhs.shape[-1]
    omega = 2.0 * np.pi * np.arange(nx) / nx
    mult = diag_shift + scale * stencil_symbol(weights, omega)
    return np.real(np.fft.ifft(np.fft.fft(rhs, axis=-1) / mult, axis=-1))


class MOLStep:
    """One Runge-Kutta step of dv/dt = -(alpha/h) L_p v with CFL number c.

    Stage form (Sec. 4.3 and its footnote): ERK stages are products with L_p,
    SDIRK stages are solves with I + a_ii c L_p:
        (I + a_ii c L_p) K_i = -c L_p (u + sum_{j<i} a_ij K_j),
        u_new = u + sum_i b_i K_i.
    The SDIRK solves use ``circulant_solve`` (FFT), not a banded factorisation.
    """

    def __init__(self, p, kind, q, c, tab=None):
        self.p, self.kind, self.q, self.c = p, kind, q, float(c)
        self.w = upwind_weights(p)
        # tab: a caller's Butcher tableau (A, b) in place of the built-in one
        self.A, self.b = tableau(kind, q) if tab is None else (np.asarray(tab[0], float), np.asarray(tab[1], float))

    def __call__(self, u):
        u = np.asarray(u, dtype=float)
        A, b, c = self.A, self.b, self.c
        s = len(b)
        K = []
        for i in range(s):
            arg = u.copy()
            for j in range(i):
                if A[i, j] != 0.0:
                    arg = arg + A[i, j] * K[j]
            rhs = -c * apply_stencil(arg, self.w)
            if A[i, i] != 0.0:
                Ki = circulant_solve(rhs, self.w, 1.0, A[i, i] * c)
            else:
                Ki = rhs
            K.append(Ki)
        out = u.copy()
        for i in range(s):
            out = out + b[i] * K[i]
        return out

    def symbol(self, omega):
        """lambda(omega) = R(-c Lhat_p(omega)) (Sec. 5.1)."""
        return stability_function(self.A, self.b, -self.c * stencil_symbol(self.w, omega))


# ---------------------------------------------------------------------------
# Semi-Lagrangian step S_p (Sec. 3, Fig. 1) and f_{p+1} (eq. fpoly_def)
# ---------------------------------------------------------------------------

def sl_extent(p):
    """Interpolation stencil j = -l..r around the east neighbour of the
    departure point; for odd p the p+1 nearest points are l = (p+1)/2,
    r = (p-1)/2 (Sec. 3).  Even p has an epsilon-dependent stencil and is not
    supported."""
    if p % 2 == 0:
        raise ValueError("semi-Lagrangian coarse operator implemented for odd p only")
    return (p + 1) // 2, (p - 1) // 2


def sl_shift(shift):
    """Split the mesh-normalised shift s = alpha*Delta/h into K = floor(s) and
    epsilon = s - K in [0, 1): the departure point of x_i is
    x_{i-K} - epsilon*h (Sec. 3)."""
    K = int(np.floor(shift))
    eps = shift - K
    return K, eps


def sl_weights(p, eps):
    """{j: weight} of degree-p Lagrange interpolation at offset -eps from the
    east neighbour, nodes j = -l..r (units of h)."""
    l, r = sl_extent(p)
    nodes = list(range(-l, r + 1))
    x = -eps
    out = {}
    for j in nodes:
        wj = 1.0
        for k in nodes:
            if k != j:
                wj *= (x - k) / (j - k)
        out[j] = wj
    return out


def sl_apply(v, p, shift):
    """(S_p v)_i = sum_j w_j v_{i-K+j}."""
    K, eps = sl_shift(shift)
    w = sl_weights(p, eps)
    out = np.zeros_like(v)
    for j, wj in w.items():
        out += wj * np.roll(v, K - j, axis=-1)
    return out


def sl_symbol(p, shift, omega):
    K, eps = sl_shift(shift)
    w = sl_weights(p, eps)
    omega = np.asarray(omega, dtype=float)
    return sum(wj * np.exp(1j * (j - K) * omega) for j, wj in w.items())


def f_poly(p, z):
    """f_{p+1}(z) = (1/(p+1)!) prod_{j=-l}^{r} (j + z), eq. (fpoly_def), over the
    semi-Lagrangian interpolation stencil."""
    l, r = sl_extent(p)
    out = 1.0
    for j in range(-l, r + 1):
        out *= (j + z)
    return out / factorial(p + 1)


# ---------------------------------------------------------------------------
# Difference matrix D^(k)_2 (eq. Dp+1_def, with s = 2, symmetric)
# ---------------------------------------------------------------------------

def dmat_weights(k):
    """Symmetric second-order approximation of h^k d^k/dx^k for even k: the
    centred k-th difference, (D v)_i = sum_{n=0}^{k} (-1)^n C(k,n) v_{i+k/2-n}.
    (Sec. 6.3 takes D^(p+1) symmetric and second-order accurate; for p+2
    points this centred stencil is the unique such one.)"""
    if k % 2 != 0:
        raise ValueError("symmetric D^(k) needs even k")
    return {k // 2 - n: float((-1) ** n * comb(k, n)) for n in range(k + 1)}


# ---------------------------------------------------------------------------
# Correction coefficients (eqs. varphi-constant-MOL-SL, MOL-SL-corrected-multilevel)
# ---------------------------------------------------------------------------

def correction_coefficients(p, kind, q, c, ms, tab=None):
    """Per-level coefficients for coarse levels l = 1..len(ms).

    ``ms[l-1]`` is the coarsening factor from level l-1 to level l, so level l
    steps by Delta_l = (prod_{k<=l} m_k) dt and its semi-Lagrangian shift is
    s_l = c * prod m (units of h).

    Returns a list of dicts with keys: shift, K, eps, phi_p (coefficient of
    D^(p+1)), phi_q (coefficient of D^(q+1); zero when q == p, where both terms
    are merged into phi_p).

    For q == p this is the paper's recursion:
        phi_1 = m_1 [c e_FD + (-c)^{p+1} e_RK] + (-1)^{p+1} f(eps_1)
        phi_l = (-1)^{p+1} [-m_l f(eps_{l-1}) + f(eps_l)] + m_l phi_{l-1}
    with the paper's uniform m replaced by the per-level factor m_l.

    For q != p (an extension: the paper pairs q = p), the two error terms of
    Lemma 3 are carried separately through the same argument as Appendix B:
        phi_p,1 = m_1 c e_FD + (-1)^{p+1} f(eps_1),
        phi_p,l = (-1)^{p+1} [-m_l f(eps_{l-1}) + f(eps_l)] + m_l phi_p,l-1,
        phi_q,l = (prod_{k<=l} m_k) (-c)^{q+1} e_RK.
    """
    A, b = tableau(kind, q) if tab is None else (np.asarray(tab[0], float), np.asarray(tab[1], float))
    efd = e_fd_closed_form(p)
    erk = e_rk(A, b, q)
    sgn = (-1.0) ** (p + 1)
    out = []
    prod = 1
    prev = None
    for lev, m in enumerate(ms, start=1):
        prod *= m
        shift = c * prod
        K, eps = sl_shift(shift)
        if lev == 1:
            if q == p:
                phi_p = m * (c * efd + (-c) ** (p + 1) * erk) + sgn * f_poly(p, eps)
                phi_q = 0.0
            else:
                phi_p = m * c * efd + sgn * f_poly(p, eps)
                phi_q = m * (-c) ** (q + 1) * erk
        else:
            phi_p = sgn * (-m * f_poly(p, prev["eps"]) + f_poly(p, eps)) + m * prev["phi_p"]
            phi_q = m * prev["phi_q"]
        rec = dict(shift=shift, K=K, eps=eps, phi_p=phi_p, phi_q=phi_q, m=m)
        out.append(rec)
        prev = rec
    return out


def gmres(apply_a, b, rtol, maxit):
    """Approximate solution of A x = b by GMRES (Saad and Schultz, 1986):
    x0 = 0, the Arnoldi basis of the Krylov space by modified Gram-Schmidt,
    the least-squares problem by Givens rotations; stops once the residual
    2-norm is at most rtol ||b||_2 (Sec. 6.3: reduced by two orders of
    magnitude), or after maxit iterations, or at an exact breakdown.  Returns
    (x, iterations)."""
    b = np.asarray(b, dtype=float)
    beta = float(np.sqrt(np.dot(b, b)))
    if beta == 0.0:
        return np.zeros_like(b), 0
    V = [b / beta]
    R = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    k = 0
    for j in range(maxit):
        w = apply_a(V[j])
        h = np.zeros(j + 2)
        for i in range(j + 1):
            h[i] = np.dot(w, V[i])
            w = w - h[i] * V[i]
        h[j + 1] = float(np.sqrt(np.dot(w, w)))
        # earlier rotations on the new column, then the one that zeroes h[j+1]
        for i in range(j):
            h[i], h[i + 1] = cs[i] * h[i] + sn[i] * h[i + 1], -sn[i] * h[i] + cs[i] * h[i + 1]
        den = float(np.hypot(h[j], h[j + 1]))
        cs[j], sn[j] = h[j] / den, h[j + 1] / den
        h[j], h[j + 1] = den, 0.0
        g[j], g[j + 1] = cs[j] * g[j], -sn[j] * g[j]
        R[: j + 1, j] = h[: j + 1]
        k = j + 1
        if abs(g[j + 1]) <= rtol * beta or den == 0.0 or j + 1 == maxit:
            break
        nrm = float(np.sqrt(np.dot(w, w)))
        if nrm == 0.0:
            break
        V.append(w / nrm)
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - np.dot(R[i, i + 1:k], y[i + 1:k])) / R[i, i]
    x = np.zeros_like(b)
    for i in range(k):
        x = x + y[i] * V[i]
    return x, k


class CorrectedSLStep:
    """Coarse time-stepper of eq. (MOL-SL-corrected-multilevel):
        Psi = (I - phi_p D^(p+1) - phi_q D^(q+1))^{-1} S_p^(Delta),
    i.e. a semi-Lagrangian step followed by one implicit periodic solve,
    done here by FFT diagonalisation (``circulant_solve``), or, with
    ``gmres=(rtol, maxit)``, approximately by GMRES from a zero start for
    every vector (Sec. 6.3)."""

    def __init__(self, p, q, shift, phi_p, phi_q=0.0, gmres=None):
        self.p, self.q, self.shift = p, q, float(shift)
        self.phi_p, self.phi_q = float(phi_p), float(phi_q)
        self.gmres = gmres
        w = {j: -self.phi_p * d for j, d in dmat_weights(p + 1).items()}
        if self.phi_q != 0.0:
            for j, d in dmat_weights(q + 1).items():
                w[j] = w.get(j, 0.0) - self.phi_q * d
        self.corr_weights = w  # stencil of -(phi_p D_p + phi_q D_q)

    def apply_t(self, x):
        """T x = (I - phi_p D^(p+1) - phi_q D^(q+1)) x."""
        return x + apply_stencil(x, self.corr_weights)

    def __call__(self, v):
        y = sl_apply(np.asarray(v, dtype=float), self.p, self.shift)
        if self.gmres is None:
            return circulant_solve(y, self.corr_weights, 1.0, 1.0)
        rtol, maxit = self.gmres
        flat = y.reshape(-1, y.shape[-1])
        out = np.array([gmres(self.apply_t, row, rtol, maxit)[0] for row in flat])
        return out.reshape(y.shape)

    def symbol(self, omega):
        """mu(omega) = Shat / (1 - phi_p Dhat_p - phi_q Dhat_q)."""
        return sl_symbol(self.p, self.shift, omega) / (
            1.0 + stencil_symbol(self.corr_weights, omega))


class RepeatedStep:
    """Phi^m as one coarse step: the ideal coarse-grid operator (Sec. 2.2)."""

    def __init__(self, step, m):
        self.step, self.m = step, m

    def __call__(self, v):
        for _ in range(self.m):
            v = self.step(v)
        return v

    def symbol(self, omega):
        return self.step.symbol(omega) ** self.m
