"""Pins of the oracle's discretization against what the paper and mathematics fix.

Every check here is independent of the oracle's own formula for the quantity it
pins: printed table values (tests/golden), closed forms, exact special cases,
polynomial exactness, and convergence orders of the paper's lemmas.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

from oracle import discretization as disc
from tests.conftest import read_table


def _table1():
    out = {}
    for kind, order, val in read_table("table1_error_constants.txt"):
        out[(kind, int(order))] = float(val)
    return out


def _rel_close_printed(a, b):
    # Table 1 prints 5 significant digits
    return abs(a - b) <= 6e-5 * abs(b)


# --------------------------------------------------------------------------
# L_p (Sec. 4.1, Lemma 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_upwind_rule_exact_on_polynomials(p):
    """L_p/h differentiates every polynomial of degree <= p exactly (it is the
    derivative of the degree-p interpolant), and not x^{p+1}."""
    w = disc.upwind_weights_exact(p)
    for k in range(0, p + 2):
        # d/dx x^k at 0 is 1 for k == 1 else 0; rule gives sum_j w_j j^k
        approx = sum(wj * Fraction(j) ** k for j, wj in w.items())
        exact = Fraction(1) if k == 1 else Fraction(0)
        if k <= p:
            assert approx == exact
        else:
            assert approx != exact


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_upwind_extent_is_upwind(p):
    l, r = disc.upwind_extent(p)
    assert l + r == p and l > r
    assert l - r == (1 if p % 2 else 2)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_e_fd_matches_table1_and_closed_form(p):
    """Leading error of L_p on x^{p+1} is h^p e_FD (p+1)!  (Lemma 2), compared
    with eq. (e_FD_def) and the value printed in Table 1."""
    w = disc.upwind_weights_exact(p)
    e_from_weights = -sum(wj * Fraction(j) ** (p + 1) for j, wj in w.items()) / factorial(p + 1)
    assert float(e_from_weights) == pytest.approx(disc.e_fd_closed_form(p), rel=1e-15)
    assert _rel_close_printed(float(e_from_weights), _table1()[("FD", p)])


# --------------------------------------------------------------------------
# Runge-Kutta (Sec. 4.2, Table 1 right, Table 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind,q", [("erk", 1), ("erk", 2), ("erk", 3), ("erk", 4), ("erk", 5),
                                    ("sdirk", 1), ("sdirk", 2), ("sdirk", 3)])
def test_linear_order_conditions(kind, q):
    A, b = disc.tableau(kind, q)
    one = np.ones(len(b))
    for j in range(1, q + 1):
        assert b @ np.linalg.matrix_power(A, j - 1) @ one == pytest.approx(1.0 / factorial(j), rel=1e-13)


@pytest.mark.parametrize("kind,q", [("erk", 1), ("erk", 2), ("erk", 3), ("erk", 4), ("erk", 5),
                                    ("sdirk", 1), ("sdirk", 2), ("sdirk", 3)])
def test_e_rk_matches_table1(kind, q):
    A, b = disc.tableau(kind, q)
    assert _rel_close_printed(disc.e_rk(A, b, q), _table1()[(kind.upper(), q)])


@pytest.mark.parametrize("kind,q", [("erk", 3), ("sdirk", 1), ("sdirk", 2), ("sdirk", 3)])
def test_e_rk_is_taylor_coefficient_of_R(kind, q):
    """e_RK is the z^{q+1} coefficient of R(z) - exp(z) (eq. e_RK_def): check by a
    finite-difference of the closed-form R around 0 (contour integral)."""
    A, b = disc.tableau(kind, q)
    rad = 0.25
    n = 256
    zs = rad * np.exp(2j * np.pi * np.arange(n) / n)
    vals = disc.stability_function(A, b, zs) - np.exp(zs)
    coef = np.mean(vals / zs ** (q + 1))
    assert coef.real == pytest.approx(disc.e_rk(A, b, q), rel=1e-9)


def test_sdirk_is_A_stable_on_imaginary_axis():
    for q in (1, 2, 3):
        A, b = disc.sdirk_tableau(q)
        y = np.linspace(-200, 200, 4001)
        assert np.max(np.abs(disc.stability_function(A, b, 1j * y))) <= 1.0 + 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_cfl_limits_table2(p):
    table = {int(a): float(b) for a, b in read_table("table2_cfl_limits.txt")}
    assert disc.cfl_limit(p) == pytest.approx(table[p], abs=6e-6)


def test_erk5_cfl_limit_conflict_is_documented():
    """ERK5: with beta_6 fixed by Table 1, c_max is 1.9403, not Table 2's
    1.96583 (parity unpinned for this one entry; see erk_tableau)."""
    table = {int(a): float(b) for a, b in read_table("table2_cfl_limits.txt")}
    cm = disc.cfl_limit(5)
    assert cm == pytest.approx(1.9403, abs=2e-3)
    assert abs(cm - table[5]) > 0.02


# --------------------------------------------------------------------------
# Method-of-lines step (eq. MOL_M_def): per-mode amplification
# --------------------------------------------------------------------------

def _taylor_R(q, z):
    return sum(z ** j / factorial(j) for j in range(q + 1))


@pytest.mark.parametrize("p,kind,q,c", [(1, "erk", 1, 0.85), (3, "erk", 3, 1.3), (5, "erk", 5, 0.9),
                                        (2, "erk", 2, 0.4), (4, "erk", 4, 0.9),
                                        (1, "sdirk", 1, 3.0), (3, "sdirk", 3, 5.0), (5, "sdirk", 3, 0.5),
                                        (2, "sdirk", 2, 2.0)])
def test_step_amplifies_fourier_mode(p, kind, q, c):
    """A discrete mode e^{i omega x_i} after n steps is lambda(omega)^n times
    itself, lambda = R(-c Lhat_p(omega)) (Sec. 5.1).  R is taken in closed form:
    the Taylor polynomial T_q for ERK1-4, T_5 + z^6/1280 for ERK5,
    1/(1-z) for backward Euler, the rational b^T(I-zA)^{-1} form otherwise."""
    nx, n = 64, 7
    step = disc.MOLStep(p, kind, q, c)
    w = disc.upwind_weights_exact(p)
    for k in (1, 5, 17, 31):
        omega = 2 * np.pi * k / nx
        lhat = sum(float(wj) * np.exp(1j * j * omega) for j, wj in w.items())
        z = -c * lhat
        if kind == "erk" and q <= 4:
            lam = _taylor_R(q, z)
        elif kind == "erk":
            lam = _taylor_R(5, z) + z ** 6 / 1280.0
        elif q == 1:
            lam = 1.0 / (1.0 - z)
        else:
            A, b = disc.sdirk_tableau(q)
            lam = disc.stability_function(A, b, z)[0]
        mode = np.exp(1j * omega * np.arange(nx))
        re, im = mode.real.copy(), mode.imag.copy()
        for _ in range(n):
            re, im = step(re), step(im)
        np.testing.assert_allclose(re + 1j * im, lam ** n * mode, atol=1e-13)


def test_erk1_u1_at_unit_cfl_is_exact_shift():
    step = disc.MOLStep(1, "erk", 1, 1.0)
    v = np.random.default_rng(0).random(50)
    np.testing.assert_array_equal(step(v), np.roll(v, 1))


@pytest.mark.parametrize("c", [0.1, 0.5, 0.85, 0.99])
def test_erk1_u1_equals_first_order_semi_lagrangian(c):
    """For c < 1 ERK1+U1 is S_1^(dt) (Sec. 6.1, footnote in Sec. 1)."""
    v = np.random.default_rng(1).random(40)
    step = disc.MOLStep(1, "erk", 1, c)
    np.testing.assert_allclose(step(v), disc.sl_apply(v, 1, c), rtol=0, atol=1e-15)


def test_circulant_solve_inverts_the_stencil():
    rng = np.random.default_rng(3)
    rhs = rng.random((3, 37))
    w = disc.upwind_weights(5)
    y = disc.circulant_solve(rhs, w, 1.0, 0.7)
    back = y + 0.7 * disc.apply_stencil(y, w)
    np.testing.assert_allclose(back, rhs, atol=1e-13)


def test_operators_commute():
    """All operators are circulant, so Phi D = D Phi and S Phi = Phi S."""
    v = np.random.default_rng(4).random(48)
    phi = disc.MOLStep(3, "sdirk", 3, 2.0)
    d = disc.dmat_weights(4)
    np.testing.assert_allclose(phi(disc.apply_stencil(v, d)), disc.apply_stencil(phi(v), d), atol=1e-13)
    np.testing.assert_allclose(phi(disc.sl_apply(v, 3, 7.3)), disc.sl_apply(phi(v), 3, 7.3), atol=1e-13)


# --------------------------------------------------------------------------
# Semi-Lagrangian S_p (Sec. 3) and D^(p+1) (eq. Dp+1_def)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 3, 5])
def test_sl_integer_shift_is_exact(p):
    v = np.random.default_rng(5).random(33)
    for K in (0, 1, 7, 40):
        np.testing.assert_array_equal(disc.sl_apply(v, p, float(K)), np.roll(v, K))


@pytest.mark.parametrize("p", [1, 3, 5])
def test_sl_reproduces_polynomials(p):
    """Lagrange interpolation of degree p is exact on polynomials of degree <= p:
    sum_j w_j(eps) j^k = (-eps)^k."""
    for eps in (0.0, 0.2, 0.5, 0.77, 0.999):
        w = disc.sl_weights(p, eps)
        for k in range(p + 1):
            assert sum(wj * j ** k for j, wj in w.items()) == pytest.approx((-eps) ** k, abs=1e-13)


@pytest.mark.parametrize("k", [2, 4, 6])
def test_dmat_moments(k):
    """D^(k)_2 annihilates polynomials of degree < k, returns k! h^k on x^k, and is
    symmetric with symbol (2 cos w - 2)^{k/2}."""
    d = disc.dmat_weights(k)
    for deg in range(k):
        assert sum(dj * j ** deg for j, dj in d.items()) == 0
    assert sum(dj * j ** k for j, dj in d.items()) == factorial(k)
    assert all(d[j] == d[-j] for j in d)
    om = np.linspace(-np.pi, np.pi, 9)
    np.testing.assert_allclose(disc.stencil_symbol(d, om).real, (2 * np.cos(om) - 2) ** (k // 2), atol=1e-12)


def test_f_poly_first_order_closed_form():
    for eps in (0.1, 0.4, 0.9):
        assert disc.f_poly(1, eps) == pytest.approx(eps * (eps - 1) / 2)


def _smooth(x, t=0.0):
    # periodic on [-1, 1), advected with unit speed
    y = x - t
    return np.sin(np.pi * y) + 0.5 * np.cos(2 * np.pi * y + 0.3)


def _order(errs, sizes):
    return np.log(errs[0] / errs[-1]) / np.log(sizes[-1] / sizes[0])


@pytest.mark.parametrize("p", [1, 3, 5])
def test_sl_truncation_lemma1(p):
    """Lemma 1: u(t+D) - S u(t) - (-1)^{p+1} f_{p+1}(eps) D u(t+D) = O(h^{p+2}),
    while u(t+D) - S u(t) alone is O(h^{p+1})."""
    sizes = [32, 64, 128]
    with_corr, plain = [], []
    for nx in sizes:
        h = 2.0 / nx
        x = -1 + h * np.arange(nx)
        shift = 3.37
        dt = shift * h
        K, eps = disc.sl_shift(shift)
        unew = _smooth(x, dt)
        lte = unew - disc.sl_apply(_smooth(x), p, shift)
        corr = (-1) ** (p + 1) * disc.f_poly(p, eps) * disc.apply_stencil(unew, disc.dmat_weights(p + 1))
        with_corr.append(np.max(np.abs(lte - corr)))
        plain.append(np.max(np.abs(lte)))
    assert _order(plain, sizes) == pytest.approx(p + 1, abs=0.3)
    assert _order(with_corr, sizes) > p + 1.7


@pytest.mark.parametrize("p,kind,q,c", [(1, "erk", 1, 0.8), (3, "erk", 3, 1.2), (5, "erk", 5, 1.1),
                                        (1, "sdirk", 1, 2.0), (3, "sdirk", 3, 3.0), (5, "sdirk", 3, 0.5)])
def test_mol_truncation_lemma3(p, kind, q, c):
    """Lemma 3 at fixed CFL: removing the predicted leading term
    -[c e_FD D^(p+1) + (-c)^{q+1} e_RK D^(q+1)] u(t+dt) leaves O(h^{p+2}) when
    q >= p (here the O(h dt^{q+1}) term is also O(h^{p+2}))."""
    A, b = disc.tableau(kind, q)
    efd, erk = disc.e_fd_closed_form(p), disc.e_rk(A, b, q)
    sizes = [32, 64, 128, 256]
    errs, plain = [], []
    for nx in sizes:
        h = 2.0 / nx
        x = -1 + h * np.arange(nx)
        dt = c * h
        unew = _smooth(x, dt)
        lte = unew - disc.MOLStep(p, kind, q, c)(_smooth(x))
        lead = -(c * efd * disc.apply_stencil(unew, disc.dmat_weights(p + 1))
                 + (-c) ** (q + 1) * erk * disc.apply_stencil(unew, disc.dmat_weights(q + 1)))
        errs.append(np.max(np.abs(lte - lead)))
        plain.append(np.max(np.abs(lte)))
    order_plain = _order(plain, sizes)
    order_corr = _order(errs, sizes)
    assert order_plain == pytest.approx(min(p, q) + 1, abs=0.3)
    assert order_corr > min(p, q) + 1.6


# --------------------------------------------------------------------------
# phi and Psi (Lemma 4, eqs. MOL-SL-corrected, MOL-SL-corrected-multilevel)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p,kind,q,c,ms", [
    (1, "erk", 1, 0.85, [4]),
    (3, "erk", 3, 0.85, [8]),
    (3, "erk", 3, 1.38, [4]),
    (5, "erk", 5, 0.9, [4]),
    (3, "sdirk", 3, 5.0, [4]),
    (1, "sdirk", 1, 1.0, [16]),
    (3, "erk", 3, 0.85, [4, 4]),
    (3, "erk", 3, 0.85, [4, 2, 2]),
    (1, "erk", 1, 0.7, [4, 4]),
    (5, "sdirk", 3, 0.5, [4]),
    (5, "sdirk", 3, 0.5, [4, 4]),
])
def test_coarse_operator_matches_ideal_to_higher_order(p, kind, q, c, ms):
    """Lemma 4 (and its multilevel form): ||Phi^M u - Psi_L u|| = O(h^{p+2}) with the
    correction coefficients, but only O(h^{p+1}) with phi = 0 (M = prod ms,
    Psi_L the corrected operator of the coarsest listed level).  For the
    mixed-order pairing (q < p, two-term correction) the orders are q+2 and q+1."""
    M = int(np.prod(ms))
    sizes = [64, 128, 256]
    corr, plain = [], []
    for nx in sizes:
        h = 2.0 / nx
        x = -1 + h * np.arange(nx)
        u = _smooth(x)
        fine = disc.MOLStep(p, kind, q, c)
        ideal = u.copy()
        for _ in range(M):
            ideal = fine(ideal)
        rec = disc.correction_coefficients(p, kind, q, c, ms)[-1]
        psi = disc.CorrectedSLStep(p, q, rec["shift"], rec["phi_p"], rec["phi_q"])
        psi0 = disc.CorrectedSLStep(p, q, rec["shift"], 0.0, 0.0)
        corr.append(np.max(np.abs(ideal - psi(u))))
        plain.append(np.max(np.abs(ideal - psi0(u))))
    # with q < p the O(h dt^{q+1}) remainder of Lemma 3 limits both orders
    k = min(p, q)
    assert _order(plain, sizes) == pytest.approx(k + 1, abs=0.35)
    assert _order(corr, sizes) > k + 1.6


def test_phi_two_term_form_reduces_to_paper_when_q_equals_p():
    """With q = p both error terms multiply the same D, and their sum is the
    paper's phi; compare against a direct evaluation of the paper's recursion."""
    p, c, ms = 3, 0.85, [8, 8, 8]
    A, b = disc.erk_tableau(3)
    efd, erk = disc.e_fd_closed_form(3), disc.e_rk(A, b, 3)
    recs = disc.correction_coefficients(p, "erk", 3, c, ms)
    f = lambda e: (e - 2) * (e - 1) * e * (e + 1) / 24.0  # f_4 over j=-2..1
    phis = []
    for lev, m in enumerate(ms, 1):
        eps = (c * 8 ** lev) % 1.0
        if lev == 1:
            phis.append(m * (c * efd + c ** 4 * erk) + f(eps))
        else:
            eps_prev = (c * 8 ** (lev - 1)) % 1.0
            phis.append(-m * f(eps_prev) + f(eps) + m * phis[-1])
    for rec, ph in zip(recs, phis):
        assert rec["phi_q"] == 0.0
        assert rec["phi_p"] == pytest.approx(ph, rel=1e-12, abs=1e-14)


def test_correction_is_dissipative():
    """(-1)^{(p+1)/2} phi <= 0 keeps |1/(1 - phi Dhat)| <= 1 for the paper's
    configurations (so Psi is stable: ||Psi|| <= 1)."""
    om = np.linspace(-np.pi, np.pi, 257)
    for p, kind, q, c, ms in [(1, "erk", 1, 0.85, [4]), (3, "erk", 3, 0.85, [8, 8, 8]),
                              (5, "erk", 5, 0.9, [16, 4, 4]), (3, "sdirk", 3, 5.0, [2] * 7)]:
        for rec in disc.correction_coefficients(p, kind, q, c, ms):
            psi = disc.CorrectedSLStep(p, q, rec["shift"], rec["phi_p"], rec["phi_q"])
            assert np.max(np.abs(psi.symbol(om))) <= 1.0 + 1e-12


def test_dense_corrected_solve_matches_fft_solve():
    """Brute force: build I - phi D as a dense matrix and solve with LU."""
    nx = 24
    rng = np.random.default_rng(6)
    v = rng.random(nx)
    psi = disc.CorrectedSLStep(3, 3, 5.6, -0.7, 0.0)
    d = disc.dmat_weights(4)
    M = np.eye(nx)
    for i in range(nx):
        for j, dj in d.items():
            M[i, (i + j) % nx] -= -0.7 * dj
    S = np.zeros((nx, nx))
    K, eps = disc.sl_shift(5.6)
    for i in range(nx):
        for j, wj in disc.sl_weights(3, eps).items():
            S[i, (i - K + j) % nx] += wj
    np.testing.assert_allclose(psi(v), np.linalg.solve(M, S @ v), atol=1e-13)


def test_caller_tableau_stage_form_matches_its_stability_polynomial():
    """The stage-form step with a caller's tableau (the four-stage
    third-order SSP method) acts on each Fourier mode by its stability
    polynomial R(z) = 1 + z + z^2/2 + z^3/6 + z^4/48 (z = -c Lhat(omega))."""
    A = [[0, 0, 0, 0], [0.5, 0, 0, 0], [0.5, 0.5, 0, 0], [1 / 6, 1 / 6, 1 / 6, 0]]
    b = [1 / 6, 1 / 6, 1 / 6, 0.5]
    nx, c = 64, 0.9
    st = disc.MOLStep(3, "erk", 3, c, (A, b))
    k = 5
    x = np.exp(2j * np.pi * k * np.arange(nx) / nx)
    z = -c * disc.stencil_symbol(disc.upwind_weights(3), 2 * np.pi * k / nx)
    R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 48
    got = st(x.real) + 1j * st(x.imag)
    assert np.max(np.abs(got - R * x)) <= 1e-14


def test_gmres_matches_a_library_gmres_and_the_direct_solve():
    """The oracle's GMRES (zero start, modified Gram-Schmidt, Givens) on the
    corrected coarse operators' periodic systems: stopped at a 1e-2 relative
    residual or 20 iterations it equals scipy's GMRES with the same rule
    (restart 20, one cycle); run to convergence it equals the FFT solve."""
    import scipy.sparse.linalg as sla
    rng = np.random.default_rng(1)
    for rec in disc.correction_coefficients(3, "erk", 3, 0.85 * disc.cfl_limit(3), [8, 8]):
        st = disc.CorrectedSLStep(3, 3, rec["shift"], rec["phi_p"], rec["phi_q"], gmres=(1e-2, 20))
        nx = 256
        b = rng.standard_normal(nx)
        x, k = disc.gmres(st.apply_t, b, 1e-2, 20)
        A = sla.LinearOperator((nx, nx), matvec=lambda v: st.apply_t(np.asarray(v, float)), dtype=float)
        xs, _ = sla.gmres(A, b, rtol=1e-2, atol=0.0, restart=20, maxiter=1)
        assert 1 <= k <= 20
        assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
        res = np.linalg.norm(b - st.apply_t(x)) / np.linalg.norm(b)
        assert res <= 1e-2 or k == 20
        xe, _ = disc.gmres(st.apply_t, b, 1e-15, nx)
        xd = disc.circulant_solve(b, st.corr_weights, 1.0, 1.0)
        assert np.linalg.norm(xe - xd) <= 1e-12 * np.linalg.norm(xd)
