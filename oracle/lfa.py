"""Local Fourier analysis of two-level MGRIT (oracle; test infrastructure only).

Sec. 5.1: lambda(omega) and mu(omega) are the symbols of the fine and coarse
time-steppers; the two-level estimate for the space-time mode (omega, theta) is
eq. (rho-omega-theta) and its worst case over theta is eq. (rho-asym).
"""
import numpy as np

from . import discretization as disc


def omega_samples(n=1 << 11, drop_near_zero=10):
    """n equispaced samples of [-pi, pi) without omega = 0 and the
    ``drop_near_zero`` samples nearest to it (footnote to eq. rho-asym)."""
    om = -np.pi + 2.0 * np.pi * np.arange(n) / n
    order = np.argsort(np.abs(om))
    keep = np.ones(n, dtype=bool)
    keep[order[: 1 + drop_near_zero]] = False
    return om[keep]


def rho_mode(lam, mu, m, nu, theta):
    """eq. (rho-omega-theta)."""
    return (np.abs(lam) ** (m * nu) * np.abs(lam ** m - mu)
            / np.abs(1.0 - np.exp(-1j * m * theta) * mu))


def rho_two_level(lam, mu, m, nu):
    """eq. (rho-asym): max over omega of |lam|^{m nu} |lam^m - mu| / (1 - |mu|)
    (infinite when some |mu| = 1, e.g. an uncorrected SL step at integer shift)."""
    with np.errstate(divide="ignore"):
        return float(np.max(np.abs(lam) ** (m * nu) * np.abs(lam ** m - mu) / (1.0 - np.abs(mu))))


def rho_for(p, kind, q, c, m, nu=1, coarse="sl_corrected", n=1 << 11, drop=10, tab=None):
    """Two-level LFA estimate for the fine step (kind, q)+Up at CFL c and
    coarsening factor m with the given coarse operator (tab: an optional
    Butcher tableau in place of the built-in one)."""
    om = omega_samples(n, drop)
    fine = disc.MOLStep(p, kind, q, c, tab)
    lam = fine.symbol(om)
    if coarse == "redisc":
        mu = disc.MOLStep(p, kind, q, m * c, tab).symbol(om)
    else:
        rec = disc.correction_coefficients(p, kind, q, c, [m], tab)[0]
        if coarse == "sl_plain":
            st = disc.CorrectedSLStep(p, q, rec["shift"], 0.0, 0.0)
        else:
            st = disc.CorrectedSLStep(p, q, rec["shift"], rec["phi_p"], rec["phi_q"])
        mu = st.symbol(om)
    return rho_two_level(lam, mu, m, nu)


def rho_check(p, efd, erk_fine, erk_coarse, c, m):
    """Theorem 1's lower bound, eq. (rho-check-MOL), for a rediscretised
    coarse operator."""
    return c ** p * abs((erk_fine - m ** p * erk_coarse) / (efd + (m * c) ** p * erk_coarse))
