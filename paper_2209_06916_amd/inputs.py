"""Seeded synthetic inputs for the advection workloads.

This module holds no part of the method's arithmetic: it only draws initial
conditions and initial MGRIT iterates.  Both the oracle-side tests and the GPU
path take their inputs from here (numpy's PCG64 generator, ``default_rng``).

Recipes (the paper's experiments are synthetic, Sec. 5.3 and Sec. 6.3):
* ``u0_sin4``: u0(x) = sin^4(pi x) on the periodic mesh x_i = x_lo + i h.
* ``u0_fourier``: sum_{k=1}^{16} k^-2 sin(pi k x + theta_k), theta_k ~ U[0, 2 pi)
  (period 2, so periodic on [-1, 1)).
* ``initial_iterate``: uniformly random U[0, 1) at every space-time point
  except t = 0, where it equals u0.
* ``u0_bumps_2d``: 2D, a sum of `count` Gaussian bumps exp(-d^2 / (2 w^2)) of
  amplitude 1 with centres U[-1, 1)^2 and d the minimum-image periodic
  distance on [-1, 1)^2.
"""
import numpy as np


def mesh(nx, x_lo=-1.0, x_hi=1.0):
    h = (x_hi - x_lo) / nx
    return x_lo + h * np.arange(nx)


def u0_sin4(nx, x_lo=-1.0, x_hi=1.0):
    x = mesh(nx, x_lo, x_hi)
    return np.sin(np.pi * x) ** 4


def u0_fourier(nx, seed, modes=16, x_lo=-1.0, x_hi=1.0):
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=modes)
    x = mesh(nx, x_lo, x_hi)
    out = np.zeros(nx)
    for k in range(1, modes + 1):
        out += np.sin(np.pi * k * x + theta[k - 1]) / (k * k)
    return out


def initial_iterate(nt, nx, u0, seed):
    rng = np.random.default_rng(seed)
    v = rng.random((nt + 1, nx))
    v[0] = u0
    return v


def u0_bumps_2d(nx, ny, count, width, seed, lo=-1.0, hi=1.0):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(lo, hi, size=(count, 2))
    L = hi - lo
    x = mesh(nx, lo, hi)[None, :]
    y = mesh(ny, lo, hi)[:, None]
    out = np.zeros((ny, nx))
    for cx, cy in centres:
        dx = (x - cx + L / 2) % L - L / 2
        dy = (y - cy + L / 2) % L - L / 2
        out += np.exp(-(dx * dx + dy * dy) / (2.0 * width * width))
    return out


def sign_vector(n, seed):
    """A seeded vector of +-1 entries: the weights of the per-time-point
    projections that full-size parity tests compare (a random sign vector sees
    an error e of any shape with magnitude about ||e||_2)."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random(n) < 0.5, -1.0, 1.0)
