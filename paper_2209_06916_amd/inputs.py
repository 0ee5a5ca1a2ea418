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
* ``initial_iterate_splitmix``: the same distribution from SplitMix64 in
  counter form (the k-th output for point (n, i), k = (n-1) nx + i), the
  generator the library draws with when given a seed instead of an iterate.
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


SPLITMIX_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed, k):
    """Outputs k (an integer array) of SplitMix64 seeded with `seed`: the state
    after k+1 steps is seed + (k+1) * 0x9E3779B97F4A7C15 (mod 2^64), mixed by
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
    z ^= z >> 31 (Steele, Lea and Flood, 2014; all arithmetic mod 2^64)."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (k + np.uint64(1)) * np.uint64(SPLITMIX_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def initial_iterate_splitmix(nt, nx, u0, seed):
    """U[0, 1) at every point (n, i), n >= 1, from the top 53 bits of
    SplitMix64 output k = (n-1) nx + i; row 0 = u0."""
    k = np.arange(nt * nx, dtype=np.uint64)
    v = np.empty((nt + 1, nx))
    v[1:] = ((splitmix64(seed, k) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53).reshape(nt, nx)
    v[0] = u0
    return v
