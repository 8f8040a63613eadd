"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.

This module holds no transform arithmetic: only random draws, the spectral
amplitude profiles of the workloads and index bookkeeping.

Workloads (each draw in one call, in m-major triangular order):
  * "inv1":  re, im ~ N(0, sigma_n^2) with sigma_n = (n+1)^-1;
  * "k3":    sigma_n = (n+1)^(-3/2) (2n+1)^(-1/2), i.e. an energy spectrum
             E(n) ~ (n+1)^-3 spread over the 2n+1 orders of degree n;
  * "white": sigma_n = 1, every coefficient of every degree with the same
             variance, so that an error confined to a few degrees or orders
             is as visible as one spread over all of them;
  * "uniform13": re, im ~ U[(n+1)^(-1/3), 2 (n+1)^(-1/3)], the random spectra
             of the paper's aliasing experiment (Sec. 4.2).
Im of every m = 0 coefficient is set to 0 (real fields).
"""

import numpy as np


def ncoef(N):
    return (N + 1) * (N + 2) // 2


def degrees(N):
    """Total wavenumber n of every slot of the m-major triangular array."""
    return np.concatenate([np.arange(m, N + 1) for m in range(N + 1)])


def orders(N):
    """Zonal wavenumber m of every slot of the m-major triangular array."""
    return np.concatenate([np.full(N + 1 - m, m) for m in range(N + 1)])


def sigma(N, profile):
    n = degrees(N).astype(np.float64)
    if profile == "inv1":
        return 1.0 / (n + 1.0)
    if profile == "k3":
        return (n + 1.0) ** -1.5 * (2.0 * n + 1.0) ** -0.5
    if profile == "white":
        return np.ones_like(n)
    raise ValueError("unknown spectral profile %r" % (profile,))


def random_spectra(N, F, seed=0, profile="k3"):
    """[F, ncoef, 2] float64 spectra; Im of m = 0 is zero."""
    rng = np.random.default_rng(seed)
    if profile == "uniform13":
        n = degrees(N).astype(np.float64)
        lo = (n + 1.0) ** (-1.0 / 3.0)
        u = rng.random((F, ncoef(N), 2))
        s = lo[None, :, None] * (1.0 + u)
    else:
        s = rng.standard_normal((F, ncoef(N), 2)) * sigma(N, profile)[None, :, None]
    s[:, orders(N) == 0, 1] = 0.0
    return s


def random_grid(F, J, I, seed=0):
    """[F, J, I] float64 standard-normal grid values (not band-limited; the
    transforms are linear maps defined for any grid)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((F, J, I))


def loss_weights(shape, seed=1):
    """c ~ U(0.5, 1.5) for the quadratic test loss sum(c * y^2)."""
    rng = np.random.default_rng(seed)
    return 0.5 + rng.random(shape)
