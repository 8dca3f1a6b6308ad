"""Seeded synthetic inputs for the FMM workloads.

This module only draws random numbers; it holds none of the method's
arithmetic, so the oracle tests, the GPU tests and the benchmark can all use
it without coupling the two implementations.

The paper's three test distributions are the "Cube", "Sphere" and "Plummer"
sets of Table I / Fig. `distribution` (Section III).  Its runs use 10^8 bodies
on a CPU cluster; here the same shapes are drawn at one rank's share:

* ``uniform_cube``  - bodies uniform in [0,1]^3, charges uniform in [-1,1].
* ``plummer``       - Plummer sphere of scale radius 1 truncated at r = 20,
  drawn by inverse-CDF sampling of the enclosed mass (Aarseth, Henon &
  Wielen 1974) with no rejection; isotropic directions.
* ``sphere_surface``- points on the unit sphere's surface (boundary-integral
  style workload): z and the azimuth uniform, which is uniform on the
  surface (Archimedes' hat-box theorem); charges uniform in [-1,1].

All draws use numpy's PCG64 ``default_rng`` in a fixed order, in float64.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_cube",
    "plummer",
    "sphere_surface",
    "sample_targets",
    "adjoint_weights",
    "fd_coordinates",
    "CONFIGS",
    "make_config",
]

# Mass fraction enclosed by r = 20 for a Plummer sphere of scale radius 1.
_M20 = 20.0 ** 3 / (20.0 ** 2 + 1.0) ** 1.5


def uniform_cube(n: int, seed: int = 0):
    """x ~ U[0,1)^3 (n x 3, row-major), q ~ U[-1,1); drawn in that order."""
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3))
    q = rng.uniform(-1.0, 1.0, n)
    return x, q, rng


def _plummer_positions(rng, n: int):
    X = rng.random(n) * _M20
    r = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    ct = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    st = np.sqrt(1.0 - ct * ct)
    x = np.empty((n, 3))
    x[:, 0] = r * st * np.cos(ph)
    x[:, 1] = r * st * np.sin(ph)
    x[:, 2] = r * ct
    return x


def plummer(n: int, seed: int = 0, charges: str = "equal"):
    """Plummer sphere (a = 1, truncated at r = 20).

    charges = "equal": q = 1/n (no extra draw).
    charges = "unit":  q = 1 - U[0,1), i.e. in (0, 1], drawn after positions.
    """
    rng = np.random.default_rng(seed)
    x = _plummer_positions(rng, n)
    if charges == "equal":
        q = np.full(n, 1.0 / n)
    elif charges == "unit":
        q = 1.0 - rng.random(n)
    else:
        raise ValueError(charges)
    return x, q, rng


def sphere_surface(n: int, seed: int = 0):
    """Points on the unit sphere (isotropic), charges uniform in [-1,1]."""
    rng = np.random.default_rng(seed)
    ct = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    st = np.sqrt(1.0 - ct * ct)
    x = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    q = rng.uniform(-1.0, 1.0, n)
    return x, q, rng


def sample_targets(n: int, k: int = 4096, seed=(0, 1)):
    """k distinct target indices in [0, n), sorted ascending."""
    k = min(k, n)
    idx = np.random.default_rng(list(seed)).choice(n, k, replace=False)
    return np.sort(idx).astype(np.int64)


def adjoint_weights(rng, n: int):
    """Loss weights w ~ U[-1,1), drawn from the workload's own stream after q."""
    return rng.uniform(-1.0, 1.0, n)


def fd_coordinates(n: int, k: int = 64, seed=(0, 2)):
    """(particle index, axis) pairs for finite-difference checks."""
    rr = np.random.default_rng(list(seed))
    idx = rr.choice(n, k, replace=False).astype(np.int64)
    ax = rr.integers(0, 3, k).astype(np.int64)
    return idx, ax


# The workloads: (name, n, distribution, p, theta, ncrit)
CONFIGS = {
    "cube16k": dict(n=16384, dist="cube", p=4, theta=0.4, ncrit=64),
    "cube1m": dict(n=1 << 20, dist="cube", p=8, theta=0.4, ncrit=64),
    "plummer4m": dict(n=1 << 22, dist="plummer", p=10, theta=0.35, ncrit=32),
    "cube1m_adjoint": dict(n=1 << 20, dist="cube", p=8, theta=0.4, ncrit=64),
    "plummer16m": dict(n=1 << 24, dist="plummer_unit", p=12, theta=0.3, ncrit=64),
    # Table I case 2 (Sphere) at one rank's share: P, theta and N_crit of the paper
    "sphere4m": dict(n=1 << 22, dist="sphere", p=10, theta=0.4, ncrit=512),
}


def make_config(name: str, n: int | None = None, seed: int = 0):
    """Return (x, q, rng) for a named workload, optionally at a smaller n."""
    c = CONFIGS[name]
    n = c["n"] if n is None else n
    if c["dist"] == "cube":
        return uniform_cube(n, seed)
    if c["dist"] == "plummer":
        return plummer(n, seed, "equal")
    if c["dist"] == "plummer_unit":
        return plummer(n, seed, "unit")
    if c["dist"] == "sphere":
        return sphere_surface(n, seed)
    raise ValueError(c["dist"])
