"""Independent reference integrals used to pin the oracle.

These compute the occulted moments directly from their definition,
alpha_n(k, z) = (1/pi) * integral over the occulted part of the stellar disc
of mu^n dA, with mu = sqrt(1 - r^2), without any of the closed forms the
oracle uses.  The limb-darkened flux of both papers' laws is a combination of
these moments (Sect. 2.1.2 and 2.2.1).
"""
from __future__ import annotations

import mpmath as mp
import numpy as np
from scipy.integrate import quad


def alpha_radial(n, k, z, dps=30):
    """alpha_n by a 1-D integral over stellar radius r: the circle of radius r
    lies inside the planet over an arc of half-angle theta(r), so
    alpha_n = (1/pi) int_0^1 mu(r)^n 2 theta(r) r dr.  The integral is split at
    the kinks r = |z-k| and r = z+k (tanh-sinh copes with the endpoint
    square-root behaviour)."""
    with mp.workdps(dps):
        k = mp.mpf(k); z = mp.mpf(z)

        def theta(r):
            if r <= k - z:
                return mp.pi
            if r <= abs(z - k) or r >= z + k:
                return mp.mpf(0)
            c = (r * r + z * z - k * k) / (2 * r * z)
            return mp.acos(max(mp.mpf(-1), min(mp.mpf(1), c)))

        f = lambda r: (1 - r * r) ** (mp.mpf(n) / 2) * 2 * theta(r) * r
        pts = sorted({mp.mpf(0), mp.mpf(1)} | {p for p in (abs(z - k), z + k) if 0 < p < 1})
        return float(mp.quad(f, pts) / mp.pi)


def ma_targets_radial(k, z, dps=30):
    """(alpha_0, alpha_1, alpha_0 - alpha_2) by radial quadrature."""
    a0, a1, a2 = (alpha_radial(n, k, z, dps) for n in (0, 1, 2))
    return np.array([a0, a1, a0 - a2])


def lens_fraction(k, z):
    """Area of the intersection of the unit disc and a disc of radius k at
    distance z, divided by pi (circle-circle overlap, elementary geometry)."""
    if z >= 1 + k:
        return 0.0
    if z <= abs(1 - k):
        return min(1.0, k) ** 2
    # segment areas: r^2 acos(d_i / r) - d_i sqrt(r^2 - d_i^2), d_i chord distances
    d1 = (z * z + 1 - k * k) / (2 * z)        # from the star centre
    d2 = z - d1                               # from the planet centre
    seg1 = np.arccos(np.clip(d1, -1, 1)) - d1 * np.sqrt(max(0.0, 1 - d1 * d1))
    seg2 = k * k * np.arccos(np.clip(d2 / k, -1, 1)) - d2 * np.sqrt(max(0.0, k * k - d2 * d2))
    return (seg1 + seg2) / np.pi


def brute_force_flux(k, z, ld, n_rho=2000, n_psi=2000):
    """Limb-darkened flux by a midpoint rule on a polar grid centred on the
    planet; cells outside the star contribute nothing.  ``ld`` maps mu to the
    normalised intensity I(mu)/I(1) and must be vectorised.  The stellar
    total is integrated separately by adaptive quadrature."""
    rho = (np.arange(n_rho) + 0.5) / n_rho * k
    psi = (np.arange(n_psi) + 0.5) / n_psi * 2 * np.pi
    R, PS = np.meshgrid(rho, psi, indexing="ij")
    x = z + R * np.cos(PS)
    y = R * np.sin(PS)
    r2 = x * x + y * y
    inside = r2 < 1.0
    mu = np.sqrt(np.where(inside, 1 - r2, 0.0))
    dA = R * (k / n_rho) * (2 * np.pi / n_psi)
    blocked = np.sum(np.where(inside, ld(mu), 0.0) * dA)
    # stellar total with r = sin(theta), mu = cos(theta): a smooth integrand
    total = quad(lambda th: float(ld(np.array([np.cos(th)]))[0]) * 2 * np.pi
                 * np.sin(th) * np.cos(th), 0.0, np.pi / 2, epsabs=1e-14, epsrel=1e-13)[0]
    return 1.0 - blocked / total
