"""Cartesian -> real-solid-harmonic matrices for the oracle, fitted numerically.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Convention (the paper is silent on spherical functions; this is the reading used):
row m (m = -l..l) of T_l gives the real solid harmonic
    S_lm(r) = sqrt(4 pi / (2l+1)) r^l Y_lm(theta, phi)    (Racah normalisation)
as a combination of the Cartesian monomials x^ax y^ay z^az of degree l, columns in the
order ax descending, then ay descending. m < 0 are the sin(|m| phi) harmonics, m > 0
the cos(m phi) ones. Sign: in every row the largest-magnitude coefficient is positive
(the first one in column order on ties). l = 0, 1 are never transformed.

The fit evaluates scipy's complex spherical harmonics at random points and solves a
least-squares problem for the monomial coefficients; nothing is taken from a closed
formula, so the independent closed form used by the HIP library can be compared with it.
"""
from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y


def cart_components(l: int):
    return [(ax, ay, l - ax - ay) for ax in range(l, -1, -1) for ay in range(l - ax, -1, -1)]


def real_ylm(l: int, m: int, theta, phi):
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    return np.sqrt(2.0) * (np.real(y) if m > 0 else np.imag(y))


def fit_tsph(l: int, npts: int = 400, seed: int = 7) -> np.ndarray:
    rng = np.random.default_rng(seed + l)
    v = rng.normal(size=(npts, 3))
    r = rng.uniform(0.5, 1.5, size=npts)
    v = v / np.linalg.norm(v, axis=1)[:, None] * r[:, None]
    x, y, z = v[:, 0], v[:, 1], v[:, 2]
    theta = np.arccos(np.clip(z / r, -1.0, 1.0))
    phi = np.arctan2(y, x)
    comps = cart_components(l)
    A = np.stack([x ** a * y ** b * z ** c for a, b, c in comps], axis=1)
    T = np.zeros((2 * l + 1, len(comps)))
    for i, m in enumerate(range(-l, l + 1)):
        target = np.sqrt(4 * np.pi / (2 * l + 1)) * r ** l * real_ylm(l, m, theta, phi)
        coef, *_ = np.linalg.lstsq(A, target, rcond=None)
        coef[np.abs(coef) < 1e-12] = 0.0
        amax = np.max(np.abs(coef))
        first = next(k for k in range(len(coef)) if abs(abs(coef[k]) - amax) <= 1e-9 * amax)
        if coef[first] < 0:
            coef = -coef
        T[i] = coef
    return T


_CACHE = {}


def tsph(l: int) -> np.ndarray:
    if l not in _CACHE:
        _CACHE[l] = fit_tsph(l)
    return _CACHE[l]


def tsph_packed() -> np.ndarray:
    """T2 (5x6) | T3 (7x10) | T4 (9x15), row-major, as the C oracle expects."""
    return np.concatenate([tsph(2).ravel(), tsph(3).ravel(), tsph(4).ravel()])
