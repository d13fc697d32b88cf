"""Spherical harmonics for the oracle (appendix on spherical-harmonic identities).

Y_l^m uses the Condon-Shortley phase (the convention the paper states under
eq. key1).  The Racah normalisation is y_l^m = sqrt(4 pi / (2l+1)) Y_l^m.
Evaluated with ``scipy.special.sph_harm_y(l, m, theta, phi)``, theta the polar
angle and phi the azimuth of the vector.
"""

from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y, eval_legendre


def angles(vec: np.ndarray):
    """Polar and azimuthal angles of vectors stacked on the last axis.

    The zero vector is mapped to the +z direction (callers zero such entries).
    """
    vec = np.asarray(vec, dtype=np.float64)
    r = np.sqrt(np.sum(vec * vec, axis=-1))
    safe = np.where(r > 0, r, 1.0)
    cos_t = np.where(r > 0, vec[..., 2] / safe, 1.0)
    theta = np.arccos(np.clip(cos_t, -1.0, 1.0))
    phi = np.arctan2(vec[..., 1], vec[..., 0])
    return theta, phi


def Ylm(ell: int, m: int, vec: np.ndarray) -> np.ndarray:
    """Complex Y_l^m(vec / |vec|), Condon-Shortley phase."""
    theta, phi = angles(vec)
    return sph_harm_y(ell, m, theta, phi)


def ylm_racah(ell: int, m: int, vec: np.ndarray) -> np.ndarray:
    """Racah-normalised y_l^m = sqrt(4 pi / (2l+1)) Y_l^m."""
    return np.sqrt(4.0 * np.pi / (2 * ell + 1)) * Ylm(ell, m, vec)


def legendre(ell: int, x):
    """Legendre polynomial L_l(x)."""
    return eval_legendre(ell, x)
