"""Catalog sums and normalisations (section on the Yamamoto estimator, eq. Hand17;
section on the Scoccimarro estimator, eq. bi_sco; generic shot-noise form,
eq. generic_noise).

With galaxy weights w_g, random weights w_r and alpha = sum w_g / sum w_r:

* I22 = alpha * sum_r nbar w^2                        (under eq. Hand17)
* I33 = alpha * sum_r nbar^2 w^3                      (under eq. bi_sco)
* N0  = (sum_g w^2 + alpha^2 sum_r w^2) / I22         (N_l^shot for l = 0)
* Sbar = sum_g w^3 - alpha^3 sum_r w^3                (the i = j = k Poisson term)
* Sbar_l^m = sum_g w^3 y_l^m*(xhat) - alpha^3 sum_r w^3 y_l^m*(xhat)

Reading (box geometry): nbar is the constant N_g / L^3 and w = 1 unless weights
are given.  xhat is the unit vector from the observer to the particle.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

from .ylm import ylm_racah


def positions(pos_u32: np.ndarray, boxsize: float) -> np.ndarray:
    """Physical positions (n, 3) from the uint32 fixed-point format."""
    return (np.asarray(pos_u32, dtype=np.float64) * (boxsize / 2.0 ** 32)).T


@dataclass
class Norms:
    alpha: float
    nbar: float
    I22: float
    I33: float
    N0: float
    Sbar: float
    sum_w: Tuple[float, float]
    sum_w2: Tuple[float, float]
    sum_w3: Tuple[float, float]
    Sbar_lm: Dict[Tuple[int, int], complex] = field(default_factory=dict)


def _w(w: Optional[np.ndarray], n: int) -> np.ndarray:
    return np.ones(n) if w is None else np.asarray(w, dtype=np.float64)


def catalog_norms(gpos, gw, rpos, rw, boxsize: float, observer: np.ndarray,
                  ells=(0, 2, 4), los: Optional[np.ndarray] = None) -> Norms:
    """All catalog-level FP64 sums; Sbar_l^m for every l in ``ells`` and all m.

    ``los`` (a fixed unit vector) replaces the per-particle line of sight.
    """
    ng, nr = gpos.shape[1], rpos.shape[1]
    wg, wr = _w(gw, ng), _w(rw, nr)
    sg = (math.fsum(wg), math.fsum(wg ** 2), math.fsum(wg ** 3))
    sr = (math.fsum(wr), math.fsum(wr ** 2), math.fsum(wr ** 3))
    alpha = sg[0] / sr[0]
    nbar = ng / boxsize ** 3
    I22 = alpha * nbar * sr[1]
    I33 = alpha * nbar ** 2 * sr[2]
    N0 = (sg[1] + alpha ** 2 * sr[1]) / I22
    Sbar = sg[2] - alpha ** 3 * sr[2]
    out = Norms(alpha, nbar, I22, I33, N0, Sbar, (sg[0], sr[0]), (sg[1], sr[1]),
                (sg[2], sr[2]))
    if los is None:
        xg = positions(gpos, boxsize) - observer
        xr = positions(rpos, boxsize) - observer
    else:
        xg = np.broadcast_to(np.asarray(los, float), (ng, 3))
        xr = np.broadcast_to(np.asarray(los, float), (nr, 3))
    for ell in ells:
        for m in range(-ell, ell + 1):
            yg = np.conj(ylm_racah(ell, m, xg))
            yr = np.conj(ylm_racah(ell, m, xr))
            re = math.fsum(wg ** 3 * yg.real) - alpha ** 3 * math.fsum(wr ** 3 * yr.real)
            im = math.fsum(wg ** 3 * yg.imag) - alpha ** 3 * math.fsum(wr ** 3 * yr.imag)
            out.Sbar_lm[(ell, m)] = complex(re, im)
    return out
