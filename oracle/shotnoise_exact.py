"""Exact coincidence terms of the Scoccimarro B_l and compressed TripoSH BB_l0l
shot noise: the FFT method of section "Validation of the analytical method in
the Sugiyama estimator" (the reference that needs no thin-shell step) applied
to every term of the generic coincidence decomposition (eq. generic_noise and
the four cases listed before it), for the two estimators of sections
"Scoccimarro estimator" and "Our efficient new estimator".

TEST INFRASTRUCTURE ONLY (see the package docstring).  These sums are the
reference the analytic thin-shell assembly of ``shotnoise`` is pinned against;
they are pinned themselves by an exact particle-level decomposition of the
triple product (``tests/test_oracle_shot_exact.py``).

Notation.  With delta_n = sum_a c_a delta_D(x - x_a) (c_a = w for galaxies,
-alpha w for randoms) and the Racah harmonics y = sqrt(4 pi/(2l+1)) Y:
    F_l(q) = sum_m y_l^m*(qhat) A_m(q),  A_m = DFT[delta y_l^m(xhat)] / W
    N(q)   = DFT[N mesh] / W              (sum_a c_a^2 e^{-iq.x_a})
    M_m(q) = DFT[N mesh y_l^m*(xhat)] / W (sum_a c_a^2 y_l^m*(xhat_a) e^{-iq.x_a})
    Sbar_l^m = sum_a c_a^3 y_l^m*(xhat_a),  C(q) the alias sum of W^2.
Scoccimarro B_l (leg 1 = the l leg on shell i, legs 2, 3 = F_0 on shells j, k):
the triple product F_l(q1) F_0(q2) F_0(q3) over closed triangles splits by
which legs fall on one particle:
    j = k != i:  P(q1)        = F_l(q1) N(q1)^* - s_l(q1)
    i = k != j:  sum_m y_l^m*(q1hat) Z_m(q2),  Z_m = F_0 M_m^* - Sbar_l^m* C / W^2
    i = j != k:  sum_m y_l^m*(q1hat) Z_m(q3)
    i = j = k:   sum_m y_l^m*(q1hat) Sbar_l^m*
The thin-shell forms of ``shotnoise.scoccimarro_shot`` replace the closure
weighted sums by Q_l(k_i), L_l(mu_12) H_l(k_j), L_l(mu_13) H_l(k_k) and
delta_l0 Sbar (the ring lemma, eq. I_l0l).
TripoSH BB_l0l (legs 1, 2 = F_0 on shells i, j; leg 3 = F_l on every mode):
    1 = 2 != 3:  P(q3)
    1 = 3 != 2:  sum_m y_l^m*(q3hat) Z_m(q2)
    2 = 3 != 1:  sum_m y_l^m*(q3hat) Z_m(q1)
    1 = 2 = 3:   sum_m y_l^m*(q3hat) Sbar_l^m*
whose thin-shell forms are the N_c/k_c-weighted Q_l mean, (-1)^l g_l(1/t) H_l(k_j),
(-1)^l g_l(t) H_l(k_i) (Lemma 2, eq. g_ell; t = k_i/k_j) and delta_l0 Sbar.
Each exact sum is a grid triple product of shell-filtered inverse transforms,
sum_x f_1 f_2 f_3 / N^3 = sum over q1 + q2 + q3 = 0 of the three spectra.
Every per-mode spectrum is zero at q = 0 and on modes with a Nyquist component.
"""

from __future__ import annotations

import numpy as np

from .mesh import nyquist_mask
from .spectra import kvectors, line_of_sight
from .ylm import ylm_racah


def _masked(A: np.ndarray) -> np.ndarray:
    out = np.where(nyquist_mask(A.shape[0]), 0.0, A).astype(np.complex128)
    out[0, 0, 0] = 0.0
    return out


def harmonic_spectrum(ell: int, m: int, nmesh: int, boxsize: float) -> np.ndarray:
    """y_l^m*(qhat) per mode (zero at q = 0 and on Nyquist-component modes)."""
    return _masked(np.conj(ylm_racah(ell, m, kvectors(nmesh, boxsize))))


def noise_harmonic_spectra(n_int: np.ndarray, ell: int, boxsize: float, observer, W,
                           los=None):
    """M_m(q) = DFT[N y_l^m*(xhat)] / W for m = -l..l (N: the de-aliased noise mesh)."""
    rvec = line_of_sight(n_int.shape[0], boxsize, observer, los)
    return {m: np.fft.fftn(n_int * np.conj(ylm_racah(ell, m, rvec))) / W
            for m in range(-ell, ell + 1)}


def leg_products(F0: np.ndarray, M: dict, Sbar_lm: dict, ell: int, C: np.ndarray,
                 W: np.ndarray) -> dict:
    """Z_m(q) = F_0(q) M_m(q)^* - Sbar_l^m* C(q) / W(q)^2 per mode."""
    return {m: _masked(F0 * np.conj(M[m]) - np.conj(Sbar_lm[(ell, m)]) * C / (W * W))
            for m in M}


def _shell(A: np.ndarray, shells: np.ndarray, b: int) -> np.ndarray:
    n = A.shape[0]
    return np.fft.ifftn(np.where(shells == b, A, 0.0)) * float(n) ** 3


def _full(A: np.ndarray) -> np.ndarray:
    n = A.shape[0]
    return np.fft.ifftn(_masked(A)) * float(n) ** 3


def _tsum(a, b, c) -> complex:
    return complex(np.sum(a * b * c))


def scoccimarro_exact_terms(ell, configs, shells, P, Z, Sbar_lm, boxsize):
    """Closure sums of the four coincidence cases of B_l per configuration (i, j, k).

    Returns a dict of complex arrays "jk", "ik", "ij", "ijk" (the sums above, before
    the (2l+1)/(I33 N_T) normalisation); their imaginary parts vanish up to rounding.
    """
    n = shells.shape[0]
    n3 = float(n) ** 3
    bins = sorted({x for c in configs for x in c})
    ind = {b: _shell(np.ones(shells.shape, np.complex128), shells, b) for b in bins}
    Pi = {b: _shell(P, shells, b) for b in sorted({c[0] for c in configs})}
    ms = sorted(Z)
    Yi = {(b, m): _shell(harmonic_spectrum(ell, m, n, boxsize), shells, b)
          for b in sorted({c[0] for c in configs}) for m in ms}
    Zb = {(b, m): _shell(Z[m], shells, b) for b in bins for m in ms}
    out = {key: np.zeros(len(configs), np.complex128) for key in ("jk", "ik", "ij", "ijk")}
    for t, (i, j, k) in enumerate(configs):
        out["jk"][t] = _tsum(Pi[i], ind[j], ind[k]) / n3
        for m in ms:
            out["ik"][t] += _tsum(Yi[(i, m)], Zb[(j, m)], ind[k]) / n3
            out["ij"][t] += _tsum(Yi[(i, m)], ind[j], Zb[(k, m)]) / n3
            out["ijk"][t] += np.conj(Sbar_lm[(ell, m)]) * _tsum(Yi[(i, m)], ind[j], ind[k]) / n3
    return out


def triposh_exact_terms(ell, pairs, shells, P, Z, Sbar_lm, boxsize):
    """Sums of the four coincidence cases of BB_l0l per pair (i, j), before the
    (2l+1)/(I33 N_i N_j) normalisation: "12", "13", "23", "123"."""
    n = shells.shape[0]
    n3 = float(n) ** 3
    bins = sorted({x for p in pairs for x in p})
    ind = {b: _shell(np.ones(shells.shape, np.complex128), shells, b) for b in bins}
    ms = sorted(Z)
    p_all = _full(P)
    Yall = {m: _full(harmonic_spectrum(ell, m, n, boxsize)) for m in ms}
    Zb = {(b, m): _shell(Z[m], shells, b) for b in bins for m in ms}
    out = {key: np.zeros(len(pairs), np.complex128) for key in ("12", "13", "23", "123")}
    for t, (i, j) in enumerate(pairs):
        out["12"][t] = _tsum(ind[i], ind[j], p_all) / n3
        for m in ms:
            out["13"][t] += _tsum(ind[i], Zb[(j, m)], Yall[m]) / n3
            out["23"][t] += _tsum(Zb[(i, m)], ind[j], Yall[m]) / n3
            out["123"][t] += np.conj(Sbar_lm[(ell, m)]) * _tsum(ind[i], ind[j], Yall[m]) / n3
    return out
