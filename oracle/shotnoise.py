"""Analytic bispectrum shot noise (section "Bispectrum Shot Noise from
Triangle-Constrained Spherical-Harmonic Integrals": Lemma 2 / eq. lemma2 and
eq. g_ell, the Scoccimarro, Sugiyama (eqs. Q_ell, H_ell, sugi_shot) and
new-estimator shot-noise results; appendix on the derivation of g_l).

g_l(t) = 1/(2t) int_{|t-1|}^{t+1} x L_l((x^2 + t^2 - 1)/(2 x t)) dx   (practical form)
evaluated with a 64-point Gauss-Legendre rule; the closed forms of
eq. g_first_five are kept as an independent cross-check.

Shell averages used by every shot-noise term (even l, Re parts):
    s_l(k) = < sum_m y_l^m(qhat) Sbar_l^m C(q) / W(q)^2 >_k
    Q_l(k) = < Re F_l(q) N(q)* >_k - s_l(k)       (eq. Q_ell; N = F_0 of the N mesh)
    H_l(k) = < Re F_0(q) F_l^N(q)* >_k - s_l(k)   (eq. H_ell; F_l^N = F_l of the N mesh)

Readings where the paper defers or is garbled:
* C(q): alias sum of the squared window, C = prod_i c(q_i) without interlacing,
  C = 1/2 [prod_i c(q_i) + prod_i c~(q_i)] with interlacing, where
  c = sum_n W1^2(q + 2 k_N n), c~ = sum_n (-1)^n W1^2(q + 2 k_N n), |n| <= 64.
* Scoccimarro (l-leg i, other legs j, k; four coincidence cases, with the
  ring average of eq. I_l0l giving the Legendre factors):
  N^(l) = (2l+1)/I33 [Q_l(k_i) + L_l(mu_ij) H_l(k_j) + L_l(mu_ik) H_l(k_k) + delta_l0 Sbar]
  with mu from bin centres, mu_ij = (k_k^2 - k_i^2 - k_j^2)/(2 k_i k_j), clipped.
* New estimator, B_l0l(k_i, k_j), t = k_i / k_j at bin centres:
  N_l0l = 1/I33 { delta_l0 Sbar + (-1)^l (2l+1) [g_l(t) H_l(k_i) + g_l(1/t) H_l(k_j)]
                  + (2l+1) sum_c N_c Q_l(k_c)/k_c / sum_c N_c/k_c },
  c running over bins |i-j| .. i+j; the i=j=k term carries 1/I33.
* FFT method for the i = j != k term of B_l0l (the two l = 0 legs share a
  particle; section "Validation of the analytical method ...", the FFT
  reference, applied to the new estimator as its shot-noise subsection
  derives that term): no thin-shell step.  With the per-mode product
      P(q) = F_l(q) N(q)^* - s_l(q)        (s_l(q): the summand of s_l above)
  the term is (2l+1)/I33 * T(i, j) / (N_i N_j), where
      T(i, j) = sum_{q1 in shell i, q2 in shell j} Re P(q1 + q2)
  is the grid sum sum_x I_i(x) I_j(x) p(x) / N^3 of the shell indicator fields
  and p = sum_q P(q) e^{iq.x}.  P(0) := 0 (F_l(0) = 0, so the q3 = 0 pairs
  carry neither signal nor noise) and modes with a Nyquist component are zero.
"""

from __future__ import annotations

import math

import numpy as np
from numpy.polynomial.legendre import leggauss

from .mesh import freq_index, nyquist_mask
from .spectra import Bins, kvectors
from .ylm import legendre, ylm_racah

_GL_NODES, _GL_WEIGHTS = leggauss(64)


def g_ell(ell: int, t: float) -> float:
    """g_l(t) from the practical integral form (64-point Gauss-Legendre)."""
    if t == 0.0:
        return 1.0 if ell == 0 else 0.0
    a, b = abs(t - 1.0), t + 1.0
    x = 0.5 * (b - a) * _GL_NODES + 0.5 * (b + a)
    arg = np.clip((x * x + t * t - 1.0) / (2.0 * x * t), -1.0, 1.0)
    return float(0.5 * (b - a) * np.sum(_GL_WEIGHTS * x * legendre(ell, arg)) / (2.0 * t))


def g_ell_closed(ell: int, t: float) -> float:
    """Closed forms of eq. g_first_five (l = 0..4)."""
    if ell == 0:
        return 1.0
    if ell == 1:
        return 2.0 * t / 3.0 if t < 1.0 else 1.0 - 1.0 / (3.0 * t * t)
    if ell == 2:
        if t == 0.0:
            return 0.0
        if t == 1.0:
            return 0.25
        lg = math.log((t + 1.0) / abs(t - 1.0))
        return (2.0 * t * (5.0 * t * t - 3.0) + 3.0 * (t * t - 1.0) ** 2 * lg) / (16.0 * t ** 3)
    if ell == 3:
        return 0.0 if t < 1.0 else (t * t - 1.0) ** 2 / t ** 4
    if ell == 4:
        if t == 0.0:
            return 0.0
        if t == 1.0:
            return -1.0 / 24.0
        lg = math.log((t + 1.0) / abs(t - 1.0))
        return (2.0 * t * (81.0 * t ** 4 - 190.0 * t * t + 105.0)
                + 15.0 * (t * t - 7.0) * (t * t - 1.0) ** 2 * lg) / (192.0 * t ** 5)
    raise ValueError("closed forms exist for l <= 4")


_KAPPA_RULE = {}


def g_ell_kappa(ell: int, t: float, npts: int = 2000) -> float:
    """g_l(t) from the kappa-integral form of eq. g_ell (independent quadrature)."""
    if npts not in _KAPPA_RULE:
        _KAPPA_RULE[npts] = leggauss(npts)
    nodes, weights = _KAPPA_RULE[npts]

    def integrand(k):
        c = np.cos(k)
        val = np.sqrt(np.clip((c * c + t * t + 2 * t * c) / (1 + t * t + 2 * t * c), 0.0, 1.0))
        return 0.5 * np.sin(k) * legendre(ell, val)

    def quad(a, b):
        if b <= a:
            return 0.0
        k = 0.5 * (b - a) * nodes + 0.5 * (b + a)
        return 0.5 * (b - a) * float(np.sum(weights * integrand(k)))

    if t > 1.0:
        return quad(0.0, math.pi)
    k0 = math.acos(-t)
    return quad(0.0, k0) + (-1) ** ell * quad(k0, math.pi)


def alias_tables(nmesh: int, scheme: int, images: int = 64):
    """(c, c~) per FFT-ordered index, FP64 image sums of W1^2 = sinc^(2p)."""
    n = freq_index(nmesh).astype(np.float64)
    c = np.zeros(nmesh)
    ct = np.zeros(nmesh)
    for j in range(-images, images + 1):
        s = np.sinc(n / nmesh + j) ** (2 * scheme)
        c += s
        ct += (-1) ** (j & 1) * s
    return c, ct


def c_shot(nmesh: int, scheme: int, interlace: bool) -> np.ndarray:
    c, ct = alias_tables(nmesh, scheme)
    full = c[:, None, None] * c[None, :, None] * c[None, None, :]
    if not interlace:
        return full
    return 0.5 * (full + ct[:, None, None] * ct[None, :, None] * ct[None, None, :])


def self_term(ell: int, Sbar_lm, bins: Bins, W: np.ndarray, C: np.ndarray) -> np.ndarray:
    """s_l(k): shell mean of sum_m y_l^m(qhat) Sbar_l^m C / W^2 (real part)."""
    kvec = kvectors(bins.nmesh, bins.boxsize)
    acc = np.zeros(W.shape, dtype=np.complex128)
    for m in range(-ell, ell + 1):
        acc += ylm_racah(ell, m, kvec) * Sbar_lm[(ell, m)]
    return bins.shell_mean(np.real(acc) * C / (W * W))


def scoccimarro_shot_terms(ell, configs, Q, H, centres, Sbar):
    """The four coincidence terms of N^(l)(i; j, k) per configuration, before the
    (2l+1)/I33 factor: "jk" = Q_l(k_i) (the two l = 0 legs on one particle),
    "ik" = L_l(mu_ij) H_l(k_j), "ij" = L_l(mu_ik) H_l(k_k) (the l leg shares a
    particle with leg k or j; ring lemma, eq. I_l0l) and "ijk" = delta_l0 Sbar.

    Pinned term by term against the exact closure sums of ``shotnoise_exact``
    (thin-shell tolerance) and, for l = 0, statistically on Poisson catalogs."""
    out = {key: np.empty(len(configs)) for key in ("jk", "ik", "ij", "ijk")}
    for t, (i, j, k) in enumerate(configs):
        ki, kj, kk = centres[i], centres[j], centres[k]
        mu_ij = np.clip((kk * kk - ki * ki - kj * kj) / (2 * ki * kj), -1.0, 1.0)
        mu_ik = np.clip((kj * kj - ki * ki - kk * kk) / (2 * ki * kk), -1.0, 1.0)
        out["jk"][t] = Q[i]
        out["ik"][t] = legendre(ell, mu_ij) * H[j]
        out["ij"][t] = legendre(ell, mu_ik) * H[k]
        out["ijk"][t] = Sbar if ell == 0 else 0.0
    return out


def scoccimarro_shot(ell, configs, Q, H, centres, I33, Sbar):
    """N^(l)(i; j, k) = (2l+1)/I33 (sum of ``scoccimarro_shot_terms``)."""
    terms = scoccimarro_shot_terms(ell, configs, Q, H, centres, Sbar)
    return (2 * ell + 1) / I33 * (terms["jk"] + terms["ik"] + terms["ij"] + terms["ijk"])


def triposh_shot_terms(ell, pairs, Q_ext, H, counts_ext, centres_ext, Sbar):
    """The four coincidence terms of N_l0l(k_i, k_j) per pair, before the 1/I33
    factor: "12" = (2l+1) sum_c N_c Q_l(k_c)/k_c / sum_c N_c/k_c (the two l = 0
    legs on one particle), "13" = (-1)^l (2l+1) g_l(1/t) H_l(k_j) and
    "23" = (-1)^l (2l+1) g_l(t) H_l(k_i) with t = k_i/k_j (the l leg shares a
    particle with the k1 or the k2 leg; Lemma 2, eq. g_ell), "123" = delta_l0 Sbar.

    Pinned term by term against the exact closure sums of ``shotnoise_exact``
    (thin-shell tolerance) and, for l = 0, statistically on Poisson catalogs."""
    out = {key: np.empty(len(pairs)) for key in ("12", "13", "23", "123")}
    sign = -1.0 if ell % 2 else 1.0
    for t, (i, j) in enumerate(pairs):
        tt = centres_ext[i] / centres_ext[j]
        cs = np.arange(abs(i - j), i + j + 1)
        wgt = counts_ext[cs] / centres_ext[cs]
        out["12"][t] = (2 * ell + 1) * float(np.sum(wgt * Q_ext[cs]) / np.sum(wgt))
        out["13"][t] = sign * (2 * ell + 1) * g_ell(ell, 1.0 / tt) * H[j]
        out["23"][t] = sign * (2 * ell + 1) * g_ell(ell, tt) * H[i]
        out["123"][t] = Sbar if ell == 0 else 0.0
    return out


def triposh_shot(ell, pairs, Q_ext, H, counts_ext, centres_ext, I33, Sbar):
    """N_l0l(k_i, k_j) per pair (i <= j) = (sum of ``triposh_shot_terms``) / I33;
    Q_ext etc. extend to bin 2 nbins - 2."""
    terms = triposh_shot_terms(ell, pairs, Q_ext, H, counts_ext, centres_ext, Sbar)
    return (terms["23"] + terms["13"] + terms["12"] + terms["123"]) / I33


def self_term_modes(ell: int, Sbar_lm, nmesh: int, boxsize: float, W: np.ndarray,
                    C: np.ndarray) -> np.ndarray:
    """s_l(q) per mode: Re sum_m y_l^m(qhat) Sbar_l^m C(q) / W(q)^2; 0 at q = 0."""
    kvec = kvectors(nmesh, boxsize)
    zero = np.all(kvec == 0.0, axis=-1)
    safe = np.where(zero[..., None], 1.0, kvec)
    acc = np.zeros(W.shape, dtype=np.complex128)
    for m in range(-ell, ell + 1):
        acc += ylm_racah(ell, m, safe) * Sbar_lm[(ell, m)]
    return np.where(zero, 0.0, np.real(acc) * C / (W * W))


def noise_product(Fl: np.ndarray, FN0: np.ndarray, s_modes: np.ndarray) -> np.ndarray:
    """P(q) = F_l(q) N(q)^* - s_l(q), zero at q = 0 and on Nyquist-component modes."""
    P = Fl * np.conj(FN0) - s_modes
    P = np.where(nyquist_mask(Fl.shape[0]), 0.0, P)
    P[0, 0, 0] = 0.0
    return P


def exact_pair_sums(P: np.ndarray, bins: Bins, pairs) -> np.ndarray:
    """T(i, j) = sum_{q1 in i, q2 in j} Re P(q1 + q2) via sum_x I_i I_j p / N^3."""
    from .bispectrum import indicator_field, triple_sum
    n = P.shape[0]
    n3 = float(n) ** 3
    p = np.fft.ifftn(P).real * n3
    shells = bins.shell_index()
    ind = {b: indicator_field(shells, b) for b in sorted({x for q in pairs for x in q})}
    return np.array([triple_sum(ind[i], ind[j], p) / n3 for i, j in pairs])


def triposh_shot_fft(ell, pairs, T, H, counts, centres, I33, Sbar):
    """N_l0l(k_i, k_j) with the i = j != k term from the exact pair sums T (the
    other terms as in triposh_shot)."""
    out = np.empty(len(pairs))
    sign = -1.0 if ell % 2 else 1.0
    for t, (i, j) in enumerate(pairs):
        tt = centres[i] / centres[j]
        term = sign * (2 * ell + 1) * (g_ell(ell, tt) * H[i] + g_ell(ell, 1.0 / tt) * H[j])
        term += (2 * ell + 1) * T[t] / (float(counts[i]) * float(counts[j]))
        if ell == 0:
            term += Sbar
        out[t] = term / I33
    return out
