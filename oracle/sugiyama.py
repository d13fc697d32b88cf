"""Sugiyama bispectrum multipoles B_l1l2L (section "Sugiyama estimator": the
tripolar expansion, eq. sugi_estimator with eq. F_and_G) and their analytic
shot noise (subsection "Sugiyama estimator" of the shot-noise derivation:
eq. S3_sugi_new with eq. q_ells, and eq. sugi_shot).  Test infrastructure of
the GPU library; plain FP64 numpy.

Definitions, with y_l^m the Racah-normalised harmonics (Condon-Shortley):
    F_l^m(x; k) = 1/N_k  sum_{q in shell k} e^{iq.x} y_l^m*(qhat) F_0(q)
    G_L^M(x)    = sum_{all q} e^{iq.x} dn_L^M(q) / W(q),
    dn_L^M(q)   = sum_x e^{-iq.x} delta(x) y_L^M*(xhat)   (delta: the
                  de-interlaced FKP mesh, xhat from the observer to the node)
    B(k1, k2)   = H N / I33 sum_{m1 m2 M} (l1 l2 L; m1 m2 M)
                  1/N^3 sum_x F_l1^m1(x; k1) F_l2^m2(x; k2) G_L^M(x)
with F_0 = D / W the compensated density spectrum (F_0(0) = 0), G zero at
q = 0 and on modes with a Nyquist component, H = (l1 l2 L; 0 0 0) and
N = (2l1+1)(2l2+1)(2L+1).  The oracle sums over every (m1, m2, M); the sum is
real (its imaginary part is a test), and the pairing of (m1, m2, M) with
(-m1, -m2, -M) into eta Re[...] is checked against it, not used by it.

Shot noise (the four coincidence terms):
    S|i=j=k      = delta_l10 delta_l20 delta_L0 Sbar / I33
    S|i!=j=k(k1) = delta_l1L delta_l20 (2L+1)/I33 H_L(k1)
    S|i=k!=j(k2) = delta_l2L delta_l10 (2L+1)/I33 H_L(k2)
    S|i=j!=k     = H N / I33 sum_c q(k1, k2, k_c) N_c Q_L(k_c)/k_c / sum_c N_c/k_c
    q(k1,k2,k3)  = sum_n (-1)^n Lr_l1^n(k1hat.k3hat) Lr_l2^-n(k2hat.k3hat) (l1 l2 L; n -n 0)
with Q_L, H_L the shell means of the other estimators, c over the bins
|i-j| .. i+j, cosines from bin centres of the closed triangle, and Lr_l^n the
Racah-normalised associated Legendre functions, y_l^n(theta, phi = 0).

Pins: the estimator against a direct sum over mode pairs, B_000 against the
compressed BB_000, realness, the pairing identity and the conjugation
symmetries.  The shot noise is pinned by its (0, 0, 0) reduction to the
compressed estimator's, by q_l0l = L_l (l 0 l; 0 0 0), by q_l1l2L equal to the
frame-free invariant of the three closed-triangle directions (spherical
harmonics from scipy, any orientation, l1, l2 > 0 included), and for (0, 0, 0),
(2, 0, 2) and (4, 0, 4) by the FFT method on a Poisson catalog (thin-shell
tolerance, lowest bins aside for (0, 0, 0) and (4, 0, 4)); for l1, l2 > 0 the
i = j != k term is a small residual that the FFT method does not resolve on
such catalogs, so its bin sum over c is pinned only through the l2 = 0 cases,
which share it.  The FFT-method term is pinned by a
direct sum over mode pairs and, for (0, 0, 0), by the compressed estimator's
FFT-method noise.

FFT method for the i = j != k term (the reference method of the section that
validates the analytic noise; no thin-shell step):
    S^FFT|i=j!=k = H N / I33 sum_{m1 m2 M} (l1 l2 L; m1 m2 M)
                   1/N^3 sum_x Y_l1^m1(x; k1) Y_l2^m2(x; k2) P_L^M(x)
    Y_l^m(x; k)  = 1/N_k sum_{q in shell k} e^{iq.x} y_l^m*(qhat)
    P_L^M(x)     = sum_q e^{iq.x} [dn_L^M(q)/W(q) N_0(q)^*/W(q) - Sbar_L^M C(q)/W(q)^2]
with N_0 the FFT of the N mesh, zero at q = 0 and on Nyquist-component modes.

Readings (the paper leaves these open): I = I33; dn_L^M carries y_L^M* of
the position (the conjugate of the printed weighting, so that
sum_M y_L^M(khat) y_L^M*(xhat) is the Legendre kernel); the k3 weighting of
the i = j != k term as for the compressed estimator (N_c / k_c); L even
(plane-parallel symmetry), so l1 + l2 even.
"""

from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from .mesh import nyquist_mask
from .spectra import Bins, kvectors, line_of_sight
from .ylm import ylm_racah


def wigner3j(j1: int, j2: int, j3: int, m1: int, m2: int, m3: int) -> float:
    """Wigner 3j symbol by the Racah formula (exact rational arithmetic, then
    one square root)."""
    if m1 + m2 + m3 != 0 or j3 < abs(j1 - j2) or j3 > j1 + j2:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(m3) > j3:
        return 0.0
    f = math.factorial
    tri = Fraction(f(j1 + j2 - j3) * f(j1 - j2 + j3) * f(-j1 + j2 + j3), f(j1 + j2 + j3 + 1))
    pref = tri * f(j1 + m1) * f(j1 - m1) * f(j2 + m2) * f(j2 - m2) * f(j3 + m3) * f(j3 - m3)
    s = Fraction(0)
    for k in range(0, j1 + j2 + j3 + 1):
        d = [k, j1 + j2 - j3 - k, j1 - m1 - k, j2 + m2 - k, j3 - j2 + m1 + k, j3 - j1 - m2 + k]
        if min(d) < 0:
            continue
        den = 1
        for x in d:
            den *= f(x)
        s += Fraction((-1) ** k, den)
    sign = -1.0 if (j1 - j2 - m3) % 2 else 1.0
    return sign * math.sqrt(pref) * float(s)


def racah_assoc_legendre(ell: int, n: int, mu: float) -> float:
    """Lr_l^n(mu) = y_l^n(theta, phi = 0) with cos theta = mu."""
    st = math.sqrt(max(0.0, 1.0 - mu * mu))
    v = np.array([st, 0.0, mu])
    return float(np.real(ylm_racah(ell, n, v)))


def sub_configs(l1: int, l2: int, L: int, paired: bool = False):
    """(m1, m2, M, weight) with m1 + m2 + M = 0 and non-zero 3j symbol; weight
    is the 3j symbol, or eta times it for the paired selection (M < 0, or
    M = 0 with m1 <= 0; eta = 1 for (0, 0, 0), 2 otherwise)."""
    out = []
    for M in range(-L, L + 1):
        for m1 in range(-l1, l1 + 1):
            m2 = -m1 - M
            if abs(m2) > l2:
                continue
            w = wigner3j(l1, l2, L, m1, m2, M)
            if w == 0.0:
                continue
            if paired:
                if M > 0 or (M == 0 and m1 > 0):
                    continue
                w *= 1.0 if (m1, m2, M) == (0, 0, 0) else 2.0
            out.append((m1, m2, M, w))
    return out


def shell_fields_lm(F0: np.ndarray, bins: Bins, ell: int, m: int):
    """F_l^m(x; k) for every shell (complex, N^3 each), including the 1/N_k."""
    n = F0.shape[0]
    kvec = kvectors(n, bins.boxsize)
    zero = np.all(kvec == 0.0, axis=-1)
    safe = np.where(zero[..., None], 1.0, kvec)
    yc = np.where(zero, 0.0, np.conj(ylm_racah(ell, m, safe)))
    shells = bins.shell_index()
    counts = bins.counts()
    out = []
    for b in range(bins.nbins):
        spec = np.where(shells == b, yc * F0, 0.0)
        out.append(np.fft.ifftn(spec) * n ** 3 / max(int(counts[b]), 1))
    return out


def los_field(delta_int: np.ndarray, W: np.ndarray, L: int, M: int, boxsize: float, observer,
              los=None) -> np.ndarray:
    """G_L^M(x) (complex N^3)."""
    n = delta_int.shape[0]
    rvec = line_of_sight(n, boxsize, observer, los)
    dn = np.fft.fftn(delta_int * np.conj(ylm_racah(L, M, rvec)))
    spec = np.where(nyquist_mask(n), 0.0, dn / W)
    spec[0, 0, 0] = 0.0
    return np.fft.ifftn(spec) * n ** 3


def sugiyama_raw(F0, delta_int, W, l1, l2, L, bins: Bins, I33, boxsize, observer, los=None,
                 return_imag=False):
    """B_l1l2L(k_i, k_j) for every (i, j) (nbins x nbins), eq. sugi_estimator
    summed over every (m1, m2, M)."""
    n = F0.shape[0]
    H = wigner3j(l1, l2, L, 0, 0, 0)
    Nn = (2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1)
    nb = bins.nbins
    acc = np.zeros((nb, nb), dtype=np.complex128)
    cacheF = {}
    cacheG = {}
    for m1, m2, M, w in sub_configs(l1, l2, L):
        if (l1, m1) not in cacheF:
            cacheF[(l1, m1)] = shell_fields_lm(F0, bins, l1, m1)
        if (l2, m2) not in cacheF:
            cacheF[(l2, m2)] = shell_fields_lm(F0, bins, l2, m2)
        if M not in cacheG:
            cacheG[M] = los_field(delta_int, W, L, M, boxsize, observer, los)
        A, B, G = cacheF[(l1, m1)], cacheF[(l2, m2)], cacheG[M]
        for i in range(nb):
            AG = A[i] * G
            for j in range(nb):
                acc[i, j] += w * np.sum(AG * B[j])
    val = H * Nn / I33 * acc / float(n) ** 3
    if return_imag:
        return val.real, val.imag
    return val.real


def q_factor(l1: int, l2: int, L: int, k1: float, k2: float, k3: float) -> float:
    """q_l1l2L of eq. q_ells with the cosines of the closed triangle."""
    mu13 = np.clip((k2 * k2 - k1 * k1 - k3 * k3) / (2 * k1 * k3), -1.0, 1.0)
    mu23 = np.clip((k1 * k1 - k2 * k2 - k3 * k3) / (2 * k2 * k3), -1.0, 1.0)
    s = 0.0
    for nn in range(-min(l1, l2), min(l1, l2) + 1):
        w = wigner3j(l1, l2, L, nn, -nn, 0)
        if w == 0.0:
            continue
        s += (-1) ** (nn & 1) * racah_assoc_legendre(l1, nn, mu13) * racah_assoc_legendre(l2, -nn, mu23) * w
    return s


def sugiyama_shot(l1, l2, L, nbins, Q_ext, H, counts_ext, centres_ext, I33, Sbar):
    """S_l1l2L(k_i, k_j) for every (i, j), the four terms above."""
    Hs = wigner3j(l1, l2, L, 0, 0, 0)
    Nn = (2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1)
    out = np.zeros((nbins, nbins))
    for i in range(nbins):
        for j in range(nbins):
            v = 0.0
            if l1 == 0 and l2 == 0 and L == 0:
                v += Sbar
            if l1 == L and l2 == 0:
                v += (2 * L + 1) * H[i]
            if l2 == L and l1 == 0:
                v += (2 * L + 1) * H[j]
            cs = np.arange(abs(i - j), i + j + 1)
            wgt = counts_ext[cs] / centres_ext[cs]
            qs = np.array([q_factor(l1, l2, L, centres_ext[i], centres_ext[j], centres_ext[c]) for c in cs])
            v += Hs * Nn * float(np.sum(wgt * qs * Q_ext[cs]) / np.sum(wgt))
            out[i, j] = v / I33
    return out


def harmonic_indicators(bins: Bins, ell: int, m: int, nmesh: int):
    """Y_l^m(x; k) for every shell (complex), including the 1/N_k."""
    ones = np.ones((nmesh,) * 3, dtype=np.complex128)
    return shell_fields_lm(ones, bins, ell, m)


def noise_los_field(delta_int, W, FN0, C, Sbar_lm, L, M, boxsize, observer, los=None):
    """P_L^M(x) (complex N^3); FN0 = N_0 / W."""
    n = delta_int.shape[0]
    rvec = line_of_sight(n, boxsize, observer, los)
    dn = np.fft.fftn(delta_int * np.conj(ylm_racah(L, M, rvec)))
    spec = dn / W * np.conj(FN0) - Sbar_lm[(L, M)] * C / (W * W)
    spec = np.where(nyquist_mask(n), 0.0, spec)
    spec[0, 0, 0] = 0.0
    return np.fft.ifftn(spec) * n ** 3


def sugiyama_fft_term(delta_int, W, FN0, C, Sbar_lm, l1, l2, L, bins: Bins, I33, boxsize, observer,
                      los=None, return_imag=False):
    """S^FFT|i=j!=k (nbins x nbins), summed over every (m1, m2, M)."""
    n = delta_int.shape[0]
    H = wigner3j(l1, l2, L, 0, 0, 0)
    Nn = (2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1)
    nb = bins.nbins
    acc = np.zeros((nb, nb), dtype=np.complex128)
    cY, cP = {}, {}
    for m1, m2, M, w in sub_configs(l1, l2, L):
        for key in ((l1, m1), (l2, m2)):
            if key not in cY:
                cY[key] = harmonic_indicators(bins, key[0], key[1], n)
        if M not in cP:
            cP[M] = noise_los_field(delta_int, W, FN0, C, Sbar_lm, L, M, boxsize, observer, los)
        A, B, Pm = cY[(l1, m1)], cY[(l2, m2)], cP[M]
        for i in range(nb):
            AP = A[i] * Pm
            for j in range(nb):
                acc[i, j] += w * np.sum(AP * B[j])
    val = H * Nn / I33 * acc / float(n) ** 3
    if return_imag:
        return val.real, val.imag
    return val.real


def sugiyama_shot_fft(l1, l2, L, nbins, fft_term, H, I33, Sbar):
    """S_l1l2L with the i = j != k term from the FFT method."""
    out = np.array(fft_term, dtype=np.float64).copy()
    for i in range(nbins):
        for j in range(nbins):
            v = 0.0
            if l1 == 0 and l2 == 0 and L == 0:
                v += Sbar
            if l1 == L and l2 == 0:
                v += (2 * L + 1) * H[i]
            if l2 == L and l1 == 0:
                v += (2 * L + 1) * H[j]
            out[i, j] += v / I33
    return out


def real_harmonic_matrix(ell: int) -> np.ndarray:
    """V^l of the real spherical harmonics X_lm = sum_n V_mn Y_l^n (appendix on
    spherical harmonics: X for m < 0, m = 0, m > 0), rows and columns m, n =
    -l..l."""
    V = np.zeros((2 * ell + 1, 2 * ell + 1), dtype=np.complex128)
    r2 = 1.0 / math.sqrt(2.0)
    for m in range(-ell, ell + 1):
        i = m + ell
        if m < 0:
            V[i, m + ell] = 1j * r2
            V[i, -m + ell] = -1j * r2 * (-1) ** (m & 1)
        elif m == 0:
            V[i, ell] = 1.0
        else:
            V[i, -m + ell] = r2
            V[i, m + ell] = r2 * (-1) ** (m & 1)
    return V


def tripolar_real_coeffs(l1: int, l2: int, L: int) -> np.ndarray:
    """A^{n1 n2 N}_{l1 l2 L} of the real decomposition of the tripolar basis:
    1/H sum_{m1 m2 M} U_m1n1 U_m2n2 U_MN (l1 l2 L; m1 m2 M), U = V^-1; indexed
    [n1 + l1, n2 + l2, N + L] (complex array; real for an isotropic basis)."""
    H = wigner3j(l1, l2, L, 0, 0, 0)
    U1 = np.linalg.inv(real_harmonic_matrix(l1))
    U2 = np.linalg.inv(real_harmonic_matrix(l2))
    U3 = np.linalg.inv(real_harmonic_matrix(L))
    A = np.zeros((2 * l1 + 1, 2 * l2 + 1, 2 * L + 1), dtype=np.complex128)
    for m1 in range(-l1, l1 + 1):
        for m2 in range(-l2, l2 + 1):
            M = -m1 - m2
            if abs(M) > L:
                continue
            w = wigner3j(l1, l2, L, m1, m2, M)
            if w == 0.0:
                continue
            A += w * np.einsum("a,b,c->abc", U1[m1 + l1], U2[m2 + l2], U3[M + L])
    return A / H
