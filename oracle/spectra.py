"""Yamamoto power-spectrum multipoles (eqs. Hand17, F_ell, hand, new_F_ell,
F_and_new_G, pk_final) and the modified high-order multipoles (eqs. legendre,
Plnew, Pllp; Table 1).

F_l(k) = 4 pi/(2l+1) sum_{m=-l..l} Y_l^m*(khat) DFT[delta_int Y_l^m(xhat)](k) / W(k)
        (eq. hand with the compensation of eq. compensation applied per field)
P_l(k)  = (2l+1)/I22 <Re F_0 F_l*>_k - delta_l0 N0          (eq. Hand17)
P_ll'   = (2(l+l')+1)/I22 <Re F_l F_l'*>_k - N_ll'          (eq. Pllp)
N_22 = 9 N0 / 5, N_44 = 17 N0 / 9, N_42 = 0, N_l0 = delta_l0 N0
P_4b, P_6b, P_8b by eq. Plnew.

Readings:
* xhat = unit vector from the observer to the mesh node (local line of sight),
  or a fixed unit vector (global line of sight, used by tests).
* F_l(0) := 0 (khat undefined at k = 0).
* k-bins are half-open [kmin + b dk, kmin + (b+1) dk); membership is decided on
  the integer n^2 = |n|^2 with thresholds T_b = ceil(((kmin + b dk)/kf)^2),
  kf = 2 pi / L, an edge within a relative 1e-9 of an integer n^2 counting as on
  it.  k = 0 and every mode with a Nyquist component are excluded.
* k_eff = mean |k| over the modes of a bin.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .mesh import node_positions, nyquist_mask, wave_indices
from .ylm import Ylm


@dataclass
class Bins:
    kmin: float
    dk: float
    nbins: int
    boxsize: float
    nmesh: int

    @property
    def kf(self) -> float:
        return 2.0 * math.pi / self.boxsize

    def thresholds(self) -> np.ndarray:
        """Integer n^2 thresholds T_b, b = 0..nbins: the smallest n^2 >= (edge/kf)^2.

        An edge whose square lies within a relative 1e-9 of an integer is taken to
        lie exactly on that integer: the rounding of dk and kf must not move a
        whole lattice shell across a half-open edge."""
        kf = 2.0 * math.pi / self.boxsize
        out = []
        for b in range(self.nbins + 1):
            x = (self.kmin + b * self.dk) / kf
            v = x * x
            r = round(v)
            out.append(int(r) if abs(v - r) <= 1e-9 * max(1.0, v) else math.ceil(v))
        return np.array(out, dtype=np.int64)

    def centres(self) -> np.ndarray:
        return self.kmin + (np.arange(self.nbins) + 0.5) * self.dk

    def shell_index(self) -> np.ndarray:
        """Bin of every mode of the full grid, -1 where excluded."""
        nx, ny, nz = wave_indices(self.nmesh)
        n2 = nx * nx + ny * ny + nz * nz
        t = self.thresholds()
        b = np.searchsorted(t, n2, side="right") - 1
        ok = (b >= 0) & (b < self.nbins) & (n2 > 0) & ~nyquist_mask(self.nmesh)
        return np.where(ok, b, -1)

    def counts(self) -> np.ndarray:
        s = self.shell_index()
        return np.bincount(s[s >= 0], minlength=self.nbins).astype(np.int64)

    def k_eff(self) -> np.ndarray:
        nx, ny, nz = wave_indices(self.nmesh)
        kk = self.kf * np.sqrt((nx * nx + ny * ny + nz * nz).astype(np.float64))
        s = self.shell_index()
        sel = s >= 0
        tot = np.bincount(s[sel], weights=np.broadcast_to(kk, s.shape)[sel],
                          minlength=self.nbins)
        return tot / np.maximum(self.counts(), 1)

    def shell_mean(self, values: np.ndarray) -> np.ndarray:
        """Mean of a (real) full-grid array over each bin."""
        s = self.shell_index()
        sel = s >= 0
        tot = np.bincount(s[sel], weights=np.asarray(values)[sel], minlength=self.nbins)
        return tot / np.maximum(self.counts(), 1)


def kvectors(nmesh: int, boxsize: float) -> np.ndarray:
    nx, ny, nz = wave_indices(nmesh)
    kf = 2.0 * math.pi / boxsize
    shape = (nmesh, nmesh, nmesh)
    return np.stack([np.broadcast_to(nx, shape), np.broadcast_to(ny, shape),
                     np.broadcast_to(nz, shape)], axis=-1).astype(np.float64) * kf


def line_of_sight(nmesh: int, boxsize: float, observer, los=None) -> np.ndarray:
    """Vectors whose directions are xhat at every mesh node, shape (N,N,N,3)."""
    if los is not None:
        v = np.asarray(los, dtype=np.float64)
        return np.broadcast_to(v, (nmesh, nmesh, nmesh, 3))
    x = node_positions(nmesh, boxsize)
    shape = (nmesh, nmesh, nmesh)
    return np.stack([np.broadcast_to(x[:, None, None] - observer[0], shape),
                     np.broadcast_to(x[None, :, None] - observer[1], shape),
                     np.broadcast_to(x[None, None, :] - observer[2], shape)], axis=-1)


def yamamoto_F(delta_int, D, ell, boxsize, observer, W, los=None):
    """F_l(k) on the full grid by the Hand et al. sum over all 2l+1 m (eq. hand)."""
    nmesh = delta_int.shape[0]
    if ell == 0:
        F = D / W
    else:
        rvec = line_of_sight(nmesh, boxsize, observer, los)
        kvec = kvectors(nmesh, boxsize)
        acc = np.zeros(D.shape, dtype=np.complex128)
        for m in range(-ell, ell + 1):
            S = np.fft.fftn(delta_int * Ylm(ell, m, rvec))
            acc += np.conj(Ylm(ell, m, kvec)) * S
        F = (4.0 * math.pi / (2 * ell + 1)) * acc / W
    F = F.copy()
    F[0, 0, 0] = 0.0
    return F


def calG(delta_int, D, ell, boxsize, observer, W, los=None):
    """The inversion-free G_l of eq. new_F_ell: 4pi/(2l+1)[f^0 + 2 sum_{m>=1} f^m]."""
    nmesh = delta_int.shape[0]
    if ell == 0:
        G = D / W
    else:
        rvec = line_of_sight(nmesh, boxsize, observer, los)
        kvec = kvectors(nmesh, boxsize)
        acc = np.zeros(D.shape, dtype=np.complex128)
        for m in range(0, ell + 1):
            S = np.fft.fftn(delta_int * Ylm(ell, m, rvec))
            f = np.conj(Ylm(ell, m, kvec)) * S
            acc += f if m == 0 else 2.0 * f
        G = (4.0 * math.pi / (2 * ell + 1)) * acc / W
    G = G.copy()
    G[0, 0, 0] = 0.0
    return G


def power_raw(Fa, Fb, bins: Bins) -> np.ndarray:
    """<Re F_a F_b*> per bin."""
    return bins.shell_mean(np.real(Fa * np.conj(Fb)))


def power_raw_imag(Fa, Fb, bins: Bins) -> np.ndarray:
    """<Im F_a F_b*> per bin."""
    return bins.shell_mean(np.imag(Fa * np.conj(Fb)))


def pk_multipole_odd(F0, Fl, ell, bins, I22):
    """Odd l: eq. pk_final with the imaginary part taken in place of the real
    part (the sentence after eq. pk_final); the shot noise is zero for l > 0."""
    return (2 * ell + 1) / I22 * power_raw_imag(F0, Fl, bins)


def pk_multipole(F0, Fl, ell, bins, I22, N0):
    """eq. Hand17: (raw, shot-subtracted)."""
    raw = (2 * ell + 1) / I22 * power_raw(F0, Fl, bins)
    return raw, raw - (N0 if ell == 0 else 0.0)


def N_llp(l1: int, l2: int, N0: float) -> float:
    """Shot noise of P_ll' (below eq. Pllp)."""
    table = {(0, 0): 1.0, (2, 2): 9.0 / 5.0, (4, 4): 17.0 / 9.0, (4, 2): 0.0,
             (2, 4): 0.0, (2, 0): 0.0, (0, 2): 0.0, (4, 0): 0.0, (0, 4): 0.0}
    return table[(l1, l2)] * N0


def pk_two_index(Fl1, Fl2, l1, l2, bins, I22, N0):
    """eq. Pllp: (raw, shot-subtracted)."""
    raw = (2 * (l1 + l2) + 1) / I22 * power_raw(Fl1, Fl2, bins)
    return raw, raw - N_llp(l1, l2, N0)


def modified_multipoles(P0, P2, P4, P22, P42, P44):
    """eq. Plnew: P_4b, P_6b, P_8b from shot-subtracted low-l pieces."""
    P4b = 35.0 / 18.0 * P22 - P2 - 3.5 * P0
    P6b = 11.0 / 5.0 * P42 - 52.0 / 63.0 * P4 - 286.0 / 175.0 * P2
    P8b = (1287.0 / 490.0 * P44 - 374.0 / 245.0 * P42 - 3553.0 / 15435.0 * P4
           - 1326.0 / 8575.0 * P2 - 2431.0 / 490.0 * P0)
    return P4b, P6b, P8b


def fft_count(estimator: str, lmax: int) -> int:
    """Table 1 closed forms for even multipoles up to lmax."""
    if estimator == "cartesian":
        return (lmax + 2) * (lmax + 4) * (2 * lmax + 3) // 24
    if estimator == "hand":
        return (lmax + 1) * (lmax + 2) // 2
    if estimator == "symmetry":
        return (lmax + 2) ** 2 // 4
    if estimator == "symmetry+legendre":
        return (lmax + 4) ** 2 // 16
    raise ValueError(estimator)


def fft_count_enumerated(estimator: str, lmax: int) -> int:
    """Table 1 by counting transforms one multipole at a time."""
    ells = range(0, lmax + 1, 2)
    if estimator == "cartesian":
        # F_l needs all monomials x^a y^b z^c with a+b+c = l: (l+1)(l+2)/2.
        return sum((l + 1) * (l + 2) // 2 for l in ells)
    if estimator == "hand":
        return sum(2 * l + 1 for l in ells)
    if estimator == "symmetry":
        return sum(l + 1 for l in ells)
    if estimator == "symmetry+legendre":
        # P_(2L)b needs F_l for l <= L only (L rounded up to even)
        half = (lmax + 1) // 2
        half += half % 2
        return sum(l + 1 for l in range(0, half + 1, 2))
    raise ValueError(estimator)
