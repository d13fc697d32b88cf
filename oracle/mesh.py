"""Mass assignment, interlacing and compensation (section on modified high-order
multipoles, validation: TSC assignment and eq. compensation).

Readings (the paper prints only the TSC window and says nothing of CIC,
interlacing or node placement):

* Box [0, L)^3, N^3 nodes, spacing H = L/N; node j of mesh A sits at x = jH.
* Grid coordinate u = p N / 2^32 (exact in FP64 for the uint32 positions).
* CIC: i = floor(u), d = u - i, weights (1 - d, d) on nodes (i, i+1).
* TSC: i = floor(u + 1/2), d = u - i in [-1/2, 1/2), weights
  (1/2 (1/2 - d)^2, 3/4 - d^2, 1/2 (1/2 + d)^2) on nodes (i-1, i, i+1).
* Periodic wrap modulo N.  The interlaced mesh B uses u - 1/2 (its node j sits
  at (j + 1/2) H).
* FKP fields: delta_n = n_g - alpha n_r (weights w) and the shot-noise mesh
  N = n_g^(w^2) + alpha^2 n_r^(w^2) (definition of N_l^m under
  eq. generic_noise).
* Interlacing: D(k) = 1/2 [D_A(k) + exp(-i k.(1,1,1) H/2) D_B(k)], every mode
  with a Nyquist component zeroed, then delta_int = IDFT(D) real.
* Compensation W(k) = prod_i sinc(k_i H / 2)^p, p = 2 (CIC) or 3 (TSC),
  sinc x = sin x / x (eq. compensation for p = 3).
* DFT convention: D(k) = sum_x mesh(x) exp(-i k.x) (forward sign of eq. key1),
  k = 2 pi n / L with n in the FFT order 0..N/2-1, -N/2..-1.
"""

from __future__ import annotations

import itertools
import math

import numpy as np

CIC = 2
TSC = 3


def grid_coordinate(pos_u32: np.ndarray, nmesh: int) -> np.ndarray:
    """u = p N / 2^32 in FP64 (exact)."""
    return np.asarray(pos_u32, dtype=np.float64) * (nmesh / 2.0 ** 32)


def stencil(u: np.ndarray, scheme: int):
    """Base node and per-offset weights along one axis."""
    if scheme == CIC:
        i = np.floor(u)
        d = u - i
        return i.astype(np.int64), [(0, 1.0 - d), (1, d)]
    if scheme == TSC:
        i = np.floor(u + 0.5)
        d = u - i
        return i.astype(np.int64), [(-1, 0.5 * (0.5 - d) ** 2), (0, 0.75 - d * d),
                                    (1, 0.5 * (0.5 + d) ** 2)]
    raise ValueError("scheme must be 2 (CIC) or 3 (TSC)")


def paint(pos_u32: np.ndarray, weights, nmesh: int, scheme: int,
          shift: float = 0.0) -> np.ndarray:
    """Sum of weights assigned to the N^3 nodes; ``shift`` = 1/2 gives mesh B."""
    n = pos_u32.shape[1]
    w = np.ones(n) if weights is None else np.asarray(weights, dtype=np.float64)
    base, sten = [], []
    for a in range(3):
        i, s = stencil(grid_coordinate(pos_u32[a], nmesh) - shift, scheme)
        base.append(i)
        sten.append(s)
    mesh = np.zeros(nmesh ** 3)
    for (ox, wx), (oy, wy), (oz, wz) in itertools.product(*sten):
        ix = (base[0] + ox) % nmesh
        iy = (base[1] + oy) % nmesh
        iz = (base[2] + oz) % nmesh
        idx = (ix * nmesh + iy) * nmesh + iz
        mesh += np.bincount(idx, weights=w * wx * wy * wz, minlength=nmesh ** 3)
    return mesh.reshape(nmesh, nmesh, nmesh)


def paint_fkp(gpos, gw, rpos, rw, alpha: float, nmesh: int, scheme: int,
              interlace: bool, noise: bool = True):
    """delta_n and N meshes for phase A (and B when interlacing)."""
    shifts = (0.0, 0.5) if interlace else (0.0,)
    gw2 = None if gw is None else np.asarray(gw, float) ** 2
    rw2 = None if rw is None else np.asarray(rw, float) ** 2
    delta, nmesh_n = [], []
    for s in shifts:
        g = paint(gpos, gw, nmesh, scheme, s)
        r = paint(rpos, rw, nmesh, scheme, s)
        delta.append(g - alpha * r)
        if noise:
            g2 = paint(gpos, gw2, nmesh, scheme, s)
            r2 = paint(rpos, rw2, nmesh, scheme, s)
            nmesh_n.append(g2 + alpha ** 2 * r2)
    return delta, (nmesh_n if noise else None)


def freq_index(nmesh: int) -> np.ndarray:
    """Integer wavenumber index in the FFT order."""
    return np.fft.fftfreq(nmesh, 1.0 / nmesh).round().astype(np.int64)


def wave_indices(nmesh: int):
    n = freq_index(nmesh)
    return n[:, None, None], n[None, :, None], n[None, None, :]


def nyquist_mask(nmesh: int) -> np.ndarray:
    """True for modes with any component at index N/2."""
    nx, ny, nz = wave_indices(nmesh)
    h = nmesh // 2
    return (np.abs(nx) == h) | (np.abs(ny) == h) | (np.abs(nz) == h)


def compensation(nmesh: int, scheme: int) -> np.ndarray:
    """W(k) = prod_i sinc(pi n_i / N)^p on the full grid."""
    w1 = np.sinc(freq_index(nmesh) / nmesh) ** scheme
    return w1[:, None, None] * w1[None, :, None] * w1[None, None, :]


def deinterlace(mesh_a: np.ndarray, mesh_b=None):
    """(D(k), delta_int(x)).  Without mesh B: D = DFT(A), delta_int = A."""
    da = np.fft.fftn(mesh_a)
    if mesh_b is None:
        return da, mesh_a
    nmesh = mesh_a.shape[0]
    nx, ny, nz = wave_indices(nmesh)
    phase = np.exp(-1j * math.pi * (nx + ny + nz) / nmesh)
    d = 0.5 * (da + phase * np.fft.fftn(mesh_b))
    d[nyquist_mask(nmesh)] = 0.0
    return d, np.fft.ifftn(d).real


def node_positions(nmesh: int, boxsize: float):
    """Mesh-A node coordinates x = jH along each axis."""
    return np.arange(nmesh) * (boxsize / nmesh)
