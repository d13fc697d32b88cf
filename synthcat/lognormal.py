"""Lognormal / Poisson / tiny synthetic catalogs and fixed-amplitude meshes.

Recipe (stand-in for the survey mocks the paper measures on, which are not
available here):

* Gaussian field on a generation grid of cell 15.625 Mpc/h (64^3 for L = 1000,
  128^3 for L = 2000), power P(k) = 2e4 (k/0.02) / (1 + (k/0.02)^2.5) (Mpc/h)^3
  times the Kaiser factor (b + f mu^2)^2 with b = 2, f = 0.8, and
  mu = khat . n_c, n_c the unit vector from the observer to the box centre.
  The k = 0 mode is zeroed.
* Lognormal density rho = exp(delta_G - sigma_G^2 / 2), sigma_G^2 the realised
  grid variance.
* Galaxies: multinomial with exactly N_g draws over generation cells with
  probability proportional to rho, uniform inside the cell, then randomly
  permuted so the catalog is not cell-ordered.
* Randoms: N_r uniform positions in the box.
* Positions are 3 x uint32 fixed point p = floor(x / L * 2^32), SoA (3, n).
* Seeds: PCG64(1000 * config + 2 * mock) for galaxies, +1 for randoms.

Observer: on the extended body diagonal of the box [0, L)^3, 1500 Mpc/h from
corner 0, i.e. r_obs = -(1500 / sqrt 3) (1, 1, 1).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

OBSERVER_DISTANCE = 1500.0  # Mpc/h from the box corner along the diagonal
GEN_CELL = 15.625  # Mpc/h, generation-grid cell size
BIAS = 2.0
GROWTH_F = 0.8


def observer_position(distance: float = OBSERVER_DISTANCE) -> np.ndarray:
    """Observer on the extended body diagonal, `distance` from corner 0."""
    return -(distance / math.sqrt(3.0)) * np.ones(3)


def field_power(k: np.ndarray) -> np.ndarray:
    """Real-space input power P(k) = 2e4 (k/0.02) / (1 + (k/0.02)^2.5)."""
    x = np.asarray(k, dtype=np.float64) / 0.02
    return 2e4 * x / (1.0 + x ** 2.5)


@dataclass(frozen=True)
class ConfigSpec:
    """Workload description of one benchmark configuration."""

    name: str
    boxsize: float
    nmesh: int
    assign: int  # 2 = CIC, 3 = TSC
    interlace: bool
    ngal: int
    nran: int
    dk: float
    nbins: int
    ells: Tuple[int, ...]
    estimators: Tuple[str, ...] = field(default=())
    nmocks: int = 1


CONFIGS = {
    1: ConfigSpec("c1: Yamamoto P0,2,4 64^3 CIC FP64", 1000.0, 64, 2, False,
                  200_000, 2_000_000, 0.01, 20, (0, 2, 4), ("pk",)),
    2: ConfigSpec("c2: Yamamoto P0..8 (P4b,P6b,P8b) 256^3 TSC+interlacing", 1000.0, 256, 3, True,
                  5_000_000, 25_000_000, 0.01, 20, (0, 2, 4), ("pk", "plb")),
    3: ConfigSpec("c3: Scoccimarro B0,B2 + TripoSH B202 256^3 TSC+interlacing", 1000.0, 256, 3, True,
                  2_000_000, 20_000_000, 0.01, 20, (0, 2), ("bk_scoccimarro", "bk_triposh")),
    4: ConfigSpec("c4: 64 uneven mocks, P0,2,4 + Scoccimarro B0, 256^3 TSC+interlacing", 1000.0, 256, 3, True,
                  0, 0, 0.01, 20, (0, 2, 4), ("pk", "bk_scoccimarro"), nmocks=64),
    5: ConfigSpec("c5: TripoSH B202 512^3 TSC+interlacing, 40 bins dk=0.005", 2000.0, 512, 3, True,
                  30_000_000, 300_000_000, 0.005, 40, (0, 2), ("bk_triposh",)),
}


def config_spec(config: int) -> ConfigSpec:
    return CONFIGS[config]


def mock_sizes_c4(nmocks: int = 64, seed: int = 4999) -> np.ndarray:
    """Galaxy counts of the uneven batch: log-uniform in [1e6, 8e6]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(math.log(1e6), math.log(8e6), size=nmocks)
    return np.rint(np.exp(u)).astype(np.int64)


def _gaussian_field(boxsize: float, ngen: int, rng: np.random.Generator,
                    los: np.ndarray) -> np.ndarray:
    cell_vol = (boxsize / ngen) ** 3
    white = rng.standard_normal((ngen, ngen, ngen))
    wk = np.fft.rfftn(white)
    kf = 2.0 * math.pi / boxsize
    kx = np.fft.fftfreq(ngen, 1.0 / ngen)[:, None, None] * kf
    ky = np.fft.fftfreq(ngen, 1.0 / ngen)[None, :, None] * kf
    kz = np.arange(ngen // 2 + 1)[None, None, :] * kf
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = (kx * los[0] + ky * los[1] + kz * los[2]) / kk
    mu[0, 0, 0] = 0.0
    pk = field_power(kk) * (BIAS + GROWTH_F * mu * mu) ** 2
    amp = np.sqrt(pk / cell_vol)
    amp[0, 0, 0] = 0.0
    return np.fft.irfftn(wk * amp, s=(ngen, ngen, ngen), axes=(0, 1, 2))


def lognormal_catalog(ngal: int, boxsize: float, seed: int,
                      gen_cell: float = GEN_CELL) -> np.ndarray:
    """Galaxy positions (3, ngal) uint32 drawn from a lognormal field."""
    ngen = int(round(boxsize / gen_cell))
    if ngen & (ngen - 1):
        raise ValueError("generation grid must be a power of two")
    rng = np.random.Generator(np.random.PCG64(seed))
    los = np.ones(3) / math.sqrt(3.0)
    delta = _gaussian_field(boxsize, ngen, rng, los)
    sigma2 = float(np.mean(delta * delta))
    rho = np.exp(delta - 0.5 * sigma2).ravel()
    prob = rho / rho.sum()
    counts = rng.multinomial(int(ngal), prob)
    cells = np.repeat(np.arange(ngen ** 3, dtype=np.int64), counts)
    shift = 32 - int(round(math.log2(ngen)))
    ix = cells // (ngen * ngen)
    iy = (cells // ngen) % ngen
    iz = cells % ngen
    pos = np.empty((3, ngal), dtype=np.uint32)
    for a, ia in enumerate((ix, iy, iz)):
        off = rng.integers(0, 1 << shift, size=ngal, dtype=np.uint32)
        pos[a] = (ia.astype(np.uint32) << np.uint32(shift)) + off
    perm = rng.permutation(ngal)
    return np.ascontiguousarray(pos[:, perm])


def random_catalog(nran: int, seed: int) -> np.ndarray:
    """Uniform random positions (3, nran) uint32 covering the whole box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, 1 << 32, size=(3, int(nran)), dtype=np.uint32)


def poisson_catalog(n: int, seed: int) -> np.ndarray:
    """Unclustered 'galaxies': uniform positions, same format as the randoms."""
    return random_catalog(n, seed)


def tiny_catalog(ngal: int = 50, nran: int = 200, seed: int = 7,
                 weights: bool = False):
    """Small catalogs for brute-force checks; optional positive FP32 weights."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.integers(0, 1 << 32, size=(3, ngal), dtype=np.uint32)
    r = rng.integers(0, 1 << 32, size=(3, nran), dtype=np.uint32)
    if not weights:
        return g, None, r, None
    gw = rng.uniform(0.5, 1.5, size=ngal).astype(np.float32)
    rw = rng.uniform(0.5, 1.5, size=nran).astype(np.float32)
    return g, gw, r, rw


def fixed_amplitude_mesh(nmesh: int, boxsize: float, seed: int,
                         los=(0.0, 0.0, 1.0), bias: float = BIAS,
                         growth: float = GROWTH_F) -> np.ndarray:
    """Real mesh whose DFT has |delta(k)|^2 = P(k)(b + f mu^2)^2 N^6 / V exactly.

    Phases are random (seeded), mu = khat . los, k = 0 and every Nyquist mode
    are zero.  The DFT convention is delta(k) = sum_x delta(x) exp(-i k.x).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    los = np.asarray(los, dtype=np.float64)
    los = los / np.linalg.norm(los)
    white = rng.standard_normal((nmesh, nmesh, nmesh))
    wk = np.fft.rfftn(white)
    kf = 2.0 * math.pi / boxsize
    nx = np.fft.fftfreq(nmesh, 1.0 / nmesh)[:, None, None]
    ny = np.fft.fftfreq(nmesh, 1.0 / nmesh)[None, :, None]
    nz = np.arange(nmesh // 2 + 1)[None, None, :]
    kk = kf * np.sqrt(nx * nx + ny * ny + nz * nz)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = kf * (nx * los[0] + ny * los[1] + nz * los[2]) / kk
    mu[0, 0, 0] = 0.0
    target = field_power(kk) * (bias + growth * mu * mu) ** 2 * nmesh ** 6 / boxsize ** 3
    mag = np.abs(wk)
    mag[mag == 0] = 1.0
    dk = wk / mag * np.sqrt(target)
    half = nmesh // 2
    dk[0, 0, 0] = 0.0
    dk[half, :, :] = 0.0
    dk[:, half, :] = 0.0
    dk[:, :, half] = 0.0
    return np.fft.irfftn(dk, s=(nmesh, nmesh, nmesh), axes=(0, 1, 2))
