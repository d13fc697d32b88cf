"""Pins of the oracle's spherical harmonics, mass assignment and interlacing.

Spherical harmonics: textbook Cartesian forms, Y_l^m(zhat), conjugation and
parity (appendix on spherical-harmonic identities, eq. sph_prop), the addition
theorem (eq. add_theorem).  Mass assignment: mass conservation, hand-computed
single-particle weights, whole-cell translation, and the exact Poisson-summation
spectrum of one painted particle (which fixes the kernel shape, node placement,
the interlacing shift and the phase sign at once).
"""

import math

import numpy as np
import pytest

from oracle import mesh as ms
from oracle.ylm import Ylm, legendre


def _rand_vecs(n, seed=1):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(n, 3))


def test_ylm_cartesian_textbook():
    v = _rand_vecs(50)
    x, y, z = v.T
    r = np.linalg.norm(v, axis=1)
    xp = (x + 1j * y) / r
    ct = z / r
    assert np.allclose(Ylm(1, 1, v), -0.5 * math.sqrt(3 / (2 * math.pi)) * xp, atol=1e-14)
    assert np.allclose(Ylm(1, 0, v), 0.5 * math.sqrt(3 / math.pi) * ct, atol=1e-14)
    assert np.allclose(Ylm(2, 0, v), 0.25 * math.sqrt(5 / math.pi) * (3 * ct ** 2 - 1), atol=1e-14)
    assert np.allclose(Ylm(2, 1, v), -0.5 * math.sqrt(15 / (2 * math.pi)) * xp * ct, atol=1e-14)
    assert np.allclose(Ylm(2, 2, v), 0.25 * math.sqrt(15 / (2 * math.pi)) * xp ** 2, atol=1e-14)
    assert np.allclose(Ylm(4, 4, v), (3 / 16) * math.sqrt(35 / (2 * math.pi)) * xp ** 4, atol=1e-14)


@pytest.mark.parametrize("ell", [0, 1, 2, 3, 4, 6, 8])
def test_ylm_identities(ell):
    v = _rand_vecs(40, seed=ell + 3)
    zhat = np.array([[0.0, 0.0, 2.5]])
    for m in range(-ell, ell + 1):
        expect = math.sqrt((2 * ell + 1) / (4 * math.pi)) if m == 0 else 0.0
        assert abs(Ylm(ell, m, zhat)[0] - expect) < 1e-14
        assert np.allclose(Ylm(ell, -m, v), (-1) ** m * np.conj(Ylm(ell, m, v)), atol=1e-14)
        assert np.allclose(Ylm(ell, m, -v), (-1) ** ell * Ylm(ell, m, v), atol=1e-14)
    a, b = v[:20], v[20:]
    cosab = np.sum(a * b, 1) / np.linalg.norm(a, axis=1) / np.linalg.norm(b, axis=1)
    s = sum(np.conj(Ylm(ell, m, a)) * Ylm(ell, m, b) for m in range(-ell, ell + 1))
    assert np.allclose(4 * math.pi / (2 * ell + 1) * s, legendre(ell, cosab), atol=1e-13)


def _one_particle(u_frac, nmesh=16):
    p = np.array([[int(u * 2 ** 32 / nmesh)] for u in u_frac], dtype=np.uint32)
    return p


def test_cic_tsc_single_particle_weights():
    nmesh = 16
    p = _one_particle([3.25, 7.5, 0.75], nmesh)
    m = ms.paint(p, None, nmesh, ms.CIC)
    assert math.isclose(m[3, 7, 0], 0.75 * 0.5 * 0.25)
    assert math.isclose(m[4, 8, 1], 0.25 * 0.5 * 0.75)
    assert math.isclose(m.sum(), 1.0)
    m = ms.paint(p, None, nmesh, ms.TSC)
    # x: u = 3.25 -> i = 3, d = 0.25: (1/2 (1/4)^2, 3/4 - 1/16, 1/2 (3/4)^2)
    wx = {2: 0.5 * 0.25 ** 2, 3: 0.75 - 0.0625, 4: 0.5 * 0.75 ** 2}
    # y: u = 7.5 -> i = 8 (ties go up), d = -0.5: (1/2, 1/2, 0)
    wy = {7: 0.5, 8: 0.5, 9: 0.0}
    # z: u = 0.75 -> i = 1, d = -0.25, node -1 wraps to 15
    wz = {0: 0.5 * 0.75 ** 2, 1: 0.75 - 0.0625, 2: 0.5 * 0.25 ** 2}
    for ix, a in wx.items():
        for iy, b in wy.items():
            for iz, c in wz.items():
                assert math.isclose(m[ix, iy, iz], a * b * c, abs_tol=1e-15)
    mb = ms.paint(p, None, nmesh, ms.TSC, shift=0.5)
    # mesh B: u - 1/2 = 2.75 -> i = 3, d = -0.25
    assert math.isclose(mb[3, 7, 0], 0.6875 * 0.75 * 0.6875)
    assert math.isclose(mb[2, 6, 15], 0.28125 * 0.125 * 0.03125)
    assert math.isclose(mb.sum(), 1.0)


@pytest.mark.parametrize("scheme", [ms.CIC, ms.TSC])
def test_mass_conservation_and_translation(scheme):
    rng = np.random.default_rng(5)
    nmesh = 16
    pos = rng.integers(0, 2 ** 32, size=(3, 300), dtype=np.uint32)
    w = rng.uniform(0.5, 2.0, 300)
    for shift in (0.0, 0.5):
        m = ms.paint(pos, w, nmesh, scheme, shift)
        assert math.isclose(m.sum(), w.sum(), rel_tol=1e-13)
        moved = (pos.astype(np.uint64) + np.array([[1], [2], [3]], dtype=np.uint64) * (2 ** 32 // nmesh)) % 2 ** 32
        m2 = ms.paint(moved.astype(np.uint32), w, nmesh, scheme, shift)
        assert np.allclose(m2, np.roll(m, (1, 2, 3), axis=(0, 1, 2)), atol=1e-13)


def _poisson_sum_1d(kidx, x_cells, nmesh, p, alternate):
    """sum_n s^n W1(k + 2 kN n) exp(-i (k + 2 kN n) x), x in cell units."""
    n = np.arange(-20000, 20001)
    arg = kidx / nmesh + n  # (k + 2 kN n) H / (2 pi)
    terms = np.sinc(arg) ** p * np.exp(-2j * math.pi * arg * x_cells)
    if alternate:
        terms = terms * np.where(n % 2 == 0, 1.0, -1.0)
    return terms.sum()


@pytest.mark.parametrize("scheme", [ms.CIC, ms.TSC])
def test_single_particle_spectrum_exact(scheme):
    """DFT of one painted particle equals the alias sum of the window (Poisson
    summation); interlacing keeps only the even-image terms, which fixes the
    B-mesh shift and the phase sign exp(-i k.(1,1,1) H/2)."""
    nmesh = 16
    ucells = np.array([3.3, 10.71, 6.02])
    p = np.array([[int(u * 2 ** 32 / nmesh)] for u in ucells], dtype=np.uint32)
    uexact = p[:, 0].astype(np.float64) * nmesh / 2 ** 32
    A = ms.paint(p, None, nmesh, scheme)
    B = ms.paint(p, None, nmesh, scheme, shift=0.5)
    DA = np.fft.fftn(A)
    D, _ = ms.deinterlace(A, B)
    nidx = ms.freq_index(nmesh)
    for k in [(1, 2, 3), (0, 5, -4), (7, -7, 2), (-3, 0, 6)]:
        s = [_poisson_sum_1d(k[a], uexact[a], nmesh, scheme, False) for a in range(3)]
        st = [_poisson_sum_1d(k[a], uexact[a], nmesh, scheme, True) for a in range(3)]
        idx = tuple(int(np.where(nidx == k[a])[0][0]) for a in range(3))
        tol = 1e-8 if scheme == ms.CIC else 1e-11  # truncation of the image sum
        assert abs(DA[idx] - s[0] * s[1] * s[2]) < tol
        expect = 0.5 * (s[0] * s[1] * s[2] + st[0] * st[1] * st[2])
        assert abs(D[idx] - expect) < tol


def test_compensation_values():
    W = ms.compensation(8, ms.TSC)
    assert W[0, 0, 0] == 1.0
    assert math.isclose(W[4, 0, 0], (2 / math.pi) ** 3, rel_tol=1e-14)
    assert math.isclose(W[2, 2, 0], (math.sin(math.pi / 4) / (math.pi / 4)) ** 6, rel_tol=1e-14)
