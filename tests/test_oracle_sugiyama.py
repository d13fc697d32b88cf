"""Pins of the oracle's Sugiyama bispectrum multipoles and their shot noise.

* Wigner 3j symbols: closed forms ((l l 0; m -m 0) = (-1)^(l-m)/sqrt(2l+1),
  (1 1 2; 0 0 0) = sqrt(2/15), (2 2 2; 0 0 0) = -sqrt(2/35)), orthogonality
  and the column-exchange symmetry.
* Racah associated Legendre: Lr_l^0 = L_l, Lr_l^n at mu = 1 vanishes for n != 0.
* Brute force: the x-space estimator equals the direct sum over mode pairs
  q1 in shell i, q2 in shell j of y*(q1hat) F_0(q1) y*(q2hat) F_0(q2)
  G_L^M(-q1 - q2) (eq. sugi_estimator written out), on a 12^3 mesh.
* B_000 equals the compressed estimator BB_000 (the same three fields).
* The sum over (m1, m2, M) is real, and the paired selection with eta Re[...]
  (eq. sym_sugi and the boxed final form) reproduces it.
* The symmetries of eq. sugi_F_and_G: F_l^-m = (-1)^(l+m) F_l^m*,
  G_L^-M = (-1)^M G_L^M*.
* FFT-method i = j != k term: real, equal to the direct sum over mode pairs of
  y*(q1hat) y*(q2hat) P_L^M(-q1 - q2), and for (0, 0, 0) the shot noise equals
  the compressed estimator's FFT-method noise.
* Shot noise: for (0, 0, 0) every term equals the compressed estimator's
  l = 0 noise; q_l0l = L_l(mu_13) (l 0 l; 0 0 0) (one n term); for (2, 2, 0)
  the i != j = k and i = k != j terms vanish.
"""

import math

import numpy as np
import pytest

from oracle import bispectrum as bk
from oracle import mesh as ms
from oracle import shotnoise as sn
from oracle import spectra as sp
from oracle import sugiyama as sg
from oracle.catalog import catalog_norms
from oracle.pipeline import MeshConfig, fkp_spectra, measure_bk, measure_sugiyama, noise_terms
from oracle.ylm import legendre, ylm_racah
import synthcat


def test_wigner3j_closed_forms_and_orthogonality():
    for l in range(0, 5):
        for m in range(-l, l + 1):
            assert math.isclose(sg.wigner3j(l, l, 0, m, -m, 0), (-1) ** (l - m) / math.sqrt(2 * l + 1),
                                rel_tol=1e-13)
    assert math.isclose(sg.wigner3j(1, 1, 2, 0, 0, 0), math.sqrt(2 / 15), rel_tol=1e-13)
    assert math.isclose(sg.wigner3j(2, 2, 2, 0, 0, 0), -math.sqrt(2 / 35), rel_tol=1e-13)
    assert sg.wigner3j(1, 1, 1, 0, 0, 0) == 0.0  # odd sum of l with m = 0
    for (a, b, c) in [(2, 2, 2), (2, 0, 2), (4, 2, 2), (2, 2, 4), (4, 4, 0)]:
        for c2 in range(abs(a - b), a + b + 1):
            for M in range(-min(c, c2), min(c, c2) + 1):
                t = sum(sg.wigner3j(a, b, c, m1, -m1 - M, M) * sg.wigner3j(a, b, c2, m1, -m1 - M, M)
                        for m1 in range(-a, a + 1))
                assert abs(t - (1.0 / (2 * c + 1) if c2 == c else 0.0)) < 1e-13
        for m1 in range(-a, a + 1):
            for m2 in range(-b, b + 1):
                M = -m1 - m2
                s = (-1) ** (a + b + c)
                assert math.isclose(sg.wigner3j(b, a, c, m2, m1, M), s * sg.wigner3j(a, b, c, m1, m2, M),
                                    abs_tol=1e-15)


def test_racah_associated_legendre():
    for l in range(5):
        for mu in (-0.7, 0.1, 0.9):
            assert math.isclose(sg.racah_assoc_legendre(l, 0, mu), legendre(l, mu), abs_tol=1e-14)
        for n in range(1, l + 1):
            assert abs(sg.racah_assoc_legendre(l, n, 1.0)) < 1e-14
    # y_2^1(theta, 0) = -sqrt(3/2) sin cos (Racah normalisation)
    mu = 0.3
    assert math.isclose(sg.racah_assoc_legendre(2, 1, mu), -math.sqrt(1.5) * mu * math.sqrt(1 - mu * mu),
                        rel_tol=1e-13)


def _tiny_setup(n=12):
    g, gw, r, rw = synthcat.tiny_catalog(60, 300, seed=21)
    obs = synthcat.observer_position()
    cfg = MeshConfig(1000.0, n, ms.TSC, True, obs)
    norms, W, F, _ = fkp_spectra(g, None, r, None, cfg, (0,))
    delta, _ = ms.paint_fkp(g, None, r, None, norms.alpha, n, ms.TSC, True, noise=False)
    _, dint = ms.deinterlace(delta[0], delta[1])
    bins = sp.Bins(0.0, 2 * math.pi / 1000.0 * 1.3, 2, 1000.0, n)
    return cfg, norms, W, F[0], dint, bins, obs


def _signed(idx, n):
    return np.where(idx > n // 2, idx - n, idx)


@pytest.mark.parametrize("l1,l2,L", [(0, 0, 0), (2, 0, 2), (2, 2, 0), (2, 2, 2), (1, 1, 2), (3, 1, 2)])
def test_sugiyama_bruteforce_mode_sums(l1, l2, L):
    cfg, norms, W, F0, dint, bins, obs = _tiny_setup()
    n = cfg.nmesh
    raw = sg.sugiyama_raw(F0, dint, W, l1, l2, L, bins, norms.I33, cfg.boxsize, obs)
    shells = bins.shell_index()
    kf = 2 * math.pi / cfg.boxsize
    H = sg.wigner3j(l1, l2, L, 0, 0, 0)
    Nn = (2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1)
    rvec = sp.line_of_sight(n, cfg.boxsize, obs)
    nyq = ms.nyquist_mask(n)
    for i in range(bins.nbins):
        for j in range(bins.nbins):
            qi = np.argwhere(shells == i)
            qj = np.argwhere(shells == j)
            tot = 0.0 + 0.0j
            for m1, m2, M, w in sg.sub_configs(l1, l2, L):
                dn = np.fft.fftn(dint * np.conj(ylm_racah(L, M, rvec)))
                g = np.where(nyq, 0.0, dn / W)
                g[0, 0, 0] = 0.0
                a = np.conj(ylm_racah(l1, m1, _signed(qi, n) * kf)) * F0[tuple(qi.T)]
                b = np.conj(ylm_racah(l2, m2, _signed(qj, n) * kf)) * F0[tuple(qj.T)]
                s3 = (-(qi[:, None, :] + qj[None, :, :])) % n
                tot += w * np.sum(a[:, None] * b[None, :] * g[s3[..., 0], s3[..., 1], s3[..., 2]])
            ref = H * Nn / norms.I33 * tot / (len(qi) * len(qj))
            assert abs(ref.imag) <= 1e-10 * max(abs(ref.real), 1e-300) + 1e-300
            assert math.isclose(raw[i, j], ref.real, rel_tol=1e-10, abs_tol=1e-12 * np.max(np.abs(raw))), (i, j)


def test_b000_equals_compressed_estimator():
    cfg, norms, W, F0, dint, bins, obs = _tiny_setup(16)
    raw = sg.sugiyama_raw(F0, dint, W, 0, 0, 0, bins, norms.I33, cfg.boxsize, obs)
    pairs = bk.triposh_pairs(bins.nbins)
    comp = bk.triposh_raw(F0, F0, 0, bins, norms.I33, pairs)
    for t, (i, j) in enumerate(pairs):
        assert math.isclose(raw[i, j], comp[t], rel_tol=1e-11)
        assert math.isclose(raw[j, i], comp[t], rel_tol=1e-11)


@pytest.mark.parametrize("l1,l2,L", [(2, 0, 2), (2, 2, 0), (2, 2, 2), (4, 2, 2), (1, 1, 0), (1, 1, 2)])
def test_sum_is_real_and_pairing(l1, l2, L):
    cfg, norms, W, F0, dint, bins, obs = _tiny_setup(16)
    re, im = sg.sugiyama_raw(F0, dint, W, l1, l2, L, bins, norms.I33, cfg.boxsize, obs, return_imag=True)
    assert np.max(np.abs(im)) < 1e-10 * np.max(np.abs(re))
    # paired selection: eta Re over one of each (m1, m2, M), (-m1, -m2, -M) pair
    n = cfg.nmesh
    H = sg.wigner3j(l1, l2, L, 0, 0, 0)
    Nn = (2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1)
    acc = np.zeros((bins.nbins, bins.nbins))
    for m1, m2, M, w in sg.sub_configs(l1, l2, L, paired=True):
        A = sg.shell_fields_lm(F0, bins, l1, m1)
        B = sg.shell_fields_lm(F0, bins, l2, m2)
        G = sg.los_field(dint, W, L, M, cfg.boxsize, obs)
        for i in range(bins.nbins):
            for j in range(bins.nbins):
                acc[i, j] += w * np.real(np.sum(A[i] * B[j] * G))
    paired = H * Nn / norms.I33 * acc / float(n) ** 3
    np.testing.assert_allclose(paired, re, rtol=1e-10, atol=1e-12 * np.max(np.abs(re)))


def test_field_conjugation_symmetries():
    cfg, norms, W, F0, dint, bins, obs = _tiny_setup(16)
    for l in (1, 2, 3, 4):
        for m in range(1, l + 1):
            Fp = sg.shell_fields_lm(F0, bins, l, m)
            Fm = sg.shell_fields_lm(F0, bins, l, -m)
            scale = max(np.max(np.abs(f)) for f in Fp + sg.shell_fields_lm(F0, bins, l, 0))
            for b in range(bins.nbins):
                np.testing.assert_allclose(Fm[b], (-1) ** (l + m) * np.conj(Fp[b]), rtol=0, atol=1e-10 * scale)
    for M in range(1, 3):
        Gp = sg.los_field(dint, W, 2, M, cfg.boxsize, obs)
        Gm = sg.los_field(dint, W, 2, -M, cfg.boxsize, obs)
        np.testing.assert_allclose(Gm, (-1) ** M * np.conj(Gp), atol=1e-10 * np.max(np.abs(Gp)))


def test_shot_noise_special_cases():
    nb = 4
    rng = np.random.default_rng(3)
    Q = rng.normal(size=2 * nb - 1)
    H = rng.normal(size=2 * nb - 1)
    cnt = rng.integers(10, 100, size=2 * nb - 1).astype(float)
    cen = (np.arange(2 * nb - 1) + 0.5) * 0.01
    s000 = sg.sugiyama_shot(0, 0, 0, nb, Q, H, cnt, cen, 2.0, 5.0)
    comp = sn.triposh_shot(0, bk.triposh_pairs(nb), Q, H, cnt, cen, 2.0, 5.0)
    for t, (i, j) in enumerate(bk.triposh_pairs(nb)):
        assert math.isclose(s000[i, j], comp[t], rel_tol=1e-13)
    for l in (2, 4):
        for k3 in (0.012, 0.02, 0.031):
            k1, k2 = 0.015, 0.025
            mu13 = (k2 * k2 - k1 * k1 - k3 * k3) / (2 * k1 * k3)
            assert math.isclose(sg.q_factor(l, 0, l, k1, k2, k3),
                                legendre(l, mu13) * sg.wigner3j(l, 0, l, 0, 0, 0), rel_tol=1e-12)
    s220 = sg.sugiyama_shot(2, 2, 0, nb, Q, np.zeros_like(H) + 7.0, cnt, cen, 2.0, 5.0)
    s220h = sg.sugiyama_shot(2, 2, 0, nb, Q, H, cnt, cen, 2.0, 5.0)
    np.testing.assert_allclose(s220, s220h, rtol=1e-14)  # no H_L term for (2, 2, 0)


def test_measure_sugiyama_runs_and_b000_shot_matches_compressed():
    g = synthcat.lognormal_catalog(8000, 1000.0, 5)
    r = synthcat.random_catalog(40000, 6)
    cfg = MeshConfig(1000.0, 32, ms.TSC, True, synthcat.observer_position())
    out = measure_sugiyama(g, None, r, None, cfg, 0.012, 3, 0, 0, 0)
    ref = measure_bk(g, None, r, None, cfg, 0.012, 3, ells=(0,), scoccimarro=(), triposh=(0,))
    for t, (i, j) in enumerate(bk.triposh_pairs(3)):
        assert math.isclose(out["raw"][i, j], ref["BB000_raw"][t], rel_tol=1e-11)
        assert math.isclose(out["shot"][i, j], ref["BB000_shot"][t], rel_tol=1e-11)


def _noise_setup(n=12, nb=2):
    g, gw, r, rw = synthcat.tiny_catalog(60, 300, seed=23)
    obs = synthcat.observer_position()
    cfg = MeshConfig(1000.0, n, ms.TSC, True, obs)
    norms, W, F, FN = fkp_spectra(g, None, r, None, cfg, (0, 2), noise_ells=(2,))
    delta, _ = ms.paint_fkp(g, None, r, None, norms.alpha, n, ms.TSC, True, noise=False)
    _, dint = ms.deinterlace(delta[0], delta[1])
    bins = sp.Bins(0.0, 2 * math.pi / 1000.0 * 1.3, nb, 1000.0, n)
    C = sn.c_shot(n, ms.TSC, True)
    return cfg, norms, W, F, FN, dint, bins, obs, C


@pytest.mark.parametrize("l1,l2,L", [(2, 0, 2), (2, 2, 0), (0, 2, 2)])
def test_fft_term_bruteforce_and_real(l1, l2, L):
    cfg, norms, W, F, FN, dint, bins, obs, C = _noise_setup()
    n = cfg.nmesh
    re, im = sg.sugiyama_fft_term(dint, W, FN[0], C, norms.Sbar_lm, l1, l2, L, bins, norms.I33, cfg.boxsize, obs,
                                  return_imag=True)
    assert np.max(np.abs(im)) < 1e-10 * np.max(np.abs(re))
    shells = bins.shell_index()
    kf = 2 * math.pi / cfg.boxsize
    H = sg.wigner3j(l1, l2, L, 0, 0, 0)
    Nn = (2 * l1 + 1) * (2 * l2 + 1) * (2 * L + 1)
    rvec = sp.line_of_sight(n, cfg.boxsize, obs)
    nyq = ms.nyquist_mask(n)
    for i in range(bins.nbins):
        for j in range(bins.nbins):
            qi, qj = np.argwhere(shells == i), np.argwhere(shells == j)
            tot = 0.0 + 0.0j
            for m1, m2, M, w in sg.sub_configs(l1, l2, L):
                dn = np.fft.fftn(dint * np.conj(ylm_racah(L, M, rvec)))
                P = dn / W * np.conj(FN[0]) - norms.Sbar_lm[(L, M)] * C / (W * W)
                P = np.where(nyq, 0.0, P)
                P[0, 0, 0] = 0.0
                a = np.conj(ylm_racah(l1, m1, _signed(qi, n) * kf))
                b = np.conj(ylm_racah(l2, m2, _signed(qj, n) * kf))
                s3 = (-(qi[:, None, :] + qj[None, :, :])) % n
                tot += w * np.sum(a[:, None] * b[None, :] * P[s3[..., 0], s3[..., 1], s3[..., 2]])
            ref = H * Nn / norms.I33 * tot / (len(qi) * len(qj))
            assert math.isclose(re[i, j], ref.real, rel_tol=1e-10, abs_tol=1e-12 * np.max(np.abs(re))), (i, j)


def test_fft_term_000_equals_compressed_fft_noise():
    g = synthcat.lognormal_catalog(8000, 1000.0, 15)
    r = synthcat.random_catalog(40000, 16)
    cfg = MeshConfig(1000.0, 32, ms.TSC, True, synthcat.observer_position())
    out = measure_sugiyama(g, None, r, None, cfg, 0.012, 3, 0, 0, 0, fft_noise=True)
    ref = measure_bk(g, None, r, None, cfg, 0.012, 3, ells=(0,), scoccimarro=(), triposh=(0,), fft_noise=True)
    for t, (i, j) in enumerate(bk.triposh_pairs(3)):
        assert math.isclose(out["shot_fft"][i, j], ref["BB000_shot_fft"][t], rel_tol=1e-11)
        assert math.isclose(out["shot_fft"][j, i], ref["BB000_shot_fft"][t], rel_tol=1e-11)


def _golden_counts():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "special_values.txt")
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, value = line.split()[:2]
            vals[name] = value
    return vals


@pytest.mark.parametrize("lls", ["112", "222", "224"])
def test_subconfiguration_counts_match_the_paper(lls):
    """The appendix on the real decomposition prints the number of non-zero
    sub-configurations of S_112, S_222, S_224: real form 11, 25, 37; complex
    form with the pairing 5, 10, 13."""
    g = _golden_counts()
    l1, l2, L = (int(c) for c in lls)
    A = sg.tripolar_real_coeffs(l1, l2, L)
    assert int(np.sum(np.abs(A) > 1e-12)) == int(g[f"real_nonzero_{lls}"])
    assert len(sg.sub_configs(l1, l2, L, paired=True)) == int(g[f"complex_paired_{lls}"])


@pytest.mark.parametrize("l1,l2,L", [(1, 1, 2), (2, 2, 2), (2, 2, 4), (2, 0, 2), (3, 1, 2)])
def test_real_decomposition_reproduces_the_basis(l1, l2, L):
    """sum A x x x equals 1/H sum 3j y y y at random directions, and A is real."""
    A = sg.tripolar_real_coeffs(l1, l2, L)
    assert np.max(np.abs(A.imag)) < 1e-13
    rng = np.random.default_rng(l1 * 100 + l2 * 10 + L)
    H = sg.wigner3j(l1, l2, L, 0, 0, 0)

    def xvec(ell, v):
        y = np.array([ylm_racah(ell, m, v) for m in range(-ell, ell + 1)])
        return sg.real_harmonic_matrix(ell) @ y  # Racah-normalised real harmonics

    for _ in range(5):
        k1, k2, nn = (rng.normal(size=3) for _ in range(3))
        ref = sum(sg.wigner3j(l1, l2, L, m1, m2, -m1 - m2) * ylm_racah(l1, m1, k1) * ylm_racah(l2, m2, k2)
                  * ylm_racah(L, -m1 - m2, nn)
                  for m1 in range(-l1, l1 + 1) for m2 in range(-l2, l2 + 1) if abs(m1 + m2) <= L) / H
        x1, x2, x3 = xvec(l1, k1), xvec(l2, k2), xvec(L, nn)
        assert np.max(np.abs(x1.imag)) < 1e-12
        got = np.einsum("abc,a,b,c->", A, x1, x2, x3)
        assert abs(got - ref) < 1e-12 * max(1.0, abs(ref))


def test_analytic_shot_noise_tracks_the_fft_method_for_b202():
    """The thin-shell i = j != k term with q_202 = L_2(mu_13) (2 0 2; 0 0 0) and
    the H_2 term agree with the FFT method (no thin-shell step) to within 1% of
    the largest value on a Poisson catalog, 64^3 and 9 bins of 0.01 (the
    section validating the analytic noise finds the same for B_202)."""
    g = synthcat.poisson_catalog(100000, seed=47)
    r = synthcat.random_catalog(1000000, seed=48)
    cfg = MeshConfig(1000.0, 64, ms.TSC, True, synthcat.observer_position())
    out = measure_sugiyama(g, None, r, None, cfg, 0.01, 9, 2, 0, 2, fft_noise=True)
    a, f = out["shot"], out["shot_fft"]
    assert np.max(np.abs(a - f)) < 0.01 * np.max(np.abs(f))


@pytest.mark.parametrize("l1,l2,L", [(1, 1, 0), (1, 1, 2), (2, 2, 0), (2, 2, 2), (3, 1, 2), (1, 2, 3),
                                     (4, 2, 2), (2, 0, 2), (3, 3, 4), (4, 4, 4)])
def test_q_factor_is_the_rotation_invariant_of_the_closed_triangle(l1, l2, L):
    """q_l1l2L of eq. q_ells is written in the frame where k3 is the polar axis
    and k1, k2 lie in the x-z plane.  It must equal the frame-free invariant
    sum over (m1, m2, M) of (l1 l2 L; m1 m2 M) y_l1^m1(k1hat) y_l2^m2(k2hat)
    y_L^M(k3hat) of a closed triangle k1 + k2 + k3 = 0 in any orientation,
    with y_l^m = sqrt(4 pi / (2l + 1)) Y_l^m from scipy.  A dropped (-1)^n, a
    swapped cosine or a wrong 3j argument fails it."""
    from scipy.special import sph_harm_y

    def y(l, m, v):
        v = v / np.linalg.norm(v)
        theta = math.acos(max(-1.0, min(1.0, float(v[2]))))
        return math.sqrt(4 * math.pi / (2 * l + 1)) * complex(sph_harm_y(l, m, theta, math.atan2(v[1], v[0])))

    rng = np.random.default_rng(5)
    for k1, k2, k3 in ((0.015, 0.025, 0.012), (0.015, 0.025, 0.02), (0.03, 0.03, 0.031), (0.02, 0.05, 0.04)):
        mu13 = (k2 * k2 - k1 * k1 - k3 * k3) / (2 * k1 * k3)
        v3 = np.array([0.0, 0.0, k3])
        v1 = k1 * np.array([math.sqrt(1 - mu13 * mu13), 0.0, mu13])
        v2 = -(v1 + v3)
        assert math.isclose(np.linalg.norm(v2), k2, rel_tol=1e-12)
        q = sg.q_factor(l1, l2, L, k1, k2, k3)
        for _ in range(3):
            rot, upper = np.linalg.qr(rng.normal(size=(3, 3)))
            rot = rot * np.sign(np.diag(upper))
            if np.linalg.det(rot) < 0:
                rot[:, 0] *= -1
            a1, a2, a3 = rot @ v1, rot @ v2, rot @ v3
            inv = 0j
            for m1 in range(-l1, l1 + 1):
                for m2 in range(-l2, l2 + 1):
                    M = -m1 - m2
                    if abs(M) <= L:
                        w = sg.wigner3j(l1, l2, L, m1, m2, M)
                        if w:
                            inv += w * y(l1, m1, a1) * y(l2, m2, a2) * y(L, M, a3)
            assert abs(inv.imag) < 1e-12
            assert abs(inv.real - q) < 1e-11 * max(abs(q), 1e-3)


@pytest.mark.parametrize("l1,l2,L,tol", [(0, 0, 0, 0.015), (4, 0, 4, 0.01)])
def test_analytic_shot_noise_tracks_the_fft_method_beyond_the_lowest_bins(l1, l2, L, tol):
    """As for B_202 above, for B_000 and B_404 on the same Poisson catalog, over
    the bins i, j >= 2: in the two lowest bins (shells of 1 to 7 modes on this
    64^3 grid) the thin-shell step of the analytic i = j != k term is off by up
    to 21% (B_000, bin pair (0, 0)) of the largest value."""
    g = synthcat.poisson_catalog(100000, seed=47)
    r = synthcat.random_catalog(1000000, seed=48)
    cfg = MeshConfig(1000.0, 64, ms.TSC, True, synthcat.observer_position())
    out = measure_sugiyama(g, None, r, None, cfg, 0.01, 9, l1, l2, L, fft_noise=True)
    a, f = out["shot"], out["shot_fft"]
    assert np.max(np.abs(a - f)[2:, 2:]) < tol * np.max(np.abs(f))
