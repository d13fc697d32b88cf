"""Pins of the oracle's bispectrum estimators and analytic shot noise.

* Grid triple sums equal brute-force sums over closed triangles (q1+q2+q3 = 0 on
  the periodic grid) of F_l(q1) F_0(q2) F_0(q3), and N_T equals the brute-force
  triangle count (eq. bi_sco written out), on 8^3 / 10^3.
* sum_k3 N_T = N1 N2 (minus the q3 = 0 pairs when k1 = k2) when the k3 bins
  cover every |q1 + q2|.
* Compression identity: sum over k3 of N_T B_l^raw(k3; k1, k2) = N1 N2 BB_l0l^raw
  (section "A New Compressed TripoSH Bispectrum Estimator"; its l = 0 case is the
  stated BB_000 = B_000).
* N_T against the thin-shell phase-space volume V_T = 8 pi^2 k1 k2 k3 dk^3
  (subsection "A generic form of bispectrum shot noise", appendix on the
  effective integration volume).
* g_l: closed forms of eq. g_first_five, g_2(1) = 1/4, g_4(1) = -1/24, the
  kappa form of eq. g_ell, the limits t -> 0 and t -> infinity, and Lemma 2
  itself by a direct surface average of Y_l^m(khat3).
* Lemma eq. I_l0l: the ring average of Y_l^m(k1hat) around k3hat equals
  L_l(cos theta_13) Y_l^m(k3hat), by direct quadrature.
* Alias sums: c = 1 - 2/3 sin^2 x (CIC), 1 - sin^2 x + 2/15 sin^4 x (TSC),
  and c~ = cos x (5 + cos^2 x)/6 (CIC).
* Poisson catalog: shot-subtracted B_0 and BB_000 are consistent with zero.
* FFT-method pair sums T(i, j) = sum_{q1 in i, q2 in j} Re P(q1 + q2): against
  the direct double loop over the shell modes for a random Hermitian P; for a
  plane wave P(q) = exp(i q.r0), T = Re[I_i(r0) I_j(r0)] with I summed mode by
  mode; for P = |q|^2, T / (N_i N_j) = <q^2>_i + <q^2>_j (the shells are
  symmetric, so the cross term averages to zero).  The FFT-method BB_000 shot
  noise of a Poisson catalog matches the raw estimator (pairs above the lowest
  bin, 10%) and stays within 5% of the thin-shell one.
"""

import math

import numpy as np
import pytest

from oracle import bispectrum as bk
from oracle import mesh as ms
from oracle import shotnoise as sn
from oracle import spectra as sp
from oracle.pipeline import MeshConfig, measure_bk
from oracle.ylm import Ylm, legendre
import synthcat


def _fields(n, seed):
    rng = np.random.default_rng(seed)
    a = np.fft.fftn(rng.normal(size=(n, n, n)))
    b = np.fft.fftn(rng.normal(size=(n, n, n)))
    return a, b


def test_triple_sums_equal_bruteforce_triangles():
    n, L = 10, 100.0
    F0, Fl = _fields(n, 1)
    bins = sp.Bins(0.0, 2 * math.pi / L, 4, L, n)
    shells = bins.shell_index()
    for (i, j, k) in [(1, 1, 1), (1, 2, 2), (2, 3, 3), (0, 1, 1), (1, 2, 3), (3, 3, 3)]:
        Xl = bk.shell_field(Fl, shells, i)
        Xj = bk.shell_field(F0, shells, j)
        Xk = bk.shell_field(F0, shells, k)
        grid = bk.triple_sum(Xl, Xj, Xk) / n ** 3
        brute, count = bk.brute_force_triangles(Fl, F0, F0, bins, i, j, k)
        assert abs(grid - brute.real) < 1e-9 * max(1.0, abs(brute))
        nt = bk.triangle_counts(bins, [(i, j, k)])[0]
        assert nt == count


def test_sum_over_k3_of_triangle_counts():
    n, L = 64, 1000.0  # |q1 + q2| stays below Nyquist
    bins = sp.Bins(0.0, 0.02, 4, L, n)
    ext = sp.Bins(0.0, 0.02, 9, L, n)
    counts = bins.counts()
    for (i, j) in [(0, 1), (2, 3), (3, 3)]:
        cfgs = [(k3, i, j) for k3 in range(ext.nbins)]
        nt = bk.triangle_counts(ext, cfgs)
        # every (q1, q2) pair closes with some q3, except q2 = -q1 (q3 = 0 is in no bin)
        assert int(nt.sum()) == int(counts[i] * counts[j]) - (int(counts[i]) if i == j else 0)


@pytest.mark.parametrize("ell", [0, 2])
def test_compression_identity(ell):
    n, L = 24, 600.0
    F0, Fl = _fields(n, 2 + ell)
    dk = 2 * math.pi / L * 1.5
    bins = sp.Bins(0.0, dk, 4, L, n)
    ext = sp.Bins(0.0, dk, 8, L, n)
    I33 = 2.5
    counts = bins.counts()
    pairs = bk.triposh_pairs(4)
    Fl_use = F0 if ell == 0 else Fl
    tri = bk.triposh_raw(F0, Fl_use, ell, bins, I33, pairs)
    for t, (i, j) in enumerate(pairs):
        cfgs = [(k3, i, j) for k3 in range(ext.nbins)]
        nt = bk.triangle_counts(ext, cfgs)
        keep = [c for c, m in zip(cfgs, nt) if m > 0]
        ntk = nt[nt > 0]
        sc = bk.scoccimarro_raw(F0, Fl_use, ell, ext, I33, keep, ntk)
        lhs = float(np.sum(ntk * sc))
        rhs = counts[i] * counts[j] * tri[t]
        assert abs(lhs - rhs) < 1e-9 * max(1.0, abs(rhs))


def test_triangle_counts_vs_phase_space_volume():
    n, L = 96, 1000.0  # shells well inside Nyquist, so no wrapped triangles
    dk = 0.0125
    bins = sp.Bins(0.0, dk, 14, L, n)
    kf = 2 * math.pi / L
    c = bins.centres()
    cfgs = [(10, 11, 12), (11, 11, 11), (12, 13, 13), (9, 12, 13), (8, 10, 11)]
    nt = bk.triangle_counts(bins, cfgs)
    for (i, j, k), m in zip(cfgs, nt):
        vt = 8 * math.pi ** 2 * c[i] * c[j] * c[k] * dk ** 3 / kf ** 6
        assert abs(m / vt - 1.0) < 0.05


def test_configuration_counts():
    assert len(bk.scoccimarro_configs(20, 0)) == 825
    assert len(bk.scoccimarro_configs(20, 2)) == 2155
    assert len(bk.triposh_pairs(20)) == 210


@pytest.mark.parametrize("ell", [0, 1, 2, 3, 4])
def test_g_ell_closed_forms(ell):
    for t in [0.1, 0.3, 0.5, 0.8, 0.95, 1.0, 1.05, 1.5, 3.0, 10.0, 79.0]:
        assert abs(sn.g_ell(ell, t) - sn.g_ell_closed(ell, t)) < 5e-10
        assert abs(sn.g_ell(ell, t) - sn.g_ell_kappa(ell, t)) < 1e-6


def test_g_ell_special_values_and_limits():
    assert math.isclose(sn.g_ell(2, 1.0), 0.25, abs_tol=1e-14)
    assert math.isclose(sn.g_ell(4, 1.0), -1.0 / 24.0, abs_tol=1e-14)
    for ell in (2, 4, 6):
        assert abs(sn.g_ell(ell, 500.0) - 1.0) < 1e-3
        assert abs(sn.g_ell(ell, 1e-3)) < 1e-3
    assert sn.g_ell(0, 0.37) == pytest.approx(1.0, abs=1e-14)


def _sphere_quadrature(npts_theta=200, npts_phi=400):
    x, w = np.polynomial.legendre.leggauss(npts_theta)
    th = np.arccos(x)
    ph = np.arange(npts_phi) * 2 * math.pi / npts_phi
    T, P = np.meshgrid(th, ph, indexing="ij")
    vec = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1)
    wt = (w[:, None] * np.ones_like(P)) * (2 * math.pi / npts_phi)
    return vec, wt


@pytest.mark.parametrize("ell", [1, 2, 4])
def test_lemma2_surface_average(ell):
    """<Y_l^m(khat3)>_{k2hat} = g_l(t) Y_l^m(k1hat), k3 = k1 + k2, t = k1/k2."""
    vec, wt = _sphere_quadrature()
    k1 = np.array([0.3, -0.4, 0.5])
    for t in (0.4, 1.7):
        k2mag = np.linalg.norm(k1) / t
        k3 = k1 + k2mag * vec
        for m in (0, 1, ell):
            avg = np.sum(wt * Ylm(ell, m, k3)) / (4 * math.pi)
            assert abs(avg - sn.g_ell(ell, t) * Ylm(ell, m, k1[None, :])[0]) < 2e-4


@pytest.mark.parametrize("ell", [1, 2, 3, 4])
def test_lemma_ring_average(ell):
    """eq. I_l0l: ring average of Y_l^m(k1hat) about k3hat at fixed angle."""
    k3 = np.array([0.2, 0.7, -0.3])
    k3 /= np.linalg.norm(k3)
    u = np.cross(k3, [1.0, 0.0, 0.0])
    u /= np.linalg.norm(u)
    v = np.cross(k3, u)
    cth = 0.37
    sth = math.sqrt(1 - cth * cth)
    g = np.arange(720) * 2 * math.pi / 720
    k1 = cth * k3[None, :] + sth * (np.cos(g)[:, None] * u + np.sin(g)[:, None] * v)
    for m in range(-ell, ell + 1):
        avg = np.mean(Ylm(ell, m, k1))
        assert abs(avg - legendre(ell, cth) * Ylm(ell, m, k3[None, :])[0]) < 1e-12


def test_alias_sum_closed_forms():
    for n in (16, 64):
        x = math.pi * ms.freq_index(n) / n
        s2 = np.sin(x) ** 2
        c, ct = sn.alias_tables(n, ms.CIC)
        assert np.allclose(c, 1 - 2.0 / 3.0 * s2, atol=1e-7)
        assert np.allclose(ct, np.cos(x) * (5 + np.cos(x) ** 2) / 6, atol=1e-7)
        c, ct = sn.alias_tables(n, ms.TSC)
        assert np.allclose(c, 1 - s2 + 2.0 / 15.0 * s2 * s2, atol=1e-10)


def test_poisson_catalog_bispectrum_matches_shot_model():
    """Unclustered galaxies: raw B_0 and BB_000 average to the analytic shot noise,
    and B_0 - N^(0) is consistent with zero (z-scores from the Gaussian variance
    s V P^3 / N_T with P = N0)."""
    L, n = 1000.0, 64  # k_max = 0.1 = k_N / 2
    for ng, seed, tol_b, tol_bb in ((3000, 41, 0.05, 0.2), (20000, 45, 0.05, 0.2)):
        g = synthcat.poisson_catalog(ng, seed=seed)
        r = synthcat.random_catalog(10 * ng, seed=seed + 1)
        cfg = MeshConfig(L, n, ms.TSC, True, synthcat.observer_position())
        out = measure_bk(g, None, r, None, cfg, 0.025, 4, ells=(0,), scoccimarro=(0,),
                         triposh=(0,))
        N0 = out["norms"].N0
        nt, cf = out["B0_ntri"], out["B0_configs"]
        sym = np.array([6 if i == j == k else (2 if (i == j or j == k) else 1) for i, j, k in cf])
        z = out["B0"] / np.sqrt(sym * L ** 3 * N0 ** 3 / nt)
        assert np.all(np.abs(z) < 4.0)
        w = nt / sym
        ratio = np.sum(w * out["B0_raw"]) / np.sum(w * out["B0_shot"])
        assert abs(ratio - 1.0) < tol_b
        ratio_bb = np.sum(out["BB000_raw"]) / np.sum(out["BB000_shot"])
        assert abs(ratio_bb - 1.0) < tol_bb


def _shell_modes(bins, b):
    shells = bins.shell_index()
    n = bins.nmesh
    idx = np.argwhere(shells == b)
    return np.where(idx > n // 2, idx - n, idx)  # signed wave indices


def _pin_bins():
    n, box = 16, 1000.0
    kf = 2 * math.pi / box
    return sp.Bins(0.0, 1.3 * kf, 3, box, n)  # |q1 + q2| components <= 6 < N / 2


def test_exact_pair_sums_bruteforce():
    bins = _pin_bins()
    n = bins.nmesh
    rng = np.random.default_rng(77)
    P = np.fft.fftn(rng.normal(size=(n, n, n)))  # Hermitian
    pairs = bk.triposh_pairs(bins.nbins)
    T = sn.exact_pair_sums(P, bins, pairs)
    for t, (i, j) in enumerate(pairs):
        qi, qj = _shell_modes(bins, i), _shell_modes(bins, j)
        s = (qi[:, None, :] + qj[None, :, :]) % n
        ref = float(np.sum(np.real(P[s[..., 0], s[..., 1], s[..., 2]])))
        assert abs(T[t] - ref) <= 1e-9 * max(1.0, np.max(np.abs(P)) * len(qi) * len(qj)), (i, j)


def test_exact_pair_sums_plane_wave_and_quadratic():
    bins = _pin_bins()
    n = bins.nmesh
    pairs = bk.triposh_pairs(bins.nbins)
    nx, ny, nz = ms.wave_indices(n)
    r0 = np.array([1.0, 3.0, -2.0])
    ph = 2 * math.pi * (nx * r0[0] + ny * r0[1] + nz * r0[2]) / n
    P = np.exp(1j * ph)
    P = np.where(ms.nyquist_mask(n), 0.0, P)
    T = sn.exact_pair_sums(P, bins, pairs)
    Ir = {}
    for b in range(bins.nbins):
        q = _shell_modes(bins, b)
        Ir[b] = np.sum(np.exp(2j * math.pi * (q @ r0) / n))
    for t, (i, j) in enumerate(pairs):
        assert abs(T[t] - np.real(Ir[i] * Ir[j])) < 1e-8 * bins.counts()[i] * bins.counts()[j]
    q2 = (nx * nx + ny * ny + nz * nz).astype(np.float64) * np.ones((n, n, n))
    T = sn.exact_pair_sums(q2, bins, pairs)
    cnt = bins.counts()
    mean_q2 = {b: float(np.mean(np.sum(_shell_modes(bins, b) ** 2, axis=1))) for b in range(bins.nbins)}
    for t, (i, j) in enumerate(pairs):
        assert math.isclose(T[t] / (cnt[i] * cnt[j]), mean_q2[i] + mean_q2[j], rel_tol=1e-11)


def test_poisson_catalog_fft_shot_noise():
    L, n = 1000.0, 64
    g = synthcat.poisson_catalog(20000, seed=45)
    r = synthcat.random_catalog(200000, seed=46)
    cfg = MeshConfig(L, n, ms.TSC, True, synthcat.observer_position())
    out = measure_bk(g, None, r, None, cfg, 0.025, 4, ells=(0,), scoccimarro=(), triposh=(0,),
                     fft_noise=True)
    # the (0, 0) pair has few modes and dominates the scatter; the rest average out
    ratio = np.sum(out["BB000_raw"][1:]) / np.sum(out["BB000_shot_fft"][1:])
    assert abs(ratio - 1.0) < 0.1
    rel = np.abs(out["BB000_shot_fft"] / out["BB000_shot"] - 1.0)
    assert np.max(rel) < 0.05


@pytest.mark.parametrize("ell", [0, 2])
def test_self_term_modes(ell):
    """Per-mode s_l(q): its shell means are s_l(k); for l = 0 it is Sbar C / W^2,
    and for l = 2 with a single particle on the z axis seen from the origin it is
    Sbar L_2(qhat_z) C / W^2 (addition theorem)."""
    from oracle.catalog import catalog_norms
    n, box = 16, 1000.0
    bins = sp.Bins(0.0, 2 * math.pi / box * 1.3, 3, box, n)
    C = sn.c_shot(n, ms.TSC, True)
    W = ms.compensation(n, ms.TSC)
    g, gw, r, rw = synthcat.tiny_catalog(50, 400, seed=5)
    obs = synthcat.observer_position()
    nm = catalog_norms(g, gw, r, rw, box, obs, (0, 2))
    s = sn.self_term_modes(ell, nm.Sbar_lm, n, box, W, C)
    assert s[0, 0, 0] == 0.0
    np.testing.assert_allclose(bins.shell_mean(s), sn.self_term(ell, nm.Sbar_lm, bins, W, C), rtol=1e-12)
    kv = sp.kvectors(n, box)
    kn = np.linalg.norm(kv, axis=-1)
    kn[0, 0, 0] = 1.0
    if ell == 0:
        ref = nm.Sbar * C / (W * W)
    else:
        # one particle at (0, 0, z) relative to the observer: Sbar_2^m vanishes for
        # m != 0 and sum_m y_2^m(q) y_2^m*(zhat) = L_2(q_z / |q|)
        one = {(2, m): (nm.Sbar if m == 0 else 0.0) for m in range(-2, 3)}
        s = sn.self_term_modes(2, one, n, box, W, C)
        ref = nm.Sbar * legendre(2, kv[..., 2] / kn) * C / (W * W)
    ref[0, 0, 0] = 0.0
    np.testing.assert_allclose(s, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))
