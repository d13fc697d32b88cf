"""Pins of the oracle's Yamamoto multipoles and the modified high-order multipoles.

* F_l from the Y_lm sum equals a brute-force Legendre-kernel DFT over the mesh
  nodes (eq. F_ell written out), on 8^3.
* Conjugation identity of eq. key1 and the parity of F_l (appendix on proofs).
* The inversion-free G_l route of eqs. new_F_ell / pk_final gives the same P_l
  below Nyquist; eq. F_and_new_G holds away from Nyquist planes.
* eq. legendre and eq. Plnew coefficients (golden files) against Legendre
  polynomials; with a global line of sight P_lb equals P_l exactly.
* Table 1 counts (golden file) from the closed forms and by enumeration.
* N_22 = 9 N0/5, N_44 = 17 N0/9 by angular quadrature.
* Kaiser: a fixed-amplitude Gaussian mesh gives the exact discrete expectation
  of (2l+1) L_l(mu) P(k)(b + f mu^2)^2, whose ratios approach the Kaiser values.
* Catalog norms: closed forms for unit weights.
* Poisson: unclustered galaxies give a shot-subtracted P_0 consistent with zero.
* Odd multipoles (imaginary part of eq. pk_final): F_1, F_3 equal the brute-
  force Legendre-kernel DFT; the G_l route gives the same Im shell means; with
  a global line of sight they vanish; F_l is anti-Hermitian for odd l.
* Cross multipoles of two tracers: a tracer crossed with itself gives its auto
  multipoles without shot noise; the l = 0 cross is symmetric in A, B.
"""

import math
from fractions import Fraction

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle import mesh as ms
from oracle import spectra as sp
from oracle.catalog import catalog_norms
from oracle.pipeline import MeshConfig, measure_pk
from oracle.ylm import Ylm, legendre
import synthcat

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _read(name):
    rows = []
    for line in open(f"{GOLDEN}/{name}"):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


def _random_field(n, seed):
    return np.random.default_rng(seed).normal(size=(n, n, n))


def test_F_ell_matches_bruteforce_legendre_dft():
    n, L = 8, 100.0
    obs = np.array([-40.0, -25.0, -60.0])
    delta = _random_field(n, 1)
    D = np.fft.fftn(delta)
    W = ms.compensation(n, ms.TSC)
    x = ms.node_positions(n, L)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1).reshape(-1, 3)
    r = X - obs
    rhat = r / np.linalg.norm(r, axis=1)[:, None]
    nidx = ms.freq_index(n)
    kf = 2 * math.pi / L
    for ell in (1, 2, 3, 4):
        F = sp.yamamoto_F(delta, D, ell, L, obs, W)
        for k in [(1, 0, 0), (1, 2, -3), (-2, 3, 1), (3, -1, 2), (0, 0, 2)]:
            kv = np.array(k, float) * kf
            kh = kv / np.linalg.norm(kv)
            brute = np.sum(delta.ravel() * np.exp(-1j * X @ kv) * legendre(ell, rhat @ kh))
            idx = tuple(int(np.where(nidx == k[a])[0][0]) for a in range(3))
            assert abs(F[idx] - brute / W[idx]) < 1e-11 * max(1.0, abs(brute))


def _neg_index(n):
    """Index map k -> -k on the FFT layout (the space inversion of the appendix)."""
    return (-np.arange(n)) % n


def test_conjugation_identity_and_parity():
    n, L = 12, 300.0
    obs = np.array([-100.0, -150.0, -130.0])
    delta = _random_field(n, 2)
    rvec = sp.line_of_sight(n, L, obs)
    neg = _neg_index(n)
    for ell in (1, 2, 3, 4):
        for m in range(1, ell + 1):
            Sp = np.fft.fftn(delta * Ylm(ell, m, rvec))
            Sm = np.fft.fftn(delta * Ylm(ell, -m, rvec))
            Sp_neg = Sp[np.ix_(neg, neg, neg)]
            assert np.allclose(Sm, (-1) ** m * np.conj(Sp_neg), atol=1e-12)
    W = ms.compensation(n, ms.CIC)
    D = np.fft.fftn(delta)
    for ell in (1, 2, 3, 4):
        F = sp.yamamoto_F(delta, D, ell, L, obs, W)
        Fneg = F[np.ix_(neg, neg, neg)]
        ok = ~ms.nyquist_mask(n)  # k -> -k maps a Nyquist plane onto itself
        assert np.allclose(F[ok], (-1) ** ell * np.conj(Fneg[ok]), atol=1e-10)


def test_calG_route_equals_F_route_below_nyquist():
    n, L = 16, 400.0
    obs = np.array([-200.0, -210.0, -190.0])
    delta = _random_field(n, 3)
    D = np.fft.fftn(delta)
    W = ms.compensation(n, ms.TSC)
    bins = sp.Bins(0.0, 2 * math.pi / L * 1.5, 5, L, n)
    F0 = sp.yamamoto_F(delta, D, 0, L, obs, W)
    neg = _neg_index(n)
    nyq = ms.nyquist_mask(n)
    for ell in (2, 4):
        F = sp.yamamoto_F(delta, D, ell, L, obs, W)
        G = sp.calG(delta, D, ell, L, obs, W)
        p_F = sp.power_raw(F0, F, bins)
        p_G = bins.shell_mean(np.real(F0 * np.conj(G)))
        assert np.allclose(p_F, p_G, rtol=1e-11, atol=1e-11 * np.max(np.abs(p_F)))
        recon = 0.5 * (G + (-1) ** ell * np.conj(G[np.ix_(neg, neg, neg)]))
        assert np.allclose(recon[~nyq], F[~nyq], atol=1e-10 * np.max(np.abs(F)))


def test_legendre_reexpansion_golden():
    x = np.linspace(-1, 1, 41)
    for tgt in (4, 6, 8):
        acc = np.zeros_like(x)
        for t, a, b, num, den in _read("legendre_reexpansion.txt"):
            if int(t) == tgt:
                acc += int(num) / int(den) * legendre(int(a), x) * legendre(int(b), x)
        assert np.allclose(acc, legendre(tgt, x), atol=1e-14)


def _legendre_product_coeffs(target):
    """Exact rational coefficients c_ab with L_target = sum c_ab L_a L_b, from the golden file."""
    return {(int(a), int(b)): Fraction(int(num), int(den))
            for t, a, b, num, den in _read("legendre_reexpansion.txt") if int(t) == target}


def test_modified_multipole_coefficients_follow_from_reexpansion():
    """eq. Plnew: P_(2L)b = (2*2L+1) sum c_ab <F_a F_b>/I22, rewritten in P_ab units."""
    got = {}
    for t, piece, num, den in _read("modified_multipoles.txt"):
        got[(int(t), piece)] = Fraction(int(num), int(den))
    for target in (4, 6, 8):
        expect = {}
        for (a, b), c in _legendre_product_coeffs(target).items():
            pref = Fraction(2 * target + 1)
            if b == 0:
                piece, norm = f"P{a}", Fraction(2 * a + 1)
            else:
                piece, norm = f"P{a}{b}", Fraction(2 * (a + b) + 1)
            expect[piece] = expect.get(piece, 0) + pref * c / norm
        for piece, val in expect.items():
            assert got[(target, piece)] == val, (target, piece)


def test_modified_multipoles_function_matches_golden():
    pieces = ("P0", "P2", "P4", "P22", "P42", "P44")
    coef = {}
    for t, piece, num, den in _read("modified_multipoles.txt"):
        coef[(int(t), piece)] = int(num) / int(den)
    for which, piece in enumerate(pieces):
        args = [np.array([1.0 if i == which else 0.0]) for i in range(6)]
        out = sp.modified_multipoles(*args)
        for t, val in zip((4, 6, 8), out):
            assert math.isclose(val[0], coef.get((t, piece), 0.0), abs_tol=1e-15)


def test_table1_fft_counts():
    est = {row[0]: (int(row[1]), int(row[2])) for row in _read("table1_fft_counts.txt")}
    for name, (c4, c8) in est.items():
        assert sp.fft_count(name, 4) == c4 and sp.fft_count(name, 8) == c8
        assert sp.fft_count_enumerated(name, 4) == c4 and sp.fft_count_enumerated(name, 8) == c8
    for lmax in (12, 16):
        for name in est:
            assert sp.fft_count(name, lmax) == sp.fft_count_enumerated(name, lmax)


def test_shot_noise_constants_of_Pllp():
    x, w = npleg.leggauss(40)
    for (l1, l2) in ((2, 2), (4, 4), (4, 2), (2, 0), (0, 0)):
        ang = 0.5 * np.sum(w * legendre(l1, x) * legendre(l2, x))
        assert math.isclose((2 * (l1 + l2) + 1) * ang, sp.N_llp(l1, l2, 1.0), abs_tol=1e-12)
    vals = {r[0]: Fraction(r[1]) for r in _read("special_values.txt")}
    assert sp.N_llp(2, 2, 1.0) == float(vals["N22_over_N0"])
    assert sp.N_llp(4, 4, 1.0) == float(vals["N44_over_N0"])


def _global_los_spectra(delta, L, los, ells):
    n = delta.shape[0]
    D = np.fft.fftn(delta)
    W = np.ones_like(D.real)
    return {l: sp.yamamoto_F(delta, D, l, L, None, W, los=los) for l in ells}


def test_global_los_modified_equals_traditional():
    n, L = 16, 500.0
    los = np.array([0.3, -0.5, 0.81])
    los /= np.linalg.norm(los)
    delta = _random_field(n, 4)
    F = _global_los_spectra(delta, L, los, (0, 2, 4, 6, 8))
    bins = sp.Bins(0.0, 2 * math.pi / L * 1.3, 6, L, n)
    I22, N0 = 3.7, 0.42
    P = {l: sp.pk_multipole(F[0], F[l], l, bins, I22, N0)[1] for l in (0, 2, 4, 6, 8)}
    PP = {(a, b): sp.pk_two_index(F[a], F[b], a, b, bins, I22, N0)[1]
          for (a, b) in ((2, 2), (4, 2), (4, 4))}
    P4b, P6b, P8b = sp.modified_multipoles(P[0], P[2], P[4], PP[(2, 2)], PP[(4, 2)], PP[(4, 4)])
    scale = max(np.max(np.abs(P[l])) for l in P)
    assert np.allclose(P4b, P[4], atol=1e-11 * scale)
    assert np.allclose(P6b, P[6], atol=1e-11 * scale)
    assert np.allclose(P8b, P[8], atol=1e-11 * scale)


def test_kaiser_fixed_amplitude_exact_and_ratios():
    n, L = 64, 1000.0
    los = np.array([0.0, 0.0, 1.0])
    delta = synthcat.fixed_amplitude_mesh(n, L, seed=11, los=los)
    F = _global_los_spectra(delta, L, los, (0, 2, 4))
    bins = sp.Bins(0.0, 0.01, 20, L, n)
    I22 = n ** 6 / L ** 3
    kvec = sp.kvectors(n, L)
    kk = np.linalg.norm(kvec, axis=-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = np.where(kk > 0, kvec[..., 2] / np.where(kk > 0, kk, 1), 0.0)
    pk = synthcat.field_power(kk) * (2.0 + 0.8 * mu * mu) ** 2
    P = {}
    for l in (0, 2, 4):
        P[l] = sp.pk_multipole(F[0], F[l], l, bins, I22, 0.0)[1]
        expect = (2 * l + 1) * bins.shell_mean(legendre(l, mu) * pk)
        assert np.allclose(P[l], expect, rtol=1e-10, atol=1e-10 * np.max(np.abs(expect)))
    b, f = 2.0, 0.8
    k0 = b * b + 2 * b * f / 3 + f * f / 5
    r2 = (4 * b * f / 3 + 4 * f * f / 7) / k0
    r4 = (8 * f * f / 35) / k0
    assert math.isclose(r2, 0.48108, abs_tol=5e-6) and math.isclose(r4, 0.028161, abs_tol=5e-7)
    sel = slice(10, 20)  # many modes per shell; the cubic lattice adds an l = 4 ripple
    assert np.allclose(P[2][sel] / P[0][sel], r2, atol=0.02)
    wts = bins.counts()[sel]
    assert abs(np.sum(wts * P[4][sel] / P[0][sel]) / np.sum(wts) - r4) < 0.02


def test_catalog_norms_closed_forms():
    g, _, r, _ = synthcat.tiny_catalog(80, 400, seed=3)
    L = 500.0
    obs = synthcat.observer_position()
    nr = catalog_norms(g, None, r, None, L, obs, (0, 2))
    ng, nrn = 80, 400
    alpha = ng / nrn
    nbar = ng / L ** 3
    assert math.isclose(nr.alpha, alpha)
    assert math.isclose(nr.I22, nbar * ng, rel_tol=1e-14)
    assert math.isclose(nr.I33, nbar ** 2 * ng, rel_tol=1e-14)
    assert math.isclose(nr.N0, (1 + alpha) / nbar, rel_tol=1e-14)
    assert math.isclose(nr.Sbar, ng - alpha ** 3 * nrn, rel_tol=1e-14)
    assert abs(nr.Sbar_lm[(0, 0)] - nr.Sbar) < 1e-10
    zl = catalog_norms(g, None, r, None, L, obs, (2, 4), los=np.array([0, 0, 1.0]))
    for (l, m), v in zl.Sbar_lm.items():
        assert abs(v - (nr.Sbar if m == 0 else 0.0)) < 1e-9


def test_poisson_catalog_pk_consistent_with_shot_noise():
    L, n = 1000.0, 32
    g = synthcat.poisson_catalog(40_000, seed=21)
    r = synthcat.random_catalog(400_000, seed=22)
    cfg = MeshConfig(L, n, ms.TSC, True, synthcat.observer_position())
    out = measure_pk(g, None, r, None, cfg, 0.0, 0.01, 8, ells=(0, 2))
    N0 = out["norms"].N0
    sigma = N0 * np.sqrt(2.0 / out["nmodes"])  # raw variance ~ 2 N0^2 per half-modes
    z = out["P0"] / sigma
    assert np.all(np.abs(z[1:]) < 5.0)
    assert abs(np.mean(out["P0_raw"][2:]) / N0 - 1.0) < 0.05


def test_odd_multipoles_G_route_and_global_los():
    n, L = 16, 400.0
    obs = np.array([-200.0, -210.0, -190.0])
    delta = _random_field(n, 5)
    D = np.fft.fftn(delta)
    W = ms.compensation(n, ms.TSC)
    bins = sp.Bins(0.0, 2 * math.pi / L * 1.5, 5, L, n)
    F0 = sp.yamamoto_F(delta, D, 0, L, obs, W)
    for ell in (1, 3):
        F = sp.yamamoto_F(delta, D, ell, L, obs, W)
        G = sp.calG(delta, D, ell, L, obs, W)
        p_F = sp.power_raw_imag(F0, F, bins)
        p_G = bins.shell_mean(np.imag(F0 * np.conj(G)))
        assert np.max(np.abs(p_F)) > 0
        assert np.allclose(p_F, p_G, rtol=1e-11, atol=1e-11 * np.max(np.abs(p_F)))
        # the real part of the full-grid shell sum vanishes for odd l (anti-Hermitian F_l)
        assert np.max(np.abs(sp.power_raw(F0, F, bins))) < 1e-11 * np.max(np.abs(p_F))
        # global line of sight: F_l = D L_l(khat . n) / W, so F_0 F_l* is real
        los = np.array([0.6, 0.0, 0.8])
        Fg = sp.yamamoto_F(delta, D, ell, L, obs, W, los=los)
        assert np.max(np.abs(sp.pk_multipole_odd(F0, Fg, ell, bins, 1.0))) < 1e-11 * np.max(np.abs(p_F))


def test_odd_multipoles_from_catalog_pipeline():
    """measure_pk returns P_1, P_3 as the imaginary-part estimator; they vanish
    for a global line of sight and not for the local one."""
    L, n = 1000.0, 32
    g = synthcat.lognormal_catalog(20_000, L, 61)
    r = synthcat.random_catalog(100_000, 62)
    obs = synthcat.observer_position()
    loc = measure_pk(g, None, r, None, MeshConfig(L, n, ms.TSC, True, obs), 0.0, 0.012, 6, ells=(0, 1, 3))
    glob = measure_pk(g, None, r, None, MeshConfig(L, n, ms.TSC, True, obs, los=np.ones(3) / math.sqrt(3)),
                      0.0, 0.012, 6, ells=(0, 1, 3))
    scale = np.max(np.abs(loc["P0"]))
    for l in (1, 3):
        assert np.max(np.abs(glob[f"P{l}"])) < 1e-10 * scale
        assert np.max(np.abs(loc[f"P{l}"])) > 1e-6 * scale


def test_cross_multipoles_self_and_symmetry():
    from oracle.pipeline import measure_pk_cross
    L, n = 1000.0, 32
    cfg = MeshConfig(L, n, ms.TSC, True, synthcat.observer_position())
    gA = synthcat.lognormal_catalog(15_000, L, 71)
    rA = synthcat.random_catalog(80_000, 72)
    gB = synthcat.lognormal_catalog(9_000, L, 73)
    rB = synthcat.random_catalog(60_000, 74)
    ells = (0, 1, 2, 3, 4)
    auto = measure_pk(gA, None, rA, None, cfg, 0.0, 0.012, 6, ells=ells)
    self_cross = measure_pk_cross(gA, None, rA, None, gA, None, rA, None, cfg, 0.0, 0.012, 6, ells=ells)
    for l in ells:
        assert np.allclose(self_cross[f"P{l}"], auto[f"P{l}_raw"], rtol=1e-12, atol=0), l
    ab = measure_pk_cross(gA, None, rA, None, gB, None, rB, None, cfg, 0.0, 0.012, 6, ells=(0,))
    ba = measure_pk_cross(gB, None, rB, None, gA, None, rA, None, cfg, 0.0, 0.012, 6, ells=(0,))
    assert np.allclose(ab["P0"], ba["P0"], rtol=1e-12)
    assert np.isclose(ab["I22"], math.sqrt(auto["norms"].I22 *
                                           measure_pk(gB, None, rB, None, cfg, 0.0, 0.012, 6, ells=(0,))["norms"].I22))


def _lattice_counts(nmesh, lo2, hi2):
    """Number of wave vectors n (|n_i| < N/2) with lo2 <= |n|^2 < hi2, by integer enumeration."""
    h = nmesh // 2
    r = np.arange(-h + 1, h)
    n2 = r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2
    return int(np.count_nonzero((n2 >= lo2) & (n2 < hi2) & (n2 > 0)))


@pytest.mark.parametrize("kmin_f, dk_f", [(0, 1), (3, 2), (0, 2)])
def test_mode_counts_on_integer_edges(kmin_f, dk_f):
    """Half-open bins whose edges fall exactly on integer |n| (reading R6): a mode
    with |n| on an edge belongs to the upper bin.  With dk = k_f the FP64 square of
    edge 27, (27 dk / k_f)^2, rounds to 729.0000000000002; the counts must not move
    the 30 modes of |n|^2 = 729 down a bin.  Reference counts by integer enumeration;
    the first few by hand from the sums of three squares r3(n^2) = 6, 12, 8, 6, 24, 24,
    0, 12, 30 for n^2 = 1..9: [0, 1) -> 0 modes, [1, 2) -> 6 + 12 + 8 = 26,
    [2, 3) -> 6 + 24 + 24 + 12 = 66."""
    n, box = 64, 1000.0
    kf = 2 * math.pi / box
    nb = 30 if dk_f == 1 else 14
    bins = sp.Bins(kmin_f * kf, dk_f * kf, nb, box, n)
    got = bins.counts()
    for b in range(nb):
        lo = (kmin_f + b * dk_f) ** 2
        hi = (kmin_f + (b + 1) * dk_f) ** 2
        assert got[b] == _lattice_counts(n, lo, hi), (b, got[b])
    if (kmin_f, dk_f) == (0, 1):
        assert list(got[:3]) == [0, 26, 66]
        assert got[27] == _lattice_counts(n, 729, 784)
