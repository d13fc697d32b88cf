"""Pins of the analytic l > 0 bispectrum shot noise (section "Derivation of shot
noise in three different bispectrum estimators": the Scoccimarro and
new-estimator subsections, eq. I_l0l, Lemma 2 / eq. g_ell).

1. The exact closure sums of ``oracle.shotnoise_exact`` are checked, case by
   case, against a brute-force split of the particle triple product on a tiny
   catalog (direct Fourier sums over the particles, no mesh): the sum over
   distinct particles of legs (1, 2, 3) is removed by enumeration and each
   coincidence case (two legs or all three on one particle) is enumerated on its
   own.  This fixes which per-mode product belongs to which case, its conjugation
   and its self-pair subtraction, independently of any thin-shell step.
2. The analytic thin-shell terms of ``oracle.shotnoise`` (Q_l, L_l(mu) H_l,
   g_l(t) H_l) are compared term by term with those exact sums on a clustered,
   anisotropic catalog at l = 2.  Planted mistakes (the Legendre factor of the
   other leg, the H of the other leg, g_l(t) for g_l(1/t)) are shown to fail the
   same tolerance, so the pin separates the right assembly from them.
   Q_l and H_l differ only by wide-angle terms at these wavenumbers, so an
   exchange of the two is not resolved here (the case split of pin 1 fixes it).
"""

from __future__ import annotations

import math

import numpy as np
import pytest

import synthcat
from oracle import bispectrum as bk
from oracle import mesh as ms
from oracle import shotnoise as sn
from oracle import shotnoise_exact as se
from oracle import spectra as sp
from oracle.pipeline import MeshConfig, fkp_spectra, noise_terms
from oracle.ylm import legendre, ylm_racah


# ---------------------------------------------------------------- pin 1 --

def _direct_spectra(ell, seed=3):
    """Per-particle Fourier sums on a 16^3 wave-vector grid (no painting: W = C = 1)."""
    rng = np.random.default_rng(seed)
    n, box = 16, 1000.0
    npart = 9
    x = rng.uniform(0, box, size=(npart, 3))
    c = rng.uniform(0.5, 1.5, size=npart) * np.where(rng.uniform(size=npart) < 0.5, 1.0, -0.3)
    obs = np.array([-800.0, -700.0, -900.0])
    xh = x - obs
    kv = sp.kvectors(n, box)
    kn = np.linalg.norm(kv, axis=-1)
    kn[0, 0, 0] = 1.0
    khat = kv / kn[..., None]
    ph = np.exp(-1j * np.einsum("abcd,pd->abcp", kv, x))
    xu = xh / np.linalg.norm(xh, axis=1)[:, None]
    Lq = legendre(ell, np.einsum("abcd,pd->abcp", khat, xu))
    d = dict(n=n, box=box, c=c, ph=ph, Lq=Lq)
    d["F0"] = np.sum(c * ph, axis=-1)
    d["Fl"] = np.sum(c * ph * Lq, axis=-1)
    Nq = np.sum(c ** 2 * ph, axis=-1)
    s = np.sum(c ** 3 * Lq, axis=-1)
    d["Sbar"] = {(ell, m): np.sum(c ** 3 * np.conj(ylm_racah(ell, m, xh))) for m in range(-ell, ell + 1)}
    M = {m: np.sum(c ** 2 * np.conj(ylm_racah(ell, m, xh)) * ph, axis=-1) for m in range(-ell, ell + 1)}
    one = np.ones((n, n, n))
    d["Z"] = se.leg_products(d["F0"], M, d["Sbar"], ell, one, one)
    P = np.where(ms.nyquist_mask(n), 0.0, d["Fl"] * np.conj(Nq) - s)
    P[0, 0, 0] = 0.0
    d["P"] = P
    return d


def _case_masks(npart):
    a = np.arange(npart)
    A, B, C = a[:, None, None], a[None, :, None], a[None, None, :]
    return {
        "23": (B == C) & (A != B),
        "13": (A == C) & (A != B),
        "12": (A == B) & (A != C),
        "123": (A == B) & (B == C),
    }


def _signed_modes(shells, b):
    n = shells.shape[0]
    idx = np.argwhere(shells == b)
    return np.where(idx > n // 2, idx - n, idx)


@pytest.mark.parametrize("ell", [0, 2])
def test_scoccimarro_cases_by_particle_enumeration(ell):
    d = _direct_spectra(ell)
    n = d["n"]
    kf = 2 * math.pi / d["box"]
    bins = sp.Bins(0.0, 1.3 * kf, 3, d["box"], n)  # |q1 + q2 + q3| components < N: no wrap
    shells = bins.shell_index()
    configs = bk.scoccimarro_configs(3, ell)
    ex = se.scoccimarro_exact_terms(ell, configs, shells, d["P"], d["Z"], d["Sbar"], d["box"])
    masks = _case_masks(len(d["c"]))
    # legs (1, 2, 3) = (l leg on shell i, shell j, shell k); case names of the module
    name = {"23": "jk", "13": "ik", "12": "ij", "123": "ijk"}
    for t, (i, j, k) in enumerate(configs):
        ref = {key: 0.0j for key in masks}
        for q1 in _signed_modes(shells, i):
            for q2 in _signed_modes(shells, j):
                q3 = -q1 - q2
                if np.any(np.abs(q3) >= n // 2) or shells[tuple(q3 % n)] != k:
                    continue
                a1, a2, a3 = tuple(q1 % n), tuple(q2 % n), tuple(q3 % n)
                e1 = d["c"] * d["ph"][a1] * d["Lq"][a1]
                e2 = d["c"] * d["ph"][a2]
                e3 = d["c"] * d["ph"][a3]
                full = np.einsum("a,b,c->abc", e1, e2, e3)
                for key, msk in masks.items():
                    ref[key] += np.sum(full[msk])
        for key, msk in masks.items():
            got = ex[name[key]][t]
            scale = max(1.0, abs(ref[key]))
            assert abs(got - ref[key]) <= 1e-10 * scale, ((i, j, k), key, got, ref[key])


def test_triposh_cases_by_particle_enumeration():
    ell = 2
    d = _direct_spectra(ell, seed=8)
    n = d["n"]
    kf = 2 * math.pi / d["box"]
    bins = sp.Bins(0.0, 1.3 * kf, 3, d["box"], n)
    shells = bins.shell_index()
    pairs = bk.triposh_pairs(3)
    ex = se.triposh_exact_terms(ell, pairs, shells, d["P"], d["Z"], d["Sbar"], d["box"])
    masks = _case_masks(len(d["c"]))
    for t, (i, j) in enumerate(pairs):
        ref = {key: 0.0j for key in masks}
        for q1 in _signed_modes(shells, i):
            for q2 in _signed_modes(shells, j):
                q3 = -q1 - q2
                if not np.any(q3):
                    continue  # F_l(0) := 0
                a1, a2, a3 = tuple(q1 % n), tuple(q2 % n), tuple(q3 % n)
                # legs (1, 2, 3) = (F_0 on shell i, F_0 on shell j, F_l on q3)
                e1 = d["c"] * d["ph"][a1]
                e2 = d["c"] * d["ph"][a2]
                e3 = d["c"] * d["ph"][a3] * d["Lq"][a3]
                full = np.einsum("a,b,c->abc", e1, e2, e3)
                for key, msk in masks.items():
                    ref[key] += np.sum(full[msk])
        for key in masks:
            got = ex[key][t]
            assert abs(got - ref[key]) <= 1e-10 * max(1.0, abs(ref[key])), ((i, j), key, got, ref[key])


# ---------------------------------------------------------------- pin 2 --

@pytest.fixture(scope="module")
def clustered_l2():
    """Kaiser lognormal catalog, 96^3 TSC + interlacing, 12 bins of 2 k_f."""
    L, n, ell = 1000.0, 96, 2
    g = synthcat.lognormal_catalog(100_000, L, 101)
    r = synthcat.random_catalog(1_000_000, 102)
    cfg = MeshConfig(L, n, ms.TSC, True, synthcat.observer_position())
    norms, W, F, FN = fkp_spectra(g, None, r, None, cfg, (0, ell), noise_ells=(0, ell))
    _, nm = ms.paint_fkp(g, None, r, None, norms.alpha, n, ms.TSC, True, noise=True)
    _, n_int = ms.deinterlace(nm[0], nm[1])
    C = sn.c_shot(n, ms.TSC, True)
    M = se.noise_harmonic_spectra(n_int, ell, L, cfg.observer, W)
    Z = se.leg_products(F[0], M, norms.Sbar_lm, ell, C, W)
    P = sn.noise_product(F[ell], FN[0], sn.self_term_modes(ell, norms.Sbar_lm, n, L, W, C))
    dk, nb = 0.0125, 12
    bins = sp.Bins(0.0, dk, nb, L, n)
    ext = sp.Bins(0.0, dk, 2 * nb - 1, L, n)
    return dict(L=L, n=n, ell=ell, cfg=cfg, norms=norms, W=W, F=F, FN=FN, Z=Z, P=P,
                bins=bins, ext=ext, bmin=5)


def _rel(exact, approx, ref):
    return float(np.max(np.abs(exact - approx)) / np.max(np.abs(ref)))


def test_scoccimarro_l2_terms_against_exact(clustered_l2):
    d = clustered_l2
    ell, bins = d["ell"], d["bins"]
    cfgs = [c for c in bk.scoccimarro_configs(bins.nbins, ell) if min(c) >= d["bmin"]]
    rng = np.random.default_rng(0)
    keep = [cfgs[s] for s in sorted(rng.choice(len(cfgs), size=30, replace=False))]
    nt = bk.triangle_counts(bins, keep).astype(np.float64)
    ex = se.scoccimarro_exact_terms(ell, keep, bins.shell_index(), d["P"], d["Z"],
                                    d["norms"].Sbar_lm, d["L"])
    Q, H, _ = noise_terms(d["F"], d["FN"], ell, bins, d["norms"], d["W"], d["cfg"])
    cen = bins.centres()
    an = sn.scoccimarro_shot_terms(ell, keep, Q, H, cen, d["norms"].Sbar)
    exr = {key: ex[key].real / nt for key in ex}
    for key in ex:
        assert np.max(np.abs(ex[key].imag / nt)) < 1e-8 * np.max(np.abs(Q))
    # thin-shell tolerances (fraction of the term's largest value): the two l = 0
    # legs on one particle need no angular step (5%); the Legendre factor of a
    # closed triangle from bin centres is the coarser step (15%)
    assert _rel(exr["jk"], an["jk"], an["jk"]) < 0.05
    assert _rel(exr["ik"], an["ik"], an["ik"]) < 0.15
    assert _rel(exr["ij"], an["ij"], an["ij"]) < 0.15
    assert np.max(np.abs(exr["ijk"])) < 1e-9 * abs(d["norms"].Sbar)  # no l = 2 cubic invariant
    # the whole term, as the estimator subtracts it
    shot = sn.scoccimarro_shot(ell, keep, Q, H, cen, d["norms"].I33, d["norms"].Sbar)
    shot_exact = (2 * ell + 1) / d["norms"].I33 * (exr["jk"] + exr["ik"] + exr["ij"] + exr["ijk"])
    assert _rel(shot_exact, shot, shot) < 0.10
    # planted mistakes fail the same bars
    mu = []
    for (i, j, k) in keep:
        ki, kj, kk = cen[i], cen[j], cen[k]
        mu.append((np.clip((kk * kk - ki * ki - kj * kj) / (2 * ki * kj), -1, 1),
                   np.clip((kj * kj - ki * ki - kk * kk) / (2 * ki * kk), -1, 1)))
    other_mu = np.array([legendre(ell, m13) * H[j] for (m12, m13), (i, j, k) in zip(mu, keep)])
    other_leg = np.array([legendre(ell, m12) * H[k] for (m12, m13), (i, j, k) in zip(mu, keep)])
    assert _rel(exr["ik"], other_mu, an["ik"]) > 0.3
    assert _rel(exr["ik"], other_leg, an["ik"]) > 0.25


def test_triposh_l2_terms_against_exact(clustered_l2):
    d = clustered_l2
    ell, bins, ext = d["ell"], d["bins"], d["ext"]
    pairs = [(i, j) for (i, j) in bk.triposh_pairs(bins.nbins) if i >= d["bmin"]]
    cnt = bins.counts().astype(np.float64)
    ex = se.triposh_exact_terms(ell, pairs, bins.shell_index(), d["P"], d["Z"],
                                d["norms"].Sbar_lm, d["L"])
    nn = np.array([cnt[i] * cnt[j] for i, j in pairs])
    exr = {key: (2 * ell + 1) * ex[key].real / nn for key in ex}
    exr["123"] = ex["123"].real / nn
    Qe, He, _ = noise_terms(d["F"], d["FN"], ell, ext, d["norms"], d["W"], d["cfg"])
    an = sn.triposh_shot_terms(ell, pairs, Qe, He, ext.counts(), ext.centres(), d["norms"].Sbar)
    assert _rel(exr["12"], an["12"], an["12"]) < 0.05
    assert _rel(exr["13"], an["13"], an["13"]) < 0.05
    assert _rel(exr["23"], an["23"], an["23"]) < 0.05
    assert np.max(np.abs(exr["123"])) < 1e-9 * abs(d["norms"].Sbar)
    shot = sn.triposh_shot(ell, pairs, Qe, He, ext.counts(), ext.centres(), d["norms"].I33,
                           d["norms"].Sbar)
    shot_exact = (exr["12"] + exr["13"] + exr["23"] + exr["123"]) / d["norms"].I33
    assert _rel(shot_exact, shot, shot) < 0.05
    # the i = j != k term agrees with the oracle's FFT-method pair sums as well
    T = sn.exact_pair_sums(d["P"], bins, pairs)
    np.testing.assert_allclose((2 * ell + 1) * T / nn, exr["12"], rtol=1e-9,
                               atol=1e-9 * np.max(np.abs(exr["12"])))
    # planted mistakes: g_l(t) and g_l(1/t) exchanged
    ce = ext.centres()
    swapped_13 = np.array([(2 * ell + 1) * sn.g_ell(ell, ce[i] / ce[j]) * He[j] for i, j in pairs])
    swapped_23 = np.array([(2 * ell + 1) * sn.g_ell(ell, ce[j] / ce[i]) * He[i] for i, j in pairs])
    assert _rel(exr["13"], swapped_13, an["13"]) > 0.3
    assert _rel(exr["23"], swapped_23, an["23"]) > 0.3
