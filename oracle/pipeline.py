"""End-to-end oracle measurements from catalogs (plain composition of the
modules of this package, in the order the estimators are defined)."""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import bispectrum as bk
from . import mesh as ms
from . import shotnoise as sn
from . import spectra as sp
from .catalog import catalog_norms


@dataclass
class MeshConfig:
    boxsize: float
    nmesh: int
    assign: int = ms.TSC
    interlace: bool = True
    observer: Optional[np.ndarray] = None
    los: Optional[np.ndarray] = None  # fixed unit vector => global line of sight


def fkp_spectra(gpos, gw, rpos, rw, cfg: MeshConfig, ells=(0, 2, 4), noise_ells=()):
    """Norms, W, and F_l of the FKP field (and of the N mesh for noise_ells)."""
    obs = cfg.observer
    sbar_ells = sorted({l for l in set(ells) | set(noise_ells) | {0} if l % 2 == 0})
    norms = catalog_norms(gpos, gw, rpos, rw, cfg.boxsize, obs, sbar_ells, cfg.los)
    want_noise = len(noise_ells) > 0
    delta, nm = ms.paint_fkp(gpos, gw, rpos, rw, norms.alpha, cfg.nmesh, cfg.assign,
                             cfg.interlace, noise=want_noise)
    W = ms.compensation(cfg.nmesh, cfg.assign)
    D, dint = ms.deinterlace(delta[0], delta[1] if cfg.interlace else None)
    F = {l: sp.yamamoto_F(dint, D, l, cfg.boxsize, obs, W, cfg.los) for l in ells}
    FN = {}
    if want_noise:
        DN, nint = ms.deinterlace(nm[0], nm[1] if cfg.interlace else None)
        FN = {l: sp.yamamoto_F(nint, DN, l, cfg.boxsize, obs, W, cfg.los)
              for l in sorted(set(noise_ells) | {0})}
    return norms, W, F, FN


def measure_pk(gpos, gw, rpos, rw, cfg: MeshConfig, kmin, dk, nbins, ells=(0, 2, 4),
               modified=False):
    norms, W, F, _ = fkp_spectra(gpos, gw, rpos, rw, cfg, ells)
    bins = sp.Bins(kmin, dk, nbins, cfg.boxsize, cfg.nmesh)
    out = {"norms": norms, "nmodes": bins.counts(), "k_eff": bins.k_eff()}
    for l in ells:
        if l % 2:
            out[f"P{l}_raw"] = out[f"P{l}"] = sp.pk_multipole_odd(F[0], F[l], l, bins, norms.I22)
            continue
        raw, sub = sp.pk_multipole(F[0], F[l], l, bins, norms.I22, norms.N0)
        out[f"P{l}_raw"], out[f"P{l}"] = raw, sub
    if modified:
        pp = {}
        for (a, b) in ((2, 2), (4, 2), (4, 4)):
            raw, sub = sp.pk_two_index(F[a], F[b], a, b, bins, norms.I22, norms.N0)
            out[f"P{a}{b}_raw"], out[f"P{a}{b}"] = raw, sub
            pp[(a, b)] = sub
        out["P4b"], out["P6b"], out["P8b"] = sp.modified_multipoles(
            out["P0"], out["P2"], out["P4"], pp[(2, 2)], pp[(4, 2)], pp[(4, 4)])
    return out


def measure_pk_cross(gA, wA, rA, wrA, gB, wB, rB, wrB, cfg: MeshConfig, kmin, dk, nbins, ells=(0, 2, 4)):
    """Cross multipoles of two tracers A and B (each with its own randoms):
    (2l+1)/I22^AB <F_0^A F_l^B*> per bin, the real part for even l and the
    imaginary part for odd l, with I22^AB = sqrt(I22^A I22^B) and no shot
    noise (distinct samples share no galaxy)."""
    nA, _, FA, _ = fkp_spectra(gA, wA, rA, wrA, cfg, (0,))
    nB, _, FB, _ = fkp_spectra(gB, wB, rB, wrB, cfg, ells)
    I22 = float(np.sqrt(nA.I22 * nB.I22))
    bins = sp.Bins(kmin, dk, nbins, cfg.boxsize, cfg.nmesh)
    out = {"I22": I22, "nmodes": bins.counts()}
    for l in ells:
        part = sp.power_raw_imag if l % 2 else sp.power_raw
        out[f"P{l}"] = (2 * l + 1) / I22 * part(FA[0], FB[l], bins)
    return out


def noise_terms(F, FN, ell, bins_ext, norms, W, cfg):
    """Q_l and H_l on the (extended) binning."""
    C = sn.c_shot(cfg.nmesh, cfg.assign, cfg.interlace)
    s = sn.self_term(ell, norms.Sbar_lm, bins_ext, W, C)
    Q = sp.power_raw(F[ell], FN[0], bins_ext) - s
    H = sp.power_raw(F[0], FN[ell], bins_ext) - s
    return Q, H, s


def measure_bk(gpos, gw, rpos, rw, cfg: MeshConfig, dk, nbins, ells=(0, 2),
               scoccimarro=(0, 2), triposh=(0, 2), fft_noise=False):
    """Scoccimarro B_l and TripoSH BB_l0l with analytic shot noise (kmin = 0);
    fft_noise adds BB_l0l with the FFT-method i = j != k term ("BBl0l_shot_fft",
    "BBl0l_fft")."""
    norms, W, F, FN = fkp_spectra(gpos, gw, rpos, rw, cfg, ells, noise_ells=ells)
    bins = sp.Bins(0.0, dk, nbins, cfg.boxsize, cfg.nmesh)
    ext = sp.Bins(0.0, dk, 2 * nbins - 1, cfg.boxsize, cfg.nmesh)
    centres = bins.centres()
    out = {"norms": norms, "nmodes": bins.counts()}
    for l in scoccimarro:
        cfgs = bk.scoccimarro_configs(nbins, l)
        nt = bk.triangle_counts(bins, cfgs)
        keep = [c for c, n in zip(cfgs, nt) if n > 0]
        nt = np.array([n for n in nt if n > 0])
        raw = bk.scoccimarro_raw(F[0], F[l], l, bins, norms.I33, keep, nt)
        Q, H, _ = noise_terms(F, FN, l, bins, norms, W, cfg)
        shot = sn.scoccimarro_shot(l, keep, Q, H, centres, norms.I33, norms.Sbar)
        out[f"B{l}_configs"], out[f"B{l}_ntri"] = keep, nt
        out[f"B{l}_raw"], out[f"B{l}_shot"], out[f"B{l}"] = raw, shot, raw - shot
    for l in triposh:
        pairs = bk.triposh_pairs(nbins)
        raw = bk.triposh_raw(F[0], F[l], l, bins, norms.I33, pairs)
        Q, H, _ = noise_terms(F, FN, l, ext, norms, W, cfg)
        shot = sn.triposh_shot(l, pairs, Q, H, ext.counts(), ext.centres(), norms.I33,
                               norms.Sbar)
        out[f"BB{l}0{l}_pairs"] = pairs
        out[f"BB{l}0{l}_raw"], out[f"BB{l}0{l}_shot"] = raw, shot
        out[f"BB{l}0{l}"] = raw - shot
        if fft_noise:
            C = sn.c_shot(cfg.nmesh, cfg.assign, cfg.interlace)
            s_modes = sn.self_term_modes(l, norms.Sbar_lm, cfg.nmesh, cfg.boxsize, W, C)
            P = sn.noise_product(F[l], FN[0], s_modes)
            T = sn.exact_pair_sums(P, bins, pairs)
            sf = sn.triposh_shot_fft(l, pairs, T, H, bins.counts(), centres, norms.I33, norms.Sbar)
            out[f"BB{l}0{l}_pairsum"] = T
            out[f"BB{l}0{l}_shot_fft"], out[f"BB{l}0{l}_fft"] = sf, raw - sf
    return out


def measure_sugiyama(gpos, gw, rpos, rw, cfg: MeshConfig, dk, nbins, l1, l2, L, fft_noise=False):
    """Sugiyama B_l1l2L(k_i, k_j) (all i, j) with its analytic shot noise (kmin = 0);
    fft_noise adds "shot_fft" and "value_fft" (the FFT-method i = j != k term)."""
    from . import sugiyama as sg
    obs = cfg.observer
    norms, W, F, FN = fkp_spectra(gpos, gw, rpos, rw, cfg, tuple(sorted({0, L})), noise_ells=(L,))
    delta, _ = ms.paint_fkp(gpos, gw, rpos, rw, norms.alpha, cfg.nmesh, cfg.assign, cfg.interlace,
                            noise=False)
    _, dint = ms.deinterlace(delta[0], delta[1] if cfg.interlace else None)
    bins = sp.Bins(0.0, dk, nbins, cfg.boxsize, cfg.nmesh)
    ext = sp.Bins(0.0, dk, 2 * nbins - 1, cfg.boxsize, cfg.nmesh)
    raw = sg.sugiyama_raw(F[0], dint, W, l1, l2, L, bins, norms.I33, cfg.boxsize, obs, cfg.los)
    Q, H, _ = noise_terms(F, FN, L, ext, norms, W, cfg)
    shot = sg.sugiyama_shot(l1, l2, L, nbins, Q, H, ext.counts(), ext.centres(), norms.I33, norms.Sbar)
    out = {"norms": norms, "raw": raw, "shot": shot, "value": raw - shot, "nmodes": bins.counts()}
    if fft_noise:
        C = sn.c_shot(cfg.nmesh, cfg.assign, cfg.interlace)
        term = sg.sugiyama_fft_term(dint, W, FN[0], C, norms.Sbar_lm, l1, l2, L, bins, norms.I33,
                                    cfg.boxsize, obs, cfg.los)
        out["fft_term"] = term
        out["shot_fft"] = sg.sugiyama_shot_fft(l1, l2, L, nbins, term, H, norms.I33, norms.Sbar)
        out["value_fft"] = raw - out["shot_fft"]
    return out
