"""End-to-end measurements composed from the C ABI calls.

Torch provides device memory and the stream; every arithmetic step runs in the
HIP library.  Results stay on the device (FP64 tensors) until the caller reads
them.
"""

from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass, field
from typing import Dict, Optional, Sequence

import torch

from . import _lib as L

_TORCH_DT = {L.F32: torch.float32, L.F64: torch.float64}


class Scratch:
    """One growable device byte buffer shared by consecutive calls on a stream."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = torch.empty(0, dtype=torch.uint8, device=device)

    def get(self, nbytes: int):
        nbytes = max(int(nbytes), 256)
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf


def _sh(stream):
    return L.stream_handle(stream)


def _empty(shape, dtype, device="cuda"):
    return torch.empty(shape, dtype=dtype, device=device)


def catalog_norms(desc, gpos, rpos, gw=None, rw=None, scratch: Optional[Scratch] = None, stream=None):
    """FP64 catalog sums of both catalogs and the normalisations (device)."""
    sc = scratch or Scratch()
    s = _sh(stream)
    ws = sc.get(L.lib.cnpc_catalog_sums_workspace_size())
    gs = _empty(L.SUMS_LEN, torch.float64)
    rs = _empty(L.SUMS_LEN, torch.float64)
    L.check(L.lib.cnpc_catalog_sums(C.byref(desc), L.ptr(gpos), L.ptr(gw), gpos.shape[1], L.ptr(gs),
                                    L.ptr(ws), ws.numel(), s))
    L.check(L.lib.cnpc_catalog_sums(C.byref(desc), L.ptr(rpos), L.ptr(rw), rpos.shape[1], L.ptr(rs),
                                    L.ptr(ws), ws.numel(), s))
    norms = _empty(L.NORMS_LEN, torch.float64)
    L.check(L.lib.cnpc_norms(C.byref(desc), L.ptr(gs), L.ptr(rs), gpos.shape[1], L.ptr(norms), s))
    return norms, gs, rs


def paint(desc, gpos, rpos, norms, gw=None, rw=None, noise=True, scratch: Optional[Scratch] = None,
          stream=None):
    sc = scratch or Scratch()
    n = desc.n
    nph = 2 if desc.interlace else 1
    dt = _TORCH_DT[desc.dtype]
    delta = _empty((nph, n, n, n), dt)
    nmesh = _empty((nph, n, n, n), dt) if noise else None
    ws = sc.get(L.lib.cnpc_paint_workspace_size(C.byref(desc), gpos.shape[1], rpos.shape[1]))
    L.check(L.lib.cnpc_paint(C.byref(desc), L.ptr(gpos), L.ptr(gw), gpos.shape[1], L.ptr(rpos),
                             L.ptr(rw), rpos.shape[1], L.ptr(norms), L.ptr(delta), L.ptr(nmesh),
                             L.ptr(ws), ws.numel(), _sh(stream)))
    return delta, nmesh


def paint_outputs(desc, noise=True):
    """Output buffers of paint_fkp: (norms, delta, noise mesh or None, galaxy
    sums, random sums)."""
    n = desc.n
    nph = 2 if desc.interlace else 1
    dt = _TORCH_DT[desc.dtype]
    return (_empty(L.NORMS_LEN, torch.float64), _empty((nph, n, n, n), dt),
            _empty((nph, n, n, n), dt) if noise else None, _empty(L.SUMS_LEN, torch.float64),
            _empty(L.SUMS_LEN, torch.float64))


def paint_fkp(desc, gpos, rpos, gw=None, rw=None, noise=True, sums_lmax=4,
              scratch: Optional[Scratch] = None, stream=None, out=None):
    """Catalog sums (Y_lm sums for l <= sums_lmax), normalisations and painting
    in one library call.  Returns (norms, delta, noise mesh or None, galaxy sums,
    random sums), written into `out` (from paint_outputs) when given."""
    sc = scratch or Scratch()
    norms, delta, nmesh, gs, rs = out if out is not None else paint_outputs(desc, noise)
    if noise and nmesh is None:
        raise ValueError("paint_fkp: noise requested without a noise mesh")
    ws = sc.get(L.lib.cnpc_paint_workspace_size(C.byref(desc), gpos.shape[1], rpos.shape[1]))
    L.check(L.lib.cnpc_paint_fkp(C.byref(desc), L.ptr(gpos), L.ptr(gw), gpos.shape[1], L.ptr(rpos),
                                 L.ptr(rw), rpos.shape[1], int(sums_lmax), L.ptr(gs), L.ptr(rs), L.ptr(norms),
                                 L.ptr(delta), L.ptr(nmesh), L.ptr(ws), ws.numel(), _sh(stream)))
    return norms, delta, nmesh, gs, rs


def fold_fused_supported(desc) -> bool:
    """cnpc_paint_deinterlace covers this mesh: interlaced 256^3 with the
    register FFT passes, the fused form not switched off by its tuning knob."""
    return (bool(desc.interlace) and desc.n == 256
            and L.lib.cnpc_tune_get(L.TUNE["fft_passes"][0]) != 1
            and L.lib.cnpc_tune_get(L.TUNE["fold_fused"][0]) != 1)


def paint_deinterlace(desc, band, gpos, rpos, gw=None, rw=None, sums_lmax=4,
                      scratch: Optional[Scratch] = None, stream=None):
    """Painting and both de-interlacing transforms in one library call
    (cnpc_paint_deinterlace).  Returns (norms, D, delta_int, DN, galaxy sums,
    random sums)."""
    sc = scratch or Scratch()
    n = desc.n
    dt = _TORCH_DT[desc.dtype]
    norms = _empty(L.NORMS_LEN, torch.float64)
    gs = _empty(L.SUMS_LEN, torch.float64)
    rs = _empty(L.SUMS_LEN, torch.float64)
    D = _empty((band_size(band), 2), dt)
    DN = _empty((band_size(band), 2), dt)
    dint = _empty((n, n, n), dt)
    weighted = int(gw is not None or rw is not None)
    ws = sc.get(L.lib.cnpc_paint_deinterlace_workspace_size(C.byref(desc), gpos.shape[1], rpos.shape[1],
                                                             weighted, band))
    L.check(L.lib.cnpc_paint_deinterlace(C.byref(desc), band, L.ptr(gpos), L.ptr(gw), gpos.shape[1],
                                         L.ptr(rpos), L.ptr(rw), rpos.shape[1], int(sums_lmax), L.ptr(gs),
                                         L.ptr(rs), L.ptr(norms), L.ptr(D), L.ptr(dint), L.ptr(DN), L.ptr(ws),
                                         ws.numel(), _sh(stream)))
    return norms, D, dint, DN, gs, rs


def band_size(band: int) -> int:
    return 4 * band ** 3


def deinterlace(desc, band, meshes, want_real=True, scratch: Optional[Scratch] = None, stream=None):
    sc = scratch or Scratch()
    n = desc.n
    dt = _TORCH_DT[desc.dtype]
    spec = _empty((band_size(band), 2), dt)
    real = _empty((n, n, n), dt) if want_real else None
    ws = sc.get(L.lib.cnpc_deinterlace_workspace_size(C.byref(desc)))
    L.check(L.lib.cnpc_deinterlace(C.byref(desc), band, L.ptr(meshes), L.ptr(spec), L.ptr(real),
                                   L.ptr(ws), ws.numel(), _sh(stream)))
    return spec, real


def ylm_spectra(desc, band, ells: Sequence[int], delta_int, scratch: Optional[Scratch] = None,
                stream=None):
    sc = scratch or Scratch()
    ells = [int(l) for l in ells if l > 0]
    nf = sum(2 * l + 1 for l in ells)
    dt = _TORCH_DT[desc.dtype]
    out = _empty((nf, band_size(band), 2), dt)
    arr = (C.c_int32 * len(ells))(*ells)
    ws = sc.get(L.lib.cnpc_ylm_r2c_workspace_size(C.byref(desc), nf, band))
    L.check(L.lib.cnpc_ylm_r2c(C.byref(desc), band, len(ells), arr, L.ptr(delta_int), L.ptr(out),
                               L.ptr(ws), ws.numel(), _sh(stream)))
    res, f = {}, 0
    for l in ells:
        res[l] = out[f:f + 2 * l + 1]
        f += 2 * l + 1
    return res


def assemble(desc, band, ell, spec0=None, ylm=None, stream=None):
    dt = _TORCH_DT[desc.dtype]
    F = _empty((band_size(band), 2), dt)
    L.check(L.lib.cnpc_assemble_F(C.byref(desc), band, ell, L.ptr(spec0), L.ptr(ylm), L.ptr(F),
                                  _sh(stream)))
    return F


def bin_means(desc, bins, band, pairs, self_ells=(), norms=None, scratch: Optional[Scratch] = None,
              stream=None, imag=False):
    """Shell means of Re F_a F_b^* (imag=False) or Im F_a F_b^* (imag=True,
    no self terms) for the (a, b) in pairs; self terms s_l; mode counts; k_eff."""
    sc = scratch or Scratch()
    if imag and self_ells:
        raise ValueError("self terms go with the real-part means")
    nb = bins.nbins
    npairs, nself = len(pairs), len(self_ells)
    means = _empty((max(npairs, 1), nb), torch.float64)
    selft = _empty((max(nself, 1), nb), torch.float64)
    nmodes = _empty(nb, torch.int64)
    keff = _empty(nb, torch.float64)
    pa = (C.c_void_p * max(npairs, 1))(*[L.ptr(a) for a, _ in pairs])
    pb = (C.c_void_p * max(npairs, 1))(*[L.ptr(b) for _, b in pairs])
    se = (C.c_int32 * max(nself, 1))(*[int(l) for l in self_ells])
    ws = sc.get(L.lib.cnpc_bin_pk_workspace_size(C.byref(bins), npairs, nself))
    if imag:
        L.check(L.lib.cnpc_bin_pk_im(C.byref(desc), C.byref(bins), band, npairs, pa, pb, L.ptr(means),
                                     L.ptr(nmodes), L.ptr(keff), L.ptr(ws), ws.numel(), _sh(stream)))
    else:
        L.check(L.lib.cnpc_bin_pk(C.byref(desc), C.byref(bins), band, npairs, pa, pb, nself, se,
                                  L.ptr(norms), L.ptr(means), L.ptr(selft), L.ptr(nmodes), L.ptr(keff),
                                  L.ptr(ws), ws.numel(), _sh(stream)))
    return means[:npairs], selft[:nself], nmodes, keff


def pk_multipole(bins, ell, mean, norms, stream=None):
    """(2l+1) mean / I22 - delta_l0 N0 for one shell-mean vector (device)."""
    out = _empty(bins.nbins, torch.float64)
    L.check(L.lib.cnpc_pk_multipole(C.byref(bins), int(ell), L.ptr(mean), L.ptr(norms), L.ptr(out),
                                    _sh(stream)))
    return out


def cross_norms(norms_a, norms_b, stream=None):
    """Normalisations of the cross multipoles of tracers A and B (device)."""
    out = _empty(L.NORMS_LEN, torch.float64)
    L.check(L.lib.cnpc_cross_norms(L.ptr(norms_a), L.ptr(norms_b), L.ptr(out), _sh(stream)))
    return out


def pk_finalize(bins, m, norms, stream=None):
    out = _empty((9, bins.nbins), torch.float64)
    g = lambda k: L.ptr(m.get(k))
    L.check(L.lib.cnpc_pk_finalize(C.byref(bins), g("00"), g("02"), g("04"), g("22"), g("42"),
                                   g("44"), L.ptr(norms), L.ptr(out), _sh(stream)))
    return out


PK_ROWS = ("P0", "P2", "P4", "P22", "P42", "P44", "P4b", "P6b", "P8b")


def measure_pk(desc, gpos, rpos, bins, ells=(0, 2, 4), modified=False, gw=None, rw=None,
               scratch: Optional[Scratch] = None, stream=None) -> Dict[str, torch.Tensor]:
    """Yamamoto P_l (and P_ll', P_4b, P_6b, P_8b when modified) of one catalog pair.
    Odd l in ells (1, 3) give the imaginary-part multipoles, with no shot noise."""
    sc = scratch or Scratch()
    norms, _, _ = catalog_norms(desc, gpos, rpos, gw, rw, sc, stream)
    delta, _ = paint(desc, gpos, rpos, norms, gw, rw, noise=False, scratch=sc, stream=stream)
    kmax = bins.kmin + bins.nbins * bins.dk
    band = L.lib.cnpc_band_for(C.byref(desc), kmax)
    hi = [l for l in ells if l > 0]
    need_real = len(hi) > 0
    D, dint = deinterlace(desc, band, delta, want_real=need_real, scratch=sc, stream=stream)
    del delta
    F = {0: assemble(desc, band, 0, spec0=D, stream=stream)}
    if hi:
        ylm = ylm_spectra(desc, band, hi, dint, sc, stream)
        for l in hi:
            F[l] = assemble(desc, band, l, ylm=ylm[l], stream=stream)
    odd = [l for l in ells if l % 2]
    ells = [l for l in ells if l % 2 == 0]
    pairs, keys = [], []
    for l in ells:
        pairs.append((F[0], F[l]))
        keys.append(f"0{l}")
    if modified:
        for (a, b) in ((2, 2), (4, 2), (4, 4)):
            pairs.append((F[a], F[b]))
            keys.append(f"{a}{b}")
    means, _, nmodes, keff = bin_means(desc, bins, band, pairs, (), norms, sc, stream)
    m = {k: means[i] for i, k in enumerate(keys)}
    out = pk_finalize(bins, m, norms, stream)
    res = {"norms": norms, "nmodes": nmodes, "k_eff": keff, "band": band}
    for i, k in enumerate(PK_ROWS):
        res[k] = out[i]
    if odd:
        # odd multipoles: the imaginary part of the same shell average
        mi, _, _, _ = bin_means(desc, bins, band, [(F[0], F[l]) for l in odd], (), norms, sc, stream, imag=True)
        for i, l in enumerate(odd):
            res[f"P{l}"] = pk_multipole(bins, l, mi[i], norms, stream)
    return res


def measure_pk_cross(desc, cat_a, cat_b, bins, ells=(0, 2, 4), scratch: Optional[Scratch] = None,
                     stream=None) -> Dict[str, torch.Tensor]:
    """Cross multipoles of two tracers A and B, each a (galaxies, randoms[,
    galaxy weights, random weights]) tuple: (2l+1)/I22^AB <F_0^A F_l^B*>, the
    real part for even l and the imaginary part for odd l, I22^AB = sqrt(I22^A
    I22^B), no shot noise."""
    sc = scratch or Scratch()
    kmax = bins.kmin + bins.nbins * bins.dk
    band = L.lib.cnpc_band_for(C.byref(desc), kmax)
    F = {}
    norms = {}
    for tag, cat, want in (("a", cat_a, (0,)), ("b", cat_b, tuple(ells))):
        g, r = cat[0], cat[1]
        gw = cat[2] if len(cat) > 2 else None
        rw = cat[3] if len(cat) > 3 else None
        nm, _, _ = catalog_norms(desc, g, r, gw, rw, sc, stream)
        delta, _ = paint(desc, g, r, nm, gw, rw, noise=False, scratch=sc, stream=stream)
        hi = [l for l in want if l > 0]
        D, dint = deinterlace(desc, band, delta, want_real=len(hi) > 0, scratch=sc, stream=stream)
        del delta
        F[(tag, 0)] = assemble(desc, band, 0, spec0=D, stream=stream)
        if hi:
            ylm = ylm_spectra(desc, band, hi, dint, sc, stream)
            for l in hi:
                F[(tag, l)] = assemble(desc, band, l, ylm=ylm[l], stream=stream)
        norms[tag] = nm
    nab = cross_norms(norms["a"], norms["b"], stream)
    res = {"norms": nab}
    for imag in (False, True):
        sel = [l for l in ells if (l % 2 == 1) == imag]
        if not sel:
            continue
        m, _, nmodes, keff = bin_means(desc, bins, band, [(F[("a", 0)], F[("b", l)]) for l in sel], (), nab,
                                       sc, stream, imag=imag)
        res["nmodes"], res["k_eff"] = nmodes, keff
        for i, l in enumerate(sel):
            res[f"P{l}"] = pk_multipole(bins, l, m[i], nab, stream)
    return res


_PLANS: Dict[tuple, "BispecPlan"] = {}


class BispecPlan:
    def __init__(self, desc, bins, estimator, ell, precision, scratch: Scratch, stream=None):
        self.desc, self.bins = desc, bins
        self.estimator, self.ell, self.precision = estimator, ell, precision
        self.ws_bytes = L.lib.cnpc_bispec_workspace_size(C.byref(desc), C.byref(bins), estimator, ell)
        ws = scratch.get(self.ws_bytes)
        h = C.c_void_p()
        L.check(L.lib.cnpc_bispec_plan_create(C.byref(h), C.byref(desc), C.byref(bins), estimator, ell,
                                              precision, L.ptr(ws), ws.numel(), _sh(stream)))
        self.handle = h
        self.nconf = L.lib.cnpc_bispec_nconfigs(h)
        self.band = L.lib.cnpc_bispec_band(h)
        self.grid = L.lib.cnpc_bispec_grid(h)
        ext = L.KBins()
        L.check(L.lib.cnpc_bispec_ext_bins(h, C.byref(ext)))
        self.ext = ext

    def indicators(self, scratch: Scratch, stream=None):
        """Shell indicator fields of a TripoSH plan (computed once, kept)."""
        if getattr(self, "_ind", None) is None:
            nbytes = L.lib.cnpc_bispec_indicator_bytes(self.handle)
            if nbytes == 0:
                raise ValueError("indicator fields belong to TripoSH plans")
            ind = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            ws = scratch.get(self.ws_bytes)
            L.check(L.lib.cnpc_bispec_indicators(self.handle, L.ptr(ind), L.ptr(ws), ws.numel(), _sh(stream)))
            torch.cuda.synchronize()  # read-only from here on, from any stream
            self._ind = ind
        return self._ind

    def configs(self):
        import numpy as np
        ijk = (C.c_int32 * (3 * self.nconf))()
        nt = (C.c_int64 * self.nconf)()
        L.check(L.lib.cnpc_bispec_configs(self.handle, ijk, nt))
        return (np.frombuffer(ijk, dtype=np.int32).reshape(-1, 3).copy(),
                np.frombuffer(nt, dtype=np.int64).copy())

    def __del__(self):
        h = getattr(self, "handle", None)
        lib = getattr(L, "lib", None) if L is not None else None  # None at interpreter exit
        if h is not None and h.value and lib is not None:
            lib.cnpc_bispec_plan_destroy(h)
            self.handle = None


def bispec_plan(desc, bins, estimator, ell, precision, scratch: Scratch, stream=None) -> BispecPlan:
    key = (bytes(desc), bytes(bins), estimator, ell, precision)
    if key not in _PLANS:
        _PLANS[key] = BispecPlan(desc, bins, estimator, ell, precision, scratch, stream)
    return _PLANS[key]


def measure_bk(desc, gpos, rpos, bins, estimator=L.EST_SCOCCIMARRO, ell=0, precision=None, gw=None,
               rw=None, scratch: Optional[Scratch] = None, stream=None, shot_noise=True, noise="analytic"):
    """Scoccimarro B_l or TripoSH B_l0l of one catalog pair, with analytic shot
    noise; noise="fft" (TripoSH) takes the i = j != k term by the FFT method."""
    sc = scratch or Scratch()
    method = noise
    if method not in ("analytic", "fft"):
        raise ValueError(f"unknown noise method {method!r}")
    if method == "fft" and (estimator != L.EST_TRIPOSH or not shot_noise):
        raise ValueError("the FFT-method shot noise is implemented for TripoSH with shot noise on")
    if precision is None:
        precision = L.PREC_F64 if desc.dtype == L.F64 else L.PREC_F32
    plan = bispec_plan(desc, bins, estimator, ell, precision, sc, stream)
    band = plan.band
    norms, _, _ = catalog_norms(desc, gpos, rpos, gw, rw, sc, stream)
    delta, nmesh = paint(desc, gpos, rpos, norms, gw, rw, noise=shot_noise, scratch=sc, stream=stream)
    D, dint = deinterlace(desc, band, delta, want_real=ell > 0, scratch=sc, stream=stream)
    del delta
    F0 = assemble(desc, band, 0, spec0=D, stream=stream)
    Fl = F0
    if ell > 0:
        ylm = ylm_spectra(desc, band, [ell], dint, sc, stream)
        Fl = assemble(desc, band, ell, ylm=ylm[ell], stream=stream)
    rows = None  # noise_means rows of cnpc_bispectrum
    if shot_noise:
        DN, nint = deinterlace(desc, band, nmesh, want_real=ell > 0, scratch=sc, stream=stream)
        FN0 = assemble(desc, band, 0, spec0=DN, stream=stream)
        FNl = FN0
        if ell > 0:
            ylmN = ylm_spectra(desc, band, [ell], nint, sc, stream)
            FNl = assemble(desc, band, ell, ylm=ylmN[ell], stream=stream)
        means, selft, _, _ = bin_means(desc, plan.ext, band, [(Fl, FN0), (F0, FNl)], (ell,), norms, sc,
                                       stream)
        rows = torch.cat([means, selft], 0).contiguous()
    raw = _empty(plan.nconf, torch.float64)
    shot = _empty(plan.nconf, torch.float64)
    val = _empty(plan.nconf, torch.float64)
    Fl_arg = Fl if (ell > 0 or estimator == L.EST_TRIPOSH) else None
    if method == "fft":
        ind = plan.indicators(sc, stream)
        ws = sc.get(plan.ws_bytes)
        L.check(L.lib.cnpc_bispectrum_fft_noise(plan.handle, L.ptr(F0), L.ptr(Fl_arg), L.ptr(FN0), L.ptr(ind),
                                                L.ptr(rows), L.ptr(norms), L.ptr(raw), L.ptr(shot),
                                                L.ptr(val), L.ptr(ws), ws.numel(), _sh(stream)))
    else:
        ws = sc.get(plan.ws_bytes)
        L.check(L.lib.cnpc_bispectrum(plan.handle, L.ptr(F0), L.ptr(Fl_arg), L.ptr(rows), L.ptr(norms),
                                      L.ptr(raw), L.ptr(shot), L.ptr(val), L.ptr(ws), ws.numel(),
                                      _sh(stream)))
    return {"raw": raw, "shot": shot, "value": val, "norms": norms, "plan": plan, "noise": rows}


class SugiPlan:
    """Plan of the Sugiyama B_l1l2L (cnpc_sugi_plan_create)."""

    def __init__(self, desc, bins, l1, l2, L_, precision):
        self.desc, self.bins = desc, bins
        self.l1, self.l2, self.L, self.precision = int(l1), int(l2), int(L_), precision
        h = C.c_void_p()
        L.check(L.lib.cnpc_sugi_plan_create(C.byref(h), C.byref(desc), C.byref(bins), self.l1, self.l2, self.L,
                                            precision))
        self.handle = h
        self.band = L.lib.cnpc_bispec_band(h)
        self.grid = L.lib.cnpc_bispec_grid(h)
        ext = L.KBins()
        L.check(L.lib.cnpc_bispec_ext_bins(h, C.byref(ext)))
        self.ext = ext
        self.ws_bytes = L.lib.cnpc_sugi_workspace_size(C.byref(desc), C.byref(bins))

    def __del__(self):
        h = getattr(self, "handle", None)
        lib = getattr(L, "lib", None) if L is not None else None  # None at interpreter exit
        if h is not None and h.value and lib is not None:
            lib.cnpc_bispec_plan_destroy(h)
            self.handle = None


def sugi_plan(desc, bins, l1, l2, L_, precision) -> SugiPlan:
    key = ("sugiyama", bytes(desc), bytes(bins), l1, l2, L_, precision)
    if key not in _PLANS:
        _PLANS[key] = SugiPlan(desc, bins, l1, l2, L_, precision)
    return _PLANS[key]


def measure_sugiyama(desc, gpos, rpos, bins, l1, l2, L_, precision=None, gw=None, rw=None,
                     scratch: Optional[Scratch] = None, stream=None, shot_noise=True, noise="analytic"):
    """Sugiyama B_l1l2L(k_i, k_j) for every pair of shells (nbins x nbins),
    with its analytic shot noise; noise="fft" takes the i = j != k term by the
    FFT method."""
    sc = scratch or Scratch()
    if noise not in ("analytic", "fft") or (noise == "fft" and not shot_noise):
        raise ValueError("noise must be 'analytic' or 'fft' (the latter with shot noise on)")
    method = noise
    if precision is None:
        precision = L.PREC_F64 if desc.dtype == L.F64 else L.PREC_F32
    plan = sugi_plan(desc, bins, l1, l2, L_, precision)
    band = plan.band
    norms, _, _ = catalog_norms(desc, gpos, rpos, gw, rw, sc, stream)
    delta, nmesh = paint(desc, gpos, rpos, norms, gw, rw, noise=shot_noise, scratch=sc, stream=stream)
    D, dint = deinterlace(desc, band, delta, want_real=L_ > 0, scratch=sc, stream=stream)
    del delta
    F0 = assemble(desc, band, 0, spec0=D, stream=stream)
    ylmL = ylm_spectra(desc, band, [L_], dint, sc, stream)[L_] if L_ > 0 else None
    rows = None
    if shot_noise:
        FL = assemble(desc, band, L_, ylm=ylmL, stream=stream) if L_ > 0 else F0
        DN, nint = deinterlace(desc, band, nmesh, want_real=L_ > 0, scratch=sc, stream=stream)
        FN0 = assemble(desc, band, 0, spec0=DN, stream=stream)
        FNL = FN0
        if L_ > 0:
            FNL = assemble(desc, band, L_, ylm=ylm_spectra(desc, band, [L_], nint, sc, stream)[L_], stream=stream)
        means, selft, _, _ = bin_means(desc, plan.ext, band, [(FL, FN0), (F0, FNL)], (L_,), norms, sc, stream)
        rows = torch.cat([means, selft], 0).contiguous()
    nb = bins.nbins
    raw = _empty((nb, nb), torch.float64)
    shot = _empty((nb, nb), torch.float64)
    val = _empty((nb, nb), torch.float64)
    ws = sc.get(plan.ws_bytes)
    if method == "fft":
        L.check(L.lib.cnpc_sugiyama_fft_noise(plan.handle, L.ptr(F0), L.ptr(ylmL), L.ptr(FN0), L.ptr(rows),
                                              L.ptr(norms), L.ptr(raw), L.ptr(shot), L.ptr(val), L.ptr(ws),
                                              ws.numel(), _sh(stream)))
    else:
        L.check(L.lib.cnpc_sugiyama(plan.handle, L.ptr(F0), L.ptr(ylmL), L.ptr(rows), L.ptr(norms), L.ptr(raw),
                                    L.ptr(shot), L.ptr(val), L.ptr(ws), ws.numel(), _sh(stream)))
    return {"raw": raw, "shot": shot, "value": val, "norms": norms, "plan": plan}


def measure_pk_bk(desc, gpos, rpos, bins, plan: "BispecPlan", ells=(0, 2, 4), gw=None, rw=None,
                  scratch: Optional[Scratch] = None, stream=None, out=None):
    """One catalog pair through the whole hot path: P_l (l in ells) and the
    Scoccimarro B_0 of `plan`, sharing the painting, the de-interlaced F_0 and
    the shot-noise spectra.  `out` (optional): dict of preallocated result
    tensors to write into ("pk": [9, nbins], "bk": [3, nconf])."""
    sc = scratch or Scratch()
    if any(l > 0 for l in ells) and fold_fused_supported(desc):
        norms, D, dint, DN, _, _ = paint_deinterlace(desc, plan.band, gpos, rpos, gw, rw,
                                                     sums_lmax=_pk_bk_lmax(plan), scratch=sc, stream=stream)
        return _spectra_stage(desc, bins, plan, (norms, None, None), ells, sc, stream, out,
                              deinterlaced=(D, dint, DN))
    painted = paint_fkp(desc, gpos, rpos, gw, rw, noise=True, sums_lmax=_pk_bk_lmax(plan), scratch=sc,
                        stream=stream)
    return _spectra_stage(desc, bins, plan, painted, ells, sc, stream, out)


def _pk_bk_lmax(plan) -> int:
    # the B_0 shot noise and P_l need only the l = 0 catalog sums
    return 0 if plan.ell == 0 else 4


def _spectra_stage(desc, bins, plan, painted, ells, sc: Scratch, stream, out, deinterlaced=None):
    """Everything of measure_pk_bk after the painting (after the de-interlacing
    too when `deinterlaced` = (D, delta_int, DN) is given)."""
    norms, delta, nmesh = painted[0], painted[1], painted[2]
    band = plan.band
    hi = [l for l in ells if l > 0]
    if deinterlaced is not None:
        D, dint, DN = deinterlaced
    else:
        D, dint = deinterlace(desc, band, delta, want_real=len(hi) > 0, scratch=sc, stream=stream)
        DN, _ = deinterlace(desc, band, nmesh, want_real=False, scratch=sc, stream=stream)
    F = {0: assemble(desc, band, 0, spec0=D, stream=stream)}
    FN0 = assemble(desc, band, 0, spec0=DN, stream=stream)
    if hi:
        ylm = ylm_spectra(desc, band, hi, dint, sc, stream)
        for l in hi:
            F[l] = assemble(desc, band, l, ylm=ylm[l], stream=stream)
    pairs = [(F[0], F[l]) for l in ells] + [(F[0], FN0)]
    means, selft, nmodes, keff = bin_means(desc, bins, band, pairs, (0,), norms, sc, stream)
    m = {f"0{l}": means[i] for i, l in enumerate(ells)}
    pk = pk_finalize(bins, m, norms, stream)
    q = means[len(ells)]
    noise = torch.stack([q, q, selft[0]], 0).contiguous()
    res = out if out is not None else {
        "pk": _empty((9, bins.nbins), torch.float64),
        "bk": _empty((3, plan.nconf), torch.float64)}
    res["pk"].copy_(pk)
    ws = sc.get(plan.ws_bytes)
    bk = res["bk"]
    L.check(L.lib.cnpc_bispectrum(plan.handle, L.ptr(F[0]), None, L.ptr(noise), L.ptr(norms),
                                  L.ptr(bk[0]), L.ptr(bk[1]), L.ptr(bk[2]), L.ptr(ws), ws.numel(),
                                  _sh(stream)))
    res["nmodes"] = nmodes
    return res


class NativeBatch:
    """The library's own batch (cnpc_batch_*): measure_pk_bk for many catalog
    pairs, round-robin over `nstreams` streams owned by the library, each with
    its slab of one workspace; run() enqueues eagerly, capture() records the
    same work into a HIP graph held by the library and replay() launches it.
    The captured graph keeps the catalog, output and workspace addresses, so
    this object holds references to them."""

    def __init__(self, desc, bins, plan: "BispecPlan", ells=(0, 2, 4), nstreams: int = 4,
                 max_ngal: int = 1, max_nran: int = 1, device="cuda"):
        ells = [int(l) for l in ells]
        h = C.c_void_p()
        arr = (C.c_int32 * len(ells))(*ells)
        L.check(L.lib.cnpc_batch_create(C.byref(h), C.byref(desc), C.byref(bins), plan.handle, len(ells), arr,
                                        int(nstreams), int(max_ngal), int(max_nran)))
        self.handle = h
        self.plan = plan  # the library keeps a pointer to it
        self.nstreams = int(nstreams)
        self.ws = torch.empty(max(256, L.lib.cnpc_batch_workspace_size(h)), dtype=torch.uint8, device=device)
        self._held = None

    def _args(self, catalogs, outs):
        n = len(catalogs)
        if n != len(outs) or n == 0:
            raise ValueError("need one output dict per catalog and at least one catalog")
        P = C.c_void_p * n
        I = C.c_int64 * n
        weighted = any(len(c) > 2 and c[2] is not None for c in catalogs)
        gw = P(*[L.ptr(c[2]) if len(c) > 2 else None for c in catalogs]) if weighted else None
        rw = P(*[L.ptr(c[3]) if len(c) > 3 else None for c in catalogs]) if weighted else None
        return (n, P(*[L.ptr(c[0]) for c in catalogs]), gw, I(*[int(c[0].shape[1]) for c in catalogs]),
                P(*[L.ptr(c[1]) for c in catalogs]), rw, I(*[int(c[1].shape[1]) for c in catalogs]),
                P(*[L.ptr(o["pk"]) for o in outs]), P(*[L.ptr(o["bk"]) for o in outs]))

    def run(self, catalogs, outs, stream=None):
        a = self._args(catalogs, outs)
        L.check(L.lib.cnpc_batch_run(self.handle, *a, L.ptr(self.ws), self.ws.numel(), _sh(stream)))

    def capture(self, catalogs, outs):
        a = self._args(catalogs, outs)
        L.check(L.lib.cnpc_batch_capture(self.handle, *a, L.ptr(self.ws), self.ws.numel()))
        self._held = (list(catalogs), list(outs))

    def replay(self, stream=None):
        L.check(L.lib.cnpc_batch_replay(self.handle, _sh(stream)))

    def __del__(self):
        h = getattr(self, "handle", None)
        lib = getattr(L, "lib", None) if L is not None else None  # None at interpreter exit
        if h is not None and h.value and lib is not None:
            lib.cnpc_batch_destroy(h)
            self.handle = None


def balanced_assignment(sizes: Sequence[int], nstreams: int, mixed: bool = False):
    """Longest-first greedy placement: items by decreasing size (ties: index),
    each on the stream with the smallest total so far (ties: lowest stream).
    Returns (item, stream) pairs in launch order: placement order, or with
    mixed=True the streams' lists interleaved with odd streams reversed
    (smallest first), so that streams running side by side hold catalogs of
    different sizes."""
    load = [0] * nstreams
    out = []
    for i in sorted(range(len(sizes)), key=lambda c: (-sizes[c], c)):
        k = min(range(nstreams), key=lambda q: (load[q], q))
        load[k] += sizes[i]
        out.append((i, k))
    if not mixed:
        return out
    lists = [[i for i, q in out if q == k] for k in range(nstreams)]
    for k in range(1, nstreams, 2):
        lists[k].reverse()
    mixed_out = []
    for step in range(max((len(x) for x in lists), default=0)):
        for k in range(nstreams):
            if step < len(lists[k]):
                mixed_out.append((lists[k][step], k))
    return mixed_out


class Batch:
    """Many catalog pairs through measure_pk_bk: the catalogs are spread over
    `nstreams` streams (each with its own scratch), so that the small and the
    tail-end kernels of one catalog overlap the work of another; `balance`
    picks the placement ("rr" round-robin, "lpt" or "mixed" by particle count,
    see assignment).  The caller's current stream is forked at the start and
    joined at the end, so the batch can be captured into one graph."""

    def __init__(self, nstreams: int = 2, device="cuda", balance: str = "rr"):
        self.device = device
        self.balance = balance
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, nstreams))]
        self.scratch = [Scratch(device) for _ in self.streams]

    def assignment(self, catalogs):
        """(catalog, stream) pairs in launch order.  balance "rr": catalog i
        on stream i mod nstreams; "lpt": by decreasing particle count, each on
        the stream with the fewest particles so far; "mixed": the same
        placement with odd streams running their catalogs smallest first."""
        ns = len(self.streams)
        if self.balance == "rr":
            return [(i, i % ns) for i in range(len(catalogs))]
        return balanced_assignment([int(g.shape[1]) + int(r.shape[1]) for g, r in catalogs], ns,
                                   mixed=self.balance == "mixed")

    def run_stream(self, k, desc, catalogs, bins, plan, outs, ells=(0, 2, 4)):
        """The catalogs that the placement puts on stream k, on the caller's
        current stream (used to capture one single-stream graph per stream)."""
        for i, q in self.assignment(catalogs):
            if q == k:
                measure_pk_bk(desc, catalogs[i][0], catalogs[i][1], bins, plan, ells=ells,
                              scratch=self.scratch[k], out=outs[i])

    def run(self, desc, catalogs, bins, plan, outs, ells=(0, 2, 4)):
        cur = torch.cuda.current_stream()
        for s in self.streams:
            s.wait_stream(cur)
        for i, k in self.assignment(catalogs):
            (g, r), o = catalogs[i], outs[i]
            with torch.cuda.stream(self.streams[k]):
                measure_pk_bk(desc, g, r, bins, plan, ells=ells, scratch=self.scratch[k], out=o)
        for s in self.streams:
            cur.wait_stream(s)
