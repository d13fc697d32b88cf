"""GPU runs of the global line of sight (CNPC_LOS_GLOBAL) against the oracle's
exact pins (section on modified high-order multipoles, eqs. Hand17, legendre and
Plnew), and of the bin edges that fall exactly on integer |n|.

* A fixed-amplitude Kaiser mesh through deinterlace, the Y_lm transforms, the
  F_l assembly and the binning gives the discrete expectation
  (2l+1) <L_l(mu) P(k) (b + f mu^2)^2>_b exactly.
* With a global line of sight P_4b, P_6b and P_8b equal the traditional P_4, P_6
  and P_8 (the Legendre re-expansion is exact and the printed N_ll' make the
  shot terms cancel), and the odd multipoles vanish.
* Half-open bins whose edges sit on integer |n| (reading R6) count every mode of
  an edge in the upper bin, bit-exact against integer enumeration.
"""

import ctypes
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # the marker deselects these on CPU runs
    pytest.skip("no GPU", allow_module_level=True)

import paper_2605_04864_amd as cn  # noqa: E402
from paper_2605_04864_amd import _lib as L  # noqa: E402
from paper_2605_04864_amd import pipeline as pl  # noqa: E402
from oracle import mesh as oms  # noqa: E402
from oracle import spectra as osp  # noqa: E402
from oracle.ylm import legendre  # noqa: E402
from oracle.pipeline import MeshConfig, measure_pk  # noqa: E402
import synthcat  # noqa: E402

TOL = {L.F64: 1e-10, L.F32: 1e-5}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("dtype", [L.F64, L.F32])
def test_kaiser_fixed_amplitude_mesh(dtype):
    n, box, nb, dk = 64, 1000.0, 20, 0.01
    los = np.array([0.0, 0.0, 1.0])
    delta = synthcat.fixed_amplitude_mesh(n, box, seed=11, los=los)
    # the library divides every assembled spectrum by the TSC window: hand it the
    # mesh whose spectrum is W(k) delta(k), so that F_0 = delta(k) exactly
    W = oms.compensation(n, oms.TSC)
    pre = np.fft.ifftn(np.fft.fftn(delta) * W).real
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=False, dtype=dtype, los=los)
    tdt = torch.float64 if dtype == L.F64 else torch.float32
    mesh = torch.from_numpy(pre[None]).to(tdt).cuda()
    bins = cn.kbins(0.0, dk, nb)
    band = L.lib.cnpc_band_for(ctypes.byref(d), nb * dk)
    sc = pl.Scratch()
    D, real = pl.deinterlace(d, band, mesh, want_real=True, scratch=sc)
    ylm = pl.ylm_spectra(d, band, (2, 4), real, sc)
    F = {0: pl.assemble(d, band, 0, spec0=D), 2: pl.assemble(d, band, 2, ylm=ylm[2]),
         4: pl.assemble(d, band, 4, ylm=ylm[4])}
    norms = torch.zeros(L.NORMS_LEN, dtype=torch.float64, device="cuda")
    means, _, nmodes, _ = pl.bin_means(d, bins, band, [(F[0], F[0]), (F[0], F[2]), (F[0], F[4])],
                                       (), norms, sc)
    I22 = n ** 6 / box ** 3
    ob = osp.Bins(0.0, dk, nb, box, n)
    assert np.array_equal(host(nmodes), ob.counts())
    kvec = osp.kvectors(n, box)
    kk = np.linalg.norm(kvec, axis=-1)
    with np.errstate(invalid="ignore", divide="ignore"):
        mu = np.where(kk > 0, kvec[..., 2] / np.where(kk > 0, kk, 1), 0.0)
    pk = synthcat.field_power(kk) * (2.0 + 0.8 * mu * mu) ** 2
    m = host(means)
    for row, ell in enumerate((0, 2, 4)):
        got = (2 * ell + 1) / I22 * m[row]
        expect = (2 * ell + 1) * ob.shell_mean(legendre(ell, mu) * pk)
        assert rel(got, expect) < TOL[dtype], ell


@pytest.mark.parametrize("dtype", [L.F64, L.F32])
def test_global_los_modified_equals_traditional(dtype):
    n, box, nb, dk = 64, 1000.0, 19, 0.01
    los = np.array([0.3, -0.5, 0.81])
    los /= np.linalg.norm(los)
    g = synthcat.lognormal_catalog(40_000, box, 131)
    r = synthcat.random_catalog(200_000, 132)
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=dtype, los=los)
    res = pl.measure_pk(d, torch.from_numpy(g).cuda(), torch.from_numpy(r).cuda(), cn.kbins(0.0, dk, nb),
                        ells=(0, 2, 4), modified=True)
    cfg = MeshConfig(box, n, oms.TSC, True, synthcat.observer_position(), los=los)
    ora = measure_pk(g, None, r, None, cfg, 0.0, dk, nb, ells=(0, 2, 4, 6, 8))
    assert np.array_equal(host(res["nmodes"]), ora["nmodes"])
    for key in ("P0", "P2", "P4"):
        assert rel(host(res[key]), ora[key]) < TOL[dtype], key
    scale = max(np.max(np.abs(ora[f"P{l}"])) for l in (0, 2, 4, 6, 8))
    # P_lb from l <= 4 fields against the oracle's traditional P_l from l = 6, 8 fields
    for got, ref in (("P4b", "P4"), ("P6b", "P6"), ("P8b", "P8")):
        err = np.max(np.abs(host(res[got]) - ora[ref])) / scale
        assert err < TOL[dtype], (got, err)


@pytest.mark.parametrize("dtype", [L.F64, L.F32])
def test_global_los_odd_multipoles_vanish(dtype):
    n, box, nb, dk = 32, 1000.0, 9, 0.01
    los = np.array([0.6, 0.0, 0.8])
    g = synthcat.lognormal_catalog(20_000, box, 61)
    r = synthcat.random_catalog(100_000, 62)
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=dtype, los=los)
    res = pl.measure_pk(d, torch.from_numpy(g).cuda(), torch.from_numpy(r).cuda(), cn.kbins(0.0, dk, nb),
                        ells=(0, 1, 2, 3, 4))
    scale = np.max(np.abs(host(res["P2"])))
    assert scale > 0
    for key in ("P1", "P3"):
        assert np.max(np.abs(host(res[key]))) < 10 * TOL[dtype] * scale, key
    # the local line of sight gives non-zero odd multipoles on the same catalog
    dl = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=dtype, observer=synthcat.observer_position())
    loc = pl.measure_pk(dl, torch.from_numpy(g).cuda(), torch.from_numpy(r).cuda(), cn.kbins(0.0, dk, nb),
                        ells=(0, 1, 2))
    assert np.max(np.abs(host(loc["P1"]))) > 1e3 * TOL[dtype] * scale


def _lattice_counts(nmesh, lo2, hi2):
    h = nmesh // 2
    r = np.arange(-h + 1, h)
    n2 = r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2
    return int(np.count_nonzero((n2 >= lo2) & (n2 < hi2) & (n2 > 0)))


@pytest.mark.parametrize("kmin_f,dk_f,nb", [(0, 1, 30), (3, 2, 14)])
def test_mode_counts_on_integer_edges(kmin_f, dk_f, nb):
    n, box = 64, 1000.0
    kf = 2 * math.pi / box
    g = synthcat.lognormal_catalog(20_000, box, 71)
    r = synthcat.random_catalog(100_000, 72)
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=True, dtype=L.F32, observer=synthcat.observer_position())
    res = pl.measure_pk(d, torch.from_numpy(g).cuda(), torch.from_numpy(r).cuda(),
                        cn.kbins(kmin_f * kf, dk_f * kf, nb), ells=(0,))
    got = host(res["nmodes"])
    ref = [_lattice_counts(n, (kmin_f + b * dk_f) ** 2, (kmin_f + (b + 1) * dk_f) ** 2) for b in range(nb)]
    assert list(got) == ref
    assert np.array_equal(got, osp.Bins(kmin_f * kf, dk_f * kf, nb, box, n).counts())
