"""Odd Yamamoto multipoles and two-tracer cross multipoles against the FP64
oracle, through the C ABI.

The odd multipoles P_1 and P_3 are the imaginary part of the same shell mean
of F_0 F_l^* that gives the even ones (the real part vanishes for odd l), with
no shot-noise term.  The cross multipoles of tracers A and B use F_0 of A and
F_l of B, normalised by sqrt(I22^A I22^B), with no shot noise.  Bars as in
the other parity tests: FP64 within 1e-10 of the largest magnitude, FP32
within 3e-5 (the odd multipoles are a few per cent of the monopole, so the
relative bar is against their own scale), mode counts bit-exact.
"""

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
from oracle.pipeline import MeshConfig, measure_pk, measure_pk_cross  # noqa: E402
import test_gpu_parity as P  # noqa: E402

TOL = {L.F64: 1e-10, L.F32: 3e-5}


def _bins(n, box, dk=0.01):
    nb = int((math.pi * n / box) // dk) - 1
    return nb, cn.kbins(0.0, dk, nb)


@pytest.mark.parametrize("dtype", [L.F64, L.F32])
@pytest.mark.parametrize("n,assign,interlace", [(32, L.CIC, False), (64, L.TSC, True)])
def test_odd_multipoles_vs_oracle(n, assign, interlace, dtype):
    box = 1000.0
    g, r = P._cat(200 + n, 40_000, 200_000)
    nb, bins = _bins(n, box)
    d = cn.mesh_desc(n, box, assign=assign, interlace=interlace, dtype=dtype, observer=P.OBS)
    ells = (0, 1, 2, 3, 4)
    res = pl.measure_pk(d, P.dev(g), P.dev(r), bins, ells=ells)
    cfg = MeshConfig(box, n, assign, interlace, P.OBS)
    ora = measure_pk(g, None, r, None, cfg, 0.0, 0.01, nb, ells=ells)
    assert np.array_equal(P.host(res["nmodes"]), ora["nmodes"])
    for key in ("P0", "P1", "P2", "P3", "P4"):
        assert P.rel(P.host(res[key]), ora[key]) < TOL[dtype], key


def test_odd_multipoles_weighted_fp64():
    n, box = 32, 1000.0
    g, r = P._cat(301, 30_000, 150_000)
    rng = np.random.default_rng(302)
    gw = rng.uniform(0.5, 1.5, g.shape[-1]).astype(np.float32)
    rw = rng.uniform(0.5, 1.5, r.shape[-1]).astype(np.float32)
    nb, bins = _bins(n, box)
    d = cn.mesh_desc(n, box, assign=L.TSC, interlace=False, dtype=L.F64, observer=P.OBS)
    res = pl.measure_pk(d, P.dev(g), P.dev(r), bins, ells=(0, 1, 3), gw=P.dev(gw), rw=P.dev(rw))
    cfg = MeshConfig(box, n, L.TSC, False, P.OBS)
    ora = measure_pk(g, gw, r, rw, cfg, 0.0, 0.01, nb, ells=(0, 1, 3))
    for key in ("P0", "P1", "P3"):
        assert P.rel(P.host(res[key]), ora[key]) < 1e-10, key


@pytest.mark.parametrize("dtype", [L.F64, L.F32])
@pytest.mark.parametrize("n,assign,interlace", [(32, L.TSC, False), (64, L.TSC, True)])
def test_cross_multipoles_vs_oracle(n, assign, interlace, dtype):
    box = 1000.0
    gA, rA = P._cat(400 + n, 30_000, 150_000)
    gB, rB = P._cat(500 + n, 20_000, 120_000)
    nb, bins = _bins(n, box)
    d = cn.mesh_desc(n, box, assign=assign, interlace=interlace, dtype=dtype, observer=P.OBS)
    ells = (0, 1, 2, 3, 4)
    res = pl.measure_pk_cross(d, (P.dev(gA), P.dev(rA)), (P.dev(gB), P.dev(rB)), bins, ells=ells)
    cfg = MeshConfig(box, n, assign, interlace, P.OBS)
    ora = measure_pk_cross(gA, None, rA, None, gB, None, rB, None, cfg, 0.0, 0.01, nb, ells=ells)
    assert np.array_equal(P.host(res["nmodes"]), ora["nmodes"])
    assert abs(float(P.host(res["norms"])[2]) - ora["I22"]) <= 1e-12 * ora["I22"]
    for l in ells:
        key = f"P{l}"
        assert P.rel(P.host(res[key]), ora[key]) < TOL[dtype], key


def test_cross_of_a_tracer_with_itself_is_its_auto_spectrum_without_noise():
    """A x A equals the auto multipoles before the shot-noise subtraction."""
    n, box = 32, 1000.0
    g, r = P._cat(601, 30_000, 150_000)
    nb, bins = _bins(n, box)
    d = cn.mesh_desc(n, box, assign=L.CIC, interlace=True, dtype=L.F64, observer=P.OBS)
    gd, rd = P.dev(g), P.dev(r)
    auto = pl.measure_pk(d, gd, rd, bins, ells=(0, 1, 2))
    cross = pl.measure_pk_cross(d, (gd, rd), (gd, rd), bins, ells=(0, 1, 2))
    n0 = float(P.host(auto["norms"])[4])
    assert n0 > 0
    assert P.rel(P.host(cross["P0"]), P.host(auto["P0"]) + n0) < 1e-10
    for key in ("P1", "P2"):
        assert P.rel(P.host(cross[key]), P.host(auto[key])) < 1e-10, key
