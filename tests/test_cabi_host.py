"""Host-side checks of the C ABI (no GPU needed).

* the shared library loads and exports every function the header declares;
* argument validation rejects bad descriptors, bins and sizes on the host,
  before anything is launched, with a message in cnpc_last_error().
"""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cnpc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cnpc_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    from paper_2605_04864_amd import _lib as L
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L.lib, n)]
    assert not missing, missing
    assert set(names) == set(L.EXPORTED)


def test_version_and_empty_error():
    from paper_2605_04864_amd import _lib as L
    assert b"gfx950" in L.lib.cnpc_version()


def _desc(**kw):
    from paper_2605_04864_amd import _lib as L
    d = L.mesh_desc(kw.get("n", 64), kw.get("box", 1000.0), assign=kw.get("assign", L.TSC),
                    interlace=kw.get("interlace", True), dtype=kw.get("dtype", L.F32),
                    observer=kw.get("observer"), los=kw.get("los"))
    return d


@pytest.mark.parametrize("kw,msg", [
    ({"n": 100}, "power of two"),
    ({"n": 8}, "power of two"),
    ({"n": 2048}, "power of two"),
    ({"assign": 4}, "assign"),
    ({"dtype": 7}, "dtype"),
    ({"box": -1.0}, "boxsize"),
    ({"observer": (10.0, 10.0, 10.0)}, "outside"),
    ({"los": (0.0, 0.0, 2.0)}, "unit vector"),
])
def test_descriptor_validation(kw, msg):
    from paper_2605_04864_amd import _lib as L
    d = _desc(**kw)
    st = L.lib.cnpc_fft_r2c(C.byref(d), 1, 0, C.c_void_p(16), C.c_void_p(32), None, 0, None)
    assert st == -1
    assert msg in L.last_error()


def test_bins_and_band_validation():
    from paper_2605_04864_amd import _lib as L
    d = _desc(n=64, box=1000.0)
    b = L.kbins(0.0, 0.05, 10)  # top edge 0.5 > k_N = 0.201
    st = L.lib.cnpc_bin_pk(C.byref(d), C.byref(b), 32, 0, None, None, 0, None, None, None, None,
                           C.c_void_p(64), None, C.c_void_p(64), 1 << 20, None)
    assert st == -1 and "Nyquist" in L.last_error()
    b = L.kbins(0.0, 0.01, 20)
    st = L.lib.cnpc_bin_pk(C.byref(d), C.byref(b), 8, 0, None, None, 0, None, None, None, None,
                           C.c_void_p(64), None, C.c_void_p(64), 1 << 20, None)
    assert st == -1 and "does not cover" in L.last_error()
    st = L.lib.cnpc_fft_r2c(C.byref(d), 1, 12, C.c_void_p(16), C.c_void_p(32), None, 0, None)
    assert st == -1 and "band" in L.last_error()
    assert L.lib.cnpc_band_for(C.byref(d), 0.2) == 32


def test_paint_and_bispec_validation():
    from paper_2605_04864_amd import _lib as L
    d = _desc(n=64, box=1000.0)
    st = L.lib.cnpc_paint(C.byref(d), C.c_void_p(16), None, 0, C.c_void_p(16), None, 10,
                          C.c_void_p(16), C.c_void_p(16), None, C.c_void_p(16), 1 << 30, None)
    assert st == -1 and "ngal" in L.last_error()
    st = L.lib.cnpc_paint(C.byref(d), C.c_void_p(16), C.c_void_p(16), 10, C.c_void_p(16), None, 10,
                          C.c_void_p(16), C.c_void_p(16), None, C.c_void_p(16), 1 << 30, None)
    assert st == -1 and "weights" in L.last_error()
    h = C.c_void_p()
    b = L.kbins(0.01, 0.01, 5)
    st = L.lib.cnpc_bispec_plan_create(C.byref(h), C.byref(d), C.byref(b), L.EST_SCOCCIMARRO, 0,
                                       L.PREC_F32, C.c_void_p(16), 1 << 20, None)
    assert st == -1 and "k = 0" in L.last_error()
    b = L.kbins(0.0, 0.01, 5)
    st = L.lib.cnpc_bispec_plan_create(C.byref(h), C.byref(d), C.byref(b), L.EST_SCOCCIMARRO, 0,
                                       L.PREC_F64, C.c_void_p(16), 1 << 20, None)
    assert st == -1 and "FP64" in L.last_error()
    assert L.lib.cnpc_paint_workspace_size(C.byref(d), 1000, 10000) > 0
    assert L.lib.cnpc_bispec_workspace_size(C.byref(d), C.byref(b), 0, 0) > 0


def test_tuning_knobs_validation():
    from paper_2605_04864_amd import _lib as L
    try:
        for name, (idx, values) in L.TUNE.items():
            for v in values:
                assert L.lib.cnpc_tune_set(idx, v) == 0, (name, v)
                assert L.lib.cnpc_tune_get(idx) == v
            for bad in (-1, 3, 128):
                if bad in values:
                    continue
                assert L.lib.cnpc_tune_set(idx, bad) == -1, (name, bad)
                assert "out of range" in L.last_error()
                assert L.lib.cnpc_tune_get(idx) == values[-1]  # rejected values change nothing
        assert L.lib.cnpc_tune_set(len(L.TUNE), 0) == -1 and "unknown tuning knob" in L.last_error()
        assert L.lib.cnpc_tune_get(len(L.TUNE)) == -1
        assert L.lib.cnpc_tune_get(-1) == -1
    finally:
        for idx, _ in L.TUNE.values():
            L.lib.cnpc_tune_set(idx, 0)


def test_autotune_coordinate_descent():
    from paper_2605_04864_amd.autotune import coordinate_descent
    # separable cost with a known optimum; start elsewhere
    opt = {"a": 3, "b": 1, "c": 2}
    cost = lambda s: 10.0 + sum((s[k] - opt[k]) ** 2 for k in opt)
    calls = []

    def measure(s):
        calls.append(dict(s))
        return cost(s)

    space = {"a": [0, 1, 2, 3, 4], "b": [0, 1], "c": [0, 1, 2]}
    best, t, trials = coordinate_descent(space, {"a": 0, "b": 0, "c": 0}, measure)
    assert best == opt and t == 10.0
    # one sweep: the start, then every value not equal to the incumbent
    assert len(calls) == 1 + 4 + 1 + 2 and len(trials) == len(calls)
    # gains below min_gain keep the incumbent
    flat = lambda s: 100.0 - 0.5 * s["a"]
    best, _, _ = coordinate_descent({"a": [0, 1]}, {"a": 0}, flat, min_gain=0.01)
    assert best == {"a": 0}


def test_autotune_cache_roundtrip(tmp_path):
    from paper_2605_04864_amd import autotune as at
    path = str(tmp_path / "sub" / "tune.json")
    assert at._cache_load(path) == {"version": 1, "entries": {}}
    e1 = {"streams": 3,
          "knobs": {"fft_passes": 0, "fft_col_w": 8, "contract_kg": 2, "sort_per": 4, "sort_threads": 0},
          "ms": 1.5, "default_ms": 2.0}
    at._cache_store(path, "sig1", e1)
    at._cache_store(path, "sig2", dict(e1, streams=1))
    d = at._cache_load(path)
    assert d["entries"]["sig1"] == e1 and d["entries"]["sig2"]["streams"] == 1
    with open(path, "w") as f:
        f.write("{not json")
    assert at._cache_load(path)["entries"] == {}


def test_balanced_stream_assignment():
    from paper_2605_04864_amd.pipeline import balanced_assignment
    import numpy as np
    sizes = [int(x) for x in np.random.default_rng(3).integers(1_000_000, 8_000_000, 64)]
    asg = balanced_assignment(sizes, 4)
    assert sorted(i for i, _ in asg) == list(range(64))          # every catalog placed once
    assert [sizes[i] for i, _ in asg] == sorted(sizes, reverse=True)  # largest first
    load = [0] * 4
    for i, k in asg:
        load[k] += sizes[i]
    assert max(load) - min(load) <= max(sizes)                    # greedy bound
    assert (max(load) - min(load)) / (sum(load) / 4) < 0.02
    assert balanced_assignment([5, 5, 5], 2) == [(0, 0), (1, 1), (2, 0)]  # deterministic ties
    assert balanced_assignment([], 3) == []
    mix = balanced_assignment(sizes, 4, mixed=True)
    assert sorted(mix) == sorted(asg)                               # same placement
    for k in range(4):
        seq = [sizes[i] for i, q in mix if q == k]
        assert seq == sorted(seq, reverse=(k % 2 == 0))             # odd streams smallest first


def test_tripolar_real_coeffs_match_oracle():
    """Host utilities of the library against the oracle and the paper's counts."""
    import ctypes as C
    import numpy as np
    from paper_2605_04864_amd import _lib as L
    from oracle import sugiyama as sg
    for (l1, l2, Lm), nz_paper, paired_paper in (((1, 1, 2), 11, 5), ((2, 2, 2), 25, 10), ((2, 2, 4), 37, 13)):
        n = (2 * l1 + 1) * (2 * l2 + 1) * (2 * Lm + 1)
        buf = (C.c_double * n)()
        nz = C.c_int32()
        L.check(L.lib.cnpc_tripolar_real_coeffs(l1, l2, Lm, buf, C.byref(nz)))
        ref = sg.tripolar_real_coeffs(l1, l2, Lm).real.reshape(-1)
        assert np.max(np.abs(np.frombuffer(buf, dtype=np.float64) - ref)) < 1e-13
        assert nz.value == nz_paper
        assert L.lib.cnpc_sugi_paired_count(l1, l2, Lm) == paired_paper
    assert L.lib.cnpc_tripolar_real_coeffs(1, 1, 1, None, None) == -1  # odd l1 + l2 + L
    assert L.lib.cnpc_tripolar_real_coeffs(2, 2, 5, None, None) == -1  # triangle rule


def test_bin_pk_noalloc_rejects_binning_beyond_static_scratch():
    """The allocation-free bin_pk holds accumulators for at most 128 bins x (16
    products + 4 self terms + 1); a larger binning is refused on the host."""
    from paper_2605_04864_amd import _lib as L
    d = L.mesh_desc(256, 1000.0, assign=L.TSC, interlace=True, dtype=L.F32)
    b = L.kbins(0.0, 0.001, 129)
    st = L.lib.cnpc_bin_pk_noalloc(C.byref(d), C.byref(b), 128, 16, None, None, 4, None, None, None, None,
                                   None, None, None)
    assert st != 0
    assert "static scratch" in L.last_error()


def test_paint_deinterlace_rejects_other_meshes():
    """The painting with fused de-interlacing covers interlaced 256^3 meshes; a
    64^3 or non-interlaced mesh is refused on the host with CNPC_EUNSUPPORTED."""
    from paper_2605_04864_amd import _lib as L
    p = C.c_void_p(16)
    for n, il in ((64, True), (256, False)):
        d = L.mesh_desc(n, 1000.0, assign=L.TSC, interlace=il, dtype=L.F32)
        st = L.lib.cnpc_paint_deinterlace(C.byref(d), 16, p, None, 10, p, None, 100, 4, None, None, p, p, p, p,
                                          p, 1 << 30, None)
        assert st == -4, (n, il, st)
        assert "256^3" in L.last_error()
