"""ctypes binding of libcnpc.so (argument marshalling only).

Every compute step runs inside the HIP library; this module converts torch
tensors to device pointers, torch streams to hipStream_t handles and status
codes to exceptions.  It raises at import time if the library is missing.
"""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcnpc.so")

F32, F64 = 0, 1
CIC, TSC = 2, 3
LOS_LOCAL, LOS_GLOBAL = 0, 1
PREC_F64, PREC_F32, PREC_BF16X3 = 0, 1, 2
EST_SCOCCIMARRO, EST_TRIPOSH, EST_SUGIYAMA = 0, 1, 2
NYLM_SUMS = 9
SUMS_LEN = 3 + 2 * NYLM_SUMS
NORMS_LEN = 6 + 2 * NYLM_SUMS
NORM_ALPHA, NORM_NBAR, NORM_I22, NORM_I33, NORM_N0, NORM_SBAR, NORM_SBARLM = range(7)


class MeshDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("assign", C.c_int32), ("interlace", C.c_int32),
                ("dtype", C.c_int32), ("los_mode", C.c_int32), ("reserved", C.c_int32),
                ("boxsize", C.c_double), ("observer", C.c_double * 3), ("los", C.c_double * 3)]


class KBins(C.Structure):
    _fields_ = [("kmin", C.c_double), ("dk", C.c_double), ("nbins", C.c_int32),
                ("reserved", C.c_int32)]


class CnpcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cnpc status {status}: {msg}")
        self.status = status


def _load():
    # torch first: its HIP runtime is then the one the library binds to, whatever
    # the caller imported first (two runtimes in one process do not see the GPU)
    import torch  # noqa: F401
    # CNPC_LIBRARY selects another build of the library (e.g. to compare two builds)
    path = os.environ.get("CNPC_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with python -m paper_2605_04864_amd.build")
    return C.CDLL(path)


lib = _load()

_vp, _cvp, _i32, _i64, _sz, _d = C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
_PD = C.POINTER(MeshDesc)
_PB = C.POINTER(KBins)

_PROTOS = {
    "cnpc_last_error": (C.c_char_p, []),
    "cnpc_version": (C.c_char_p, []),
    "cnpc_catalog_sums_workspace_size": (_sz, []),
    "cnpc_catalog_sums": (_i32, [_PD, _cvp, _cvp, _i64, _vp, _vp, _sz, _vp]),
    "cnpc_norms": (_i32, [_PD, _cvp, _cvp, _i64, _vp, _vp]),
    "cnpc_paint_workspace_size": (_sz, [_PD, _i64, _i64]),
    "cnpc_paint": (_i32, [_PD, _cvp, _cvp, _i64, _cvp, _cvp, _i64, _cvp, _vp, _vp, _vp, _sz, _vp]),
    "cnpc_paint_fkp": (_i32, [_PD, _cvp, _cvp, _i64, _cvp, _cvp, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                              _sz, _vp]),
    "cnpc_fft_workspace_size": (_sz, [_PD, _i32, _i32]),
    "cnpc_fft_r2c": (_i32, [_PD, _i32, _i32, _cvp, _vp, _vp, _sz, _vp]),
    "cnpc_fft_c2r": (_i32, [_PD, _i32, _i32, _cvp, _vp, _vp, _sz, _vp]),
    "cnpc_band_for": (_i32, [_PD, _d]),
    "cnpc_deinterlace_workspace_size": (_sz, [_PD]),
    "cnpc_paint_deinterlace_workspace_size": (_sz, [_PD, _i64, _i64, _i32, _i32]),
    "cnpc_paint_deinterlace": (_i32, [_PD, _i32, _cvp, _cvp, _i64, _cvp, _cvp, _i64, _i32, _vp, _vp, _vp, _vp, _vp,
                                      _vp, _vp, _sz, _vp]),
    "cnpc_deinterlace": (_i32, [_PD, _i32, _cvp, _vp, _vp, _vp, _sz, _vp]),
    "cnpc_ylm_fields": (_i32, [_PD, _i32, _cvp, _vp, _vp]),
    "cnpc_ylm_r2c_workspace_size": (_sz, [_PD, _i32, _i32]),
    "cnpc_ylm_r2c": (_i32, [_PD, _i32, _i32, C.POINTER(_i32), _cvp, _vp, _vp, _sz, _vp]),
    "cnpc_assemble_F": (_i32, [_PD, _i32, _i32, _cvp, _cvp, _vp, _vp]),
    "cnpc_bin_pk_workspace_size": (_sz, [_PB, _i32, _i32]),
    "cnpc_bin_pk": (_i32, [_PD, _PB, _i32, _i32, C.POINTER(_vp), C.POINTER(_vp), _i32,
                           C.POINTER(_i32), _cvp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "cnpc_bin_pk_noalloc": (_i32, [_PD, _PB, _i32, _i32, C.POINTER(_vp), C.POINTER(_vp), _i32,
                                   C.POINTER(_i32), _cvp, _vp, _vp, _vp, _vp, _vp]),
    "cnpc_pk_finalize": (_i32, [_PB, _cvp, _cvp, _cvp, _cvp, _cvp, _cvp, _cvp, _vp, _vp]),
    "cnpc_bispec_workspace_size": (_sz, [_PD, _PB, _i32, _i32]),
    "cnpc_bispec_plan_create": (_i32, [C.POINTER(_vp), _PD, _PB, _i32, _i32, _i32, _vp, _sz, _vp]),
    "cnpc_bispec_plan_destroy": (None, [_vp]),
    "cnpc_bispec_nconfigs": (_i32, [_vp]),
    "cnpc_bispec_configs": (_i32, [_vp, C.POINTER(_i32), C.POINTER(_i64)]),
    "cnpc_bispec_band": (_i32, [_vp]),
    "cnpc_bispec_grid": (_i32, [_vp]),
    "cnpc_bispec_ext_bins": (_i32, [_vp, _PB]),
    "cnpc_bispectrum": (_i32, [_vp, _cvp, _cvp, _cvp, _cvp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "cnpc_batch_create": (_i32, [C.POINTER(_vp), _PD, _PB, _vp, _i32, C.POINTER(_i32), _i32, _i64, _i64]),
    "cnpc_batch_workspace_size": (_sz, [_vp]),
    "cnpc_batch_run": (_i32, [_vp, _i32, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_i64), C.POINTER(_vp),
                              C.POINTER(_vp), C.POINTER(_i64), C.POINTER(_vp), C.POINTER(_vp), _vp, _sz, _vp]),
    "cnpc_batch_capture": (_i32, [_vp, _i32, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_i64), C.POINTER(_vp),
                                  C.POINTER(_vp), C.POINTER(_i64), C.POINTER(_vp), C.POINTER(_vp), _vp, _sz]),
    "cnpc_batch_replay": (_i32, [_vp, _vp]),
    "cnpc_batch_destroy": (None, [_vp]),
    "cnpc_tripolar_real_coeffs": (_i32, [_i32, _i32, _i32, C.POINTER(_d), C.POINTER(_i32)]),
    "cnpc_sugi_paired_count": (_i32, [_i32, _i32, _i32]),
    "cnpc_sugi_workspace_size": (_sz, [_PD, _PB]),
    "cnpc_sugi_plan_create": (_i32, [C.POINTER(_vp), _PD, _PB, _i32, _i32, _i32, _i32]),
    "cnpc_sugiyama": (_i32, [_vp, _cvp, _cvp, _cvp, _cvp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "cnpc_sugiyama_fft_noise": (_i32, [_vp, _cvp, _cvp, _cvp, _cvp, _cvp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "cnpc_bispec_indicator_bytes": (_sz, [_vp]),
    "cnpc_bispec_indicators": (_i32, [_vp, _vp, _vp, _sz, _vp]),
    "cnpc_bispectrum_fft_noise": (_i32, [_vp, _cvp, _cvp, _cvp, _cvp, _cvp, _cvp, _vp, _vp, _vp, _vp, _sz,
                                         _vp]),
    "cnpc_ktimer_start": (_i32, [C.c_uint32, _i32]),
    "cnpc_ktimer_stop": (_i32, [C.POINTER(_d), C.POINTER(_i64)]),
    "cnpc_bin_pk_im": (_i32, [_PD, _PB, _i32, _i32, C.POINTER(_vp), C.POINTER(_vp), _vp, _vp, _vp, _vp,
                              _sz, _vp]),
    "cnpc_pk_multipole": (_i32, [_PB, _i32, _vp, _vp, _vp, _vp]),
    "cnpc_cross_norms": (_i32, [_vp, _vp, _vp, _vp]),
    "cnpc_tune_set": (_i32, [_i32, _i32]),
    "cnpc_tune_get": (_i32, [_i32]),
}

KT = {"paint": 1, "sort": 2, "fold": 3, "zr2c": 4, "col": 5, "zc2r": 6, "contract": 7, "bin": 8,
      "sums": 9}

# tuning knobs (cnpc_tune_set / cnpc_tune_get): name -> (index, allowed values)
TUNE = {"fft_passes": (0, (0, 1)), "fft_col_w": (1, (0, 1, 2, 4, 8, 16, 32, 64)),
        "contract_kg": (2, (0, 1, 2, 4)), "sort_per": (3, (0, 1, 2, 4)),
        "sort_threads": (4, (0, 512, 1024)), "sort_fused": (5, (0, 1, 2)), "fold_fused": (6, (0, 1)),
        "bucket": (7, (0, 1, 2, 3)), "ylm_basis": (8, (0, 1)), "shell_fused": (9, (0, 1))}

EXPORTED = tuple(_PROTOS)

for _name, (_res, _args) in _PROTOS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def last_error() -> str:
    return lib.cnpc_last_error().decode()


def check(status: int) -> None:
    if status != 0:
        raise CnpcError(status, last_error())


def ptr(t) -> int | None:
    """Device (or host) pointer of a torch tensor, None for None."""
    if t is None:
        return None
    return t.data_ptr()


def stream_handle(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def mesh_desc(n, boxsize, assign=TSC, interlace=True, dtype=F32, observer=None, los=None) -> MeshDesc:
    d = MeshDesc()
    d.n = int(n)
    d.assign = int(assign)
    d.interlace = int(bool(interlace))
    d.dtype = int(dtype)
    d.boxsize = float(boxsize)
    if los is not None:
        d.los_mode = LOS_GLOBAL
        for i in range(3):
            d.los[i] = float(los[i])
    else:
        d.los_mode = LOS_LOCAL
        obs = observer if observer is not None else (-866.0254037844386,) * 3
        for i in range(3):
            d.observer[i] = float(obs[i])
    return d


def kbins(kmin, dk, nbins) -> KBins:
    b = KBins()
    b.kmin, b.dk, b.nbins = float(kmin), float(dk), int(nbins)
    return b
