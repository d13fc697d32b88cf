"""MI355X-native FFT power-spectrum / bispectrum multipole estimators.

Python binding of the HIP library ``libcnpc.so`` (C ABI in ``include/cnpc.h``).
Importing the package fails loudly when the library has not been built.
"""

from . import _lib
from ._lib import (CIC, TSC, F32, F64, EST_SCOCCIMARRO, EST_TRIPOSH, PREC_F32, PREC_F64,
                   PREC_BF16X3, CnpcError, kbins, mesh_desc)

__all__ = ["_lib", "CIC", "TSC", "F32", "F64", "EST_SCOCCIMARRO", "EST_TRIPOSH", "PREC_F32",
           "PREC_F64", "PREC_BF16X3", "CnpcError", "kbins", "mesh_desc"]
