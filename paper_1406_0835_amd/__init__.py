"""MI355X finite-temperature orbital-free DFT hot path (arXiv:1406.0835).

The compute lives in libofdft.so (hand-written HIP for gfx950 behind the C ABI
declared in include/ofdft.h).  This package is the Python binding: argument
marshalling only.  Importing it does not load the library; the first Context
does, and raises if the library has not been built.
"""
from .binding import (  # noqa: F401
    APBEF, CG, FP64, KST2, LPP_GAUSS, LPP_HA, MIXED, SGA, TF, TN, TW, VT84F, VWTF, XC_KSDT, XC_NONE, XC_PZ81,
    Context, OFDFTError, Options, Report, batch_minimize, default_options, ewald, library_path, load_library,
)
