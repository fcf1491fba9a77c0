"""MI355X (gfx950) radiation spectral synthesis: the in-situ Lienard-Wiechert
spectral integral of a particle sample (paper, Section 2.2), as a HIP library
with a C ABI (include/lw.h) and this thin Python binding, plus a learned
spectrum surrogate (``surrogate``) that runs on the library's own kernels.
"""
from .lw import (LIB_PATH, PATHS, MLP, Context, DeviceBatch, Graph, LWError, load_library,  # noqa: F401
                 LW_OK, LW_EINVAL, LW_ENOMEM, LW_EDEVICE, LW_ESTATE, LW_ERANGE, LW_EUNSUPPORTED)
from .insitu import Recorder  # noqa: F401
