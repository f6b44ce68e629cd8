"""MI355X-native velocity-gauge real-time TDDFTB density-matrix propagation.

The compute path is the HIP library libvgtb.so (C ABI in include/vgtb.h);
this package holds its sources (csrc/), the in-tree build step (build.py)
and the ctypes binding (vgtb.py).
"""
from .vgtb import (  # noqa: F401
    EXPORTED,
    Group,
    LIB_PATH,
    Propagator,
    Server,
    VgtbError,
    VGTB_OK,
    VGTB_E_INVAL,
    VGTB_E_STATE,
    VGTB_E_NOT_PD,
    VGTB_E_UNSTABLE,
    VGTB_E_NOMEM,
    VGTB_E_DEVICE,
    VGTB_E_NONFINITE,
    load_library,
    make_options,
    make_system_struct,
    spectrum_noalloc,
    vgtb_workspace_size,
    vgtb_zgemm,
)
