"""MI355X (gfx950) Virtual Transmission Method over EVS-split SPD systems.

The compute path lives in ``libvtm.so`` (C ABI in ``include/vtm.h``); this
package only marshals arguments to it.
"""
from .binding import (  # noqa: F401
    VTM,
    VTMError,
    VTM_FP64,
    VTM_FP32_IR,
    VTM_Z_DIAG,
    VTM_Z_USER,
    VTM_Z_LEARNED,
    lib,
)
