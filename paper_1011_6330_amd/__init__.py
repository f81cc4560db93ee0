"""MI355X-native 1D polar-cap PIC time step (Barzilay, polar-cap paper, Part I).

The compute path is the gfx950 HIP library ``libpcpic.so`` behind the C ABI of
``include/pcpic.h``; ``Tube`` is its ctypes binding.  Importing this package
does not load the library; constructing a ``Tube`` does, and fails loudly if
it is not built or no GPU is present.
"""
from ._binding import (ABI_VERSION, B_STEADY_INIT, FP32_BULK, FP64, FREEZE_FIELDS, GR_ALPHA, NO_AUTO_INJECT,  # noqa: F401
                       RHO_FRAME_DRAG, RHO_GR,  # noqa: F401
                       RHO_KNOTS, RHO_UNIFORM, ST_CAPACITY, ST_NONFINITE, Batch, PicError, Tube, load,
                       make_params, workspace_bytes)
