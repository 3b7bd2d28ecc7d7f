"""MI355X (gfx950) FastNeRF cached renderer.

The compute path is the HIP library ``libfastnerf.so`` (C ABI in
``include/fastnerf.h``); this package is its thin Python binding. PyTorch
supplies device memory and streams only.
"""
from ._lib import (BF16, F16, F32, FP8, IN_BOX, LINEAR, NEAR_FAR, NEAREST, Cache,  # noqa: F401
                   FastNeRFError, Mlp, Server, debug_lookup, filter_direction, get_schedule,
                   lib, lod_select, make_desc, mlp_desc, model_bytes, render, render_batch,
                   set_schedule)
