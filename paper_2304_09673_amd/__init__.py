"""MI355X-native synchronized tracing of blobtrees (Zanni 2023, arXiv 2304.09673).

The compute path is the HIP library ``libsynctrace.so`` (C ABI in
``include/st.h``); this package is its thin binding.
"""
from .st import (EXPORTS, LIB_PATH, ST_STEP_LEARNED, ST_STEP_OVERRELAX, ST_STEP_PLAIN, Scene, StError,
                 default_tuning, lib, make_camera)

__all__ = ["EXPORTS", "LIB_PATH", "Scene", "StError", "default_tuning", "lib", "make_camera",
           "ST_STEP_PLAIN", "ST_STEP_OVERRELAX", "ST_STEP_LEARNED"]
