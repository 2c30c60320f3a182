"""MI355X Segment Linking (Line Segment Tracking, arXiv:2209.13711).

The compute lives in ``_lib/liblst.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/lst.h``); ``lst`` is its ctypes binding.
"""
from .lst import (LST_MD, LST_SEG, LST_T3, LST_T5, LST_T5_KEPT, LST_MODE_CUTS, LST_MODE_MLP,  # noqa: F401
                  LST_OK, LST_E_INVALID, LST_E_STATE, LST_E_CAPACITY, LST_E_HIP, LST_E_NOMEM,
                  LST_E_FAULT, LST_TC_PT5, LST_TC_PT3, LST_TC_T5, LST_TC_PLS, LST_MLP_NFEAT, LST_MLP_NPARAM, WIDTH, Context, LSTError, default_caps,
                  load_library, lst_build_map, lst_stream_copy)
