"""MI355X-native cooperative conjugate gradient (cCG): HIP kernels behind a C ABI.

The solver lives in ``libccg.so`` (sources under ``csrc/``, header
``include/ccg.h``); ``ccg.py`` is its Python binding.  Build with
``python -m paper_1204_0069_amd.build``.
"""
from .ccg import (CCG_ESCALATE, CCG_SYM_AD, CCG_REINFLATE, CCG_NO_TIER, CCG_HOST_PTRS, CCG_NO_GRAPH, CCG_PROFILE, CCG_PROFILE_SAMPLED, EXPORTS, LIB_PATH,
                  PREC, STATUS, CcgError, Context, load_library, make_opts)

__all__ = ["Context", "CcgError", "load_library", "make_opts", "LIB_PATH", "EXPORTS", "PREC",
           "STATUS", "CCG_HOST_PTRS", "CCG_NO_GRAPH", "CCG_PROFILE", "CCG_PROFILE_SAMPLED", "CCG_ESCALATE",
           "CCG_SYM_AD", "CCG_REINFLATE", "CCG_NO_TIER"]
