"""MI355X (gfx950) implementation of the energy-stable FAS step for the
hydrodynamic PFC / CDFT freezing models (arXiv 1503.07416).

The numerical work runs in ``libhfz.so`` (HIP kernels behind the C ABI of
include/hfz.h); :mod:`.hfz` is its ctypes binding.
"""
from .hfz import (CDFT, CDFT_GF, FP64, MIXED, PFC, PFC_GF, Batch, HfzError, Simulation,  # noqa: F401
                  Simulation3, load, make_params, step_noalloc, workspace_bytes)
