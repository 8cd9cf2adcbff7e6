"""MI355X (gfx950) implementation of the energy-stable FAS step for the
hydrodynamic PFC / CDFT freezing models (arXiv 1503.07416).

The numerical work runs in ``libhfz.so`` (HIP kernels behind the C ABI of
include/hfz.h); :mod:`.hfz` is its ctypes binding.
"""
from .hfz import (CDFT, FP64, MIXED, PFC, Batch, HfzError, Simulation, load, make_params,  # noqa: F401
                  workspace_bytes)
