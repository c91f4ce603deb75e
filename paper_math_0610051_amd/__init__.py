"""MI355X (gfx950) implementation of the wedge-localised fast FIO apply.

The compute path is the HIP library libfio.so (C ABI in include/fio.h);
`fio` is its ctypes binding.  Build it with `python -m
paper_math_0610051_amd.build` or `__graft_entry__.build()`.
"""
from .fio import (FioError, Learned, Plan, apply_multi, autotune, copy, host_eigh, load_library,  # noqa: F401
                  make_phase, PHASE_KINDS)

__all__ = ["FioError", "Learned", "Plan", "autotune", "apply_multi", "copy", "host_eigh", "load_library", "make_phase", "PHASE_KINDS"]
