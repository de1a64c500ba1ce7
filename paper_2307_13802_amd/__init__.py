"""MI355X (gfx950) force engine for sheared dense suspensions.

The per-timestep hot path of the pairwise contact, lubrication and Brownian
model of Li, Royer & Ness (arXiv 2307.13802) runs in hand-written HIP kernels
behind the C ABI declared in ``include/sim.h``; this package is a thin ctypes
binding with the same function names (argument marshalling only).
"""
from .sim import (Config, Sim, lib, library_path, build, SimError, FP64, MIXED,  # noqa: F401
                  FREEZE_X, NO_LUB, NO_PAIR_BROWN, NO_CONTACT, NO_ONEBODY, LUB_ROT, REBUILD_EACH_STEP, NO_GRAPH,
                  HALF_OCC_ON, HALF_OCC_OFF, SMALL_QUEUE, TRACK_DISPLACEMENT, KERNEL_AUTO, KERNEL_HALF, set_tune_cache,
                  use_torch_allocator, use_default_allocator, STRESS_CONTACT, STRESS_LUB, STRESS_BROWN, STRESS_DRAG, STRESS_TOTAL,
                  STRESS_LAST, STRESS_MEAN)
