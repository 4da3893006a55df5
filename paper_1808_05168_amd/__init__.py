"""fnlb: fluctuating two-species D2Q9 lattice Boltzmann on MI355X (gfx950).

The hot path (collision, forcing, noise, streaming, structure-factor and
pressure accumulation) runs in the HIP library ``libfnlb.so`` behind the C ABI
of ``include/fnlb.h``; this package is its thin Python binding.
"""
from .fnlb import (ASTAR, DEFAULT_FLAGS, FIELD_C, FIELD_RHO, FIELD_UX, FIELD_UZ, FORCE_LITERAL,
                   FP32_DEV, FP64, NO_GRAPH, NOISE_LOC, ONE_STEP, SAMPLE_VELOCITY, STATIC_WORK_BYTES,
                   TWO_STEP,
                   WALL_UZ_FIX, FnlbError,
                   Lattice, bytes_required, load, p_misfit, sq_misfit, tune_cache_load,
                   tune_cache_save, tune_lookup)

__all__ = ["ASTAR", "DEFAULT_FLAGS", "FIELD_C", "FIELD_RHO", "FIELD_UX", "FIELD_UZ",
           "FORCE_LITERAL", "FP32_DEV", "FP64", "NO_GRAPH", "NOISE_LOC", "SAMPLE_VELOCITY",
           "STATIC_WORK_BYTES", "TWO_STEP", "ONE_STEP",
           "WALL_UZ_FIX", "FnlbError", "Lattice", "bytes_required", "load", "p_misfit",
           "sq_misfit", "tune_cache_load", "tune_cache_save", "tune_lookup"]
