"""MI355X (gfx950) implementation of the rank-adaptive sweep-based SI-DSA for the
steady first-order radiative transfer equation (Guo & Peng, arXiv 2603.25233).

The computation lives in the HIP library librte.so (C ABI in include/rte.h); this
package is its Python binding.  Build it with `python -m paper_2603_25233_amd.build`.
"""
from .rte import (RTE_FP64, RTE_MIXED, SIDE_B, SIDE_L, SIDE_R, SIDE_T, Problem, RTEError, SweepPlan,
                  adjoint_sweep, backward_euler_step, box_source_moments, cl_quadrature,
                  cross_section_gradient,
                  default_params, exit_currents, gaussian_source_moments, inflow_moments, lib,
                  release_cached_memory, solve, sweep, sweep_noalloc)
from .rte import detector_misfit as detector_misfit_data
from .autograd import DetectorMisfit, DetectorMisfitBatch, detector_misfit, detector_misfit_batch

__all__ = ["RTE_FP64", "RTE_MIXED", "SIDE_L", "SIDE_R", "SIDE_B", "SIDE_T", "Problem", "RTEError", "SweepPlan",
           "adjoint_sweep", "backward_euler_step", "box_source_moments", "gaussian_source_moments", "cl_quadrature",
           "cross_section_gradient",
           "default_params", "exit_currents", "inflow_moments", "lib", "release_cached_memory", "solve",
           "sweep", "sweep_noalloc",
           "detector_misfit_data", "DetectorMisfit", "detector_misfit", "DetectorMisfitBatch",
           "detector_misfit_batch"]
