"""FP64 CPU oracle of the HWENO-I scheme -- test infrastructure only.

Imported by the tests, by the package smoke check and by the CPU-baseline leg
of the benchmark; never by the product path.
"""
from .hweno import (Problem, rhs, step, run, run_fixed, max_speed, time_step,  # noqa: F401
                    hweno_cell, central_D, mixed_flux, smoothness_indicators,
                    nonlinear_weights, make_system, pad, Euler)
