"""HWENO-I on MI355X: the fifth-order interpolation-based Hermite WENO scheme's
spatial operator and SSP-RK3 update as hand-written HIP kernels for gfx950.

The binding (``paper_2411_11229_amd.hweno``) loads the C-ABI library built
from ``csrc/`` lazily, on first use, and raises if it is missing.
"""
