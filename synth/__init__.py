"""Seeded synthetic return panels for YAND-MVSK workloads.

This module only draws random inputs (return matrices, coefficient vectors,
return targets).  It holds none of the solver's arithmetic, so both the FP64
CPU oracle and the GPU path can take their inputs from it without sharing any
part of the method.
"""

from .factor_model import (  # noqa: F401
    factor_returns,
    priced_factor_returns,
    uniform_returns,
    crra_coefficients,
    WORKLOADS,
    workload_returns,
    frontier_targets,
    ragged_universe_sizes,
)
from .conditioning import conditioned_returns, conditioning_spectrum  # noqa: F401
