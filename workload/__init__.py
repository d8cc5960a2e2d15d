"""Seeded synthetic inputs for the Galilean-PSATD PIC step.

This module is the only code the oracle and the HIP path both use.  It holds
workload descriptions and random-number draws (positions, momenta, a laser
envelope sampled on the nodes) and none of the method's arithmetic: no
shapes, transforms, coefficients, updates or pushes.

Inputs are generated so that every value is exactly representable in
float32 where the mixed-precision path stores it (in-cell offsets and
momenta), which lets the FP64 oracle and the mixed path start from bit-equal
states.
"""

from .configs import CONFIGS, RunConfig, batched_runs, get_config  # noqa: F401
from .gen import (  # noqa: F401
    laser_fields,
    particles_for,
    split_positions,
)
