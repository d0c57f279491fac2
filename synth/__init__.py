"""Seeded synthetic inputs shared by the FP64 oracle, the GPU path, the tests and the benchmark.

This package only draws and lays out initial conditions and request traces. It holds none of the
method's arithmetic: no pair force, no integrator, no growth rule and no L1 test.
"""

from .binary import (  # noqa: F401
    BinaryIC,
    make_binary,
    particle_counts,
    element_diameter,
    orbital_omega,
    with_velocity_noise,
    paper_law_params,
)
from .trace import Request, make_trace  # noqa: F401
