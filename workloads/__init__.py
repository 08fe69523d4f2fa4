"""Seeded synthetic workloads shared by the GPU path and the FP64 oracle.

This package only draws random inputs: disk packings that stand in for the
axon substrate of the paper (section 2.2: non-overlapping circles of
Gamma-distributed radius in a square) and start points for the initial
pulses (section 4.1: points drawn uniformly in the extracellular region).
It holds none of the method's arithmetic (no mesh, no operator, no time
stepping, no moments), so that neither side of a parity test can lean on
the other through it.
"""

from .geometry import rsa_disks, start_points, Geometry, make_geometry  # noqa: F401
from .configs import CONFIGS, config, batch_geometry_params, batch_workload  # noqa: F401
