"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package only draws positions, charges, velocities and masses. It holds
none of the multilevel-summation arithmetic, so both implementations can take
their inputs from here without sharing any of the method.

The paper (Introduction; Section 2) targets explicit-water biomolecular systems
(a 30 x 65 x 65 nm box) and gives no data set. The generators below stand in
for that with point charges and rigid 3-site water molecules (TIP3P charges and
geometry) on a jittered lattice at about 100 atoms per nm^3.
"""
from .water import (  # noqa: F401
    Workload,
    uniform_pm,
    uniform_pm_box,
    water_box,
    water_box_dims,
    maxwell_velocities,
    uneven_batch_sizes,
    water_model_arrays,
    rigid_water_velocities,
    named,
)
