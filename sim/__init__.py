"""Seeded synthetic ptychography workloads.

This module only draws inputs: object, probe, scan positions, diffraction
intensities, initial guesses and per-sweep position orders.  It holds none of
the reconstruction's arithmetic (no modulus projection, no update, no
schedule); the diffraction data are produced by a plain far-field forward
simulation with scipy's FFT.  Both the oracle's tests and the GPU path read
their inputs from here, so it imports neither of them.
"""
from .configs import (  # noqa: F401
    Workload, make_config, make_workload, make_probe, make_object,
    raster_positions, fermat_positions, object_extent, simulate_intensities,
    initial_probe, sweep_order, live_plan, CONFIGS, make_multiscan,
)
