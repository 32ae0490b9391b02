"""Seeded synthetic inputs for the turbulent gas-kinetic scheme.

This package produces initial states, grids, boundary data and frozen k/omega
fields.  It holds none of the scheme's arithmetic (no fluxes, moments or
updates); both the FP64 CPU oracle and the HIP library consume what it makes.
"""
from .cases import (  # noqa: F401
    Case, BC_NAMES, nvar_of, mixing_layer, sbli, isotropic_box, shock_tube,
    sod_tube, shear_wave, entropy_wave, uniform_flow, batch_cases, serve_trace,
    cons_from_prim, config_case,
)
