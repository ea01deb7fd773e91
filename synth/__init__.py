"""Seeded synthetic inputs for the plane-wave H·psi / block-Davidson path.

This package only *draws* problem data (cell, atoms, well depths, nonlocal
coefficients, overlap augmentation, k-points, starting bands) and samples the analytic input
functions (Gaussian local wells on the real-space grid, Gaussian-radial
projectors at given wave vectors).  It holds none of the method's
arithmetic: no sphere enumeration, no FFT, no Hamiltonian application, no
eigensolver.  Both the CPU oracle and the GPU path are fed from here.
"""
from .cells import (  # noqa: F401
    CONFIGS,
    Cell,
    make_cell,
    vloc_on_grid,
    projectors,
    psi_start,
    smooth_grid,
    alias_free_min,
    with_augmentation,
)
