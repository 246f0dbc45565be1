"""Seeded synthetic inputs for grouped full-spectrum fitting.

This package draws the random numbers and builds the arrays that both the
FP64 oracle and the HIP path consume: wavelength grids, interpolator
coefficient spectra ("basis"), observed spectra with their inverse variance,
initial guesses and the injected truths.  It holds none of the fitting
method's arithmetic: observed spectra are simulated analytically (a
Doppler-shifted Gaussian line convolved in closed form with a Gaussian
broadening profile, then averaged over each pixel's wavelength bin), not
with the model the fit evaluates.
"""

from .generator import (  # noqa: F401
    BOX_HI,
    BOX_LO,
    C_KMS,
    EXPONENTS,
    REGIME_EDGES,
    Shape,
    SpectraBatch,
    class_weights,
    linear_grid_basis,
    make_basis,
    make_spectra,
    make_spectra_parallel,
    poisson_requests,
    shape_by_name,
    wave_grid,
)
