"""Seeded synthetic inputs for the MOMFBD hot path.

This package produces *inputs* only: pupil masks, the Zernike modal basis,
phase-diversity maps, Kolmogorov modal coefficients, random solar-like object
fields, apodization windows and noise.  It holds none of the method's
arithmetic (no wavefront-to-PSF chain, no Fourier-domain accumulators, no
loss).  Both the FP64 oracle and the GPU library consume the arrays made
here; neither imports the other.
"""

from .geometry import (noll_to_nm, zernike_basis, pupil_mask, pupil_radius_px,
                       hann_window, defocus_diversity)
from .turbulence import noll_covariance, draw_kolmogorov, kl_transform, kl_basis
from .fields import object_field, gaussian_noise
from .configs import (Problem, make_problem, config0, config1_geometry,
                      config1_alpha, config1_object, config1_problem,
                      config1_d_over_r0, config4_geometry, config4_template,
                      config4_alpha, config4_objects, config4_problem, patch_grid,
                      SEED_ROOT)

__all__ = [
    "noll_to_nm", "zernike_basis", "pupil_mask", "pupil_radius_px", "hann_window",
    "defocus_diversity", "noll_covariance", "draw_kolmogorov", "kl_transform", "kl_basis",
    "object_field",
    "gaussian_noise", "Problem", "make_problem", "config0", "config1_geometry",
    "config1_alpha", "config1_object", "config1_problem", "config1_d_over_r0",
    "config4_geometry", "config4_template", "config4_alpha", "config4_objects",
    "config4_problem",
    "patch_grid", "SEED_ROOT",
]
