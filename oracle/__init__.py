"""FP64 CPU oracle of the MOMFBD hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, direct-DFT NumPy implementation of what the GPU library
computes, written from the paper's equations.  Only the test-suite, the
package smoke check and the CPU-baseline leg of the benchmark may import it;
the product path never calls it and shares no code with it.
"""

from .momfbd import (dft2, idft2_un, expand_half, wavefront, pupil_field, psf_field,
                     psf, otf, accumulators, evaluate_patch, evaluate,
                     object_image, prepare_data, patch_spectra, simulate_frames,
                     loss_literal, smoothness_gamma)
from .lbfgs import lbfgs_minimize

__all__ = [
    "dft2", "idft2_un", "expand_half", "wavefront", "pupil_field", "psf_field",
    "psf", "otf", "accumulators", "evaluate_patch", "evaluate", "object_image",
    "prepare_data", "patch_spectra", "simulate_frames", "loss_literal", "smoothness_gamma",
    "lbfgs_minimize",
]
