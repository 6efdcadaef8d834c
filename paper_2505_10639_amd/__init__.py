"""MI355X-native MOMFBD hot path: loss, gradient and Wiener object of
multi-object multi-frame blind deconvolution on hand-written gfx950 kernels.

The compute lives in libmomfbd.so (C-ABI declared in include/momfbd.h);
this package is its binding.  `import paper_2505_10639_amd` does not load
the library; the first call does, and fails loudly if it is not built.
"""

from ._lib import (MomfbdError, LIB_PATH, momfbd_status_string, momfbd_plan_create,
                   momfbd_plan_destroy, momfbd_workspace_size, momfbd_plan_dims,
                   momfbd_object_filtered, momfbd_mosaic, filter_spec,
                   momfbd_synthesize, momfbd_lbfgs_rounds, momfbd_power_spectrum,
                   momfbd_plan_set_tuning, momfbd_plan_get_tuning, momfbd_plan_autotune,
                   momfbd_cnn_create, momfbd_cnn_destroy,
                   momfbd_cnn_sizes, momfbd_cnn_init, momfbd_cnn_load, momfbd_cnn_forward,
                   momfbd_cnn_loss_grad, momfbd_cnn_adam, momfbd_cnn_input,
                   momfbd_smoothness_gamma,
                   momfbd_prepare_data, momfbd_forward, momfbd_loss_grad,
                   momfbd_object_estimate, momfbd_profile_start, momfbd_profile_repeat,
                   momfbd_profile_stop, momfbd_lbfgs_state_size, momfbd_lbfgs_init,
                   momfbd_lbfgs_step, lbfgs_params, lib)

__all__ = [
    "MomfbdError", "LIB_PATH", "momfbd_status_string", "momfbd_plan_create",
    "momfbd_plan_destroy", "momfbd_workspace_size", "momfbd_plan_dims", "momfbd_smoothness_gamma",
    "momfbd_object_filtered", "momfbd_mosaic", "filter_spec", "momfbd_synthesize",
    "momfbd_lbfgs_rounds", "momfbd_power_spectrum", "momfbd_plan_set_tuning",
    "momfbd_plan_get_tuning", "momfbd_plan_autotune",
    "momfbd_cnn_create", "momfbd_cnn_destroy", "momfbd_cnn_sizes", "momfbd_cnn_init",
    "momfbd_cnn_load", "momfbd_cnn_forward", "momfbd_cnn_loss_grad", "momfbd_cnn_adam",
    "momfbd_cnn_input",
    "WarmStartNet",
    "momfbd_prepare_data",
    "momfbd_forward", "momfbd_loss_grad", "momfbd_object_estimate", "momfbd_profile_start",
    "momfbd_profile_repeat", "momfbd_profile_stop", "momfbd_lbfgs_state_size", "momfbd_lbfgs_init",
    "momfbd_lbfgs_step",
    "lbfgs_params", "lib", "Plan", "Solver",
    "MomfbdLoss", "momfbd_loss",
]


def __getattr__(name):
    if name in ("Plan", "Solver"):
        from . import plan
        return getattr(plan, name)
    if name == "WarmStartNet":
        from . import warmstart
        return warmstart.WarmStartNet
    if name in ("MomfbdLoss", "momfbd_loss"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
