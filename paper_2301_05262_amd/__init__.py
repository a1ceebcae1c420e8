"""Neural shadow mapping hot path for MI355X (gfx950).

The compute lives in ``libnsm.so`` (hand-written HIP kernels behind a C ABI,
``include/nsm.h``); this package only marshals arguments.  Importing the
package does not load the library; the first call into it does, and raises
if the library has not been built.
"""
from ._lib import (  # noqa: F401
    NsmError,
    EXPORTS,
    LIB_PATH,
    load,
    nsm_abi_version,
    nsm_status_str,
    nsm_features_workspace_bytes,
    nsm_build_features,
    nsm_build_features_stored,
    nsm_create,
    nsm_destroy,
    nsm_param_count,
    nsm_set_weights,
    nsm_workspace_bytes,
    nsm_forward,
    nsm_forward_stored,
    nsm_backward,
    nsm_forward_train,
    nsm_backward_saved,
    frame_params,
    nsm_trace_enable,
    nsm_trace_read,
    nsm_autotune,
    nsm_autotune_stored,
    nsm_set_stage_variant,
    nsm_get_stage_variants,
    nsm_perturbation_loss_workspace_bytes,
    nsm_perturbation_loss,
    nsm_perturbation_loss_noalloc,
    nsm_temporal_workspace_bytes,
    nsm_temporal_instability,
)


def __getattr__(name):
    if name in ("FeatureBuilder", "ShadowNet", "NSMForward"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
