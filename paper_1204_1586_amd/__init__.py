"""MI355X-native fast CP gradient (all-mode MTTKRP) and CP_ALS.

Python side of libcpgrad: thin wrappers with the C ABI's names
(``include/cpgrad.h``) that take torch tensors on the GPU.  All computation
runs in the library's HIP kernels; importing this package fails if the
library has not been built (``python -m paper_1204_1586_amd.build``).
"""
from ._lib import (  # noqa: F401
    NFEAT, Mlp, cp_fit_extrapolated, cpals_extrapolate, cpals_features, cpals_learned_step, cpmlp_create, cpmlp_destroy, cpmlp_forward,
    cpmlp_get_params, cpmlp_gradients, cpmlp_num_params, cpmlp_set_params, cpmlp_train_step,
)
from ._lib import (  # noqa: F401
    CPG_BF16, CPG_F16, CPG_F32, CPG_F64, CPG_MODE_BF16, CPG_MODE_F16_SCALED, CPG_MODE_F16_SCALED_REFINED, CPG_MODE_BF16_REFINED, CPG_MODE_NATIVE, CPG_OPT_FORCE_NSTAR,
    CPG_OPT_KERNEL, CPG_OPT_MFMA_COLS, NOALLOC_SCRATCH_BYTES, CPG_OPT_PROFILE, EXPORTS, LIB, LIB_PATH, CpgError, Plan, cp_fit, cpals_step, cpgrad_all_modes, cpgrad_all_modes_noalloc, cpgrad_bind, cpgrad_e_gradient,
    cpgrad_mode_gradient, cpntf_step,
    cpgrad_destroy, cpgrad_last_fit, cpgrad_plan, cpgrad_plan_info, cpgrad_plan_path, cpgrad_profile_read, cpgrad_query, cpgrad_set_option, cpgrad_version,
)
