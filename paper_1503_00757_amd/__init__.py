"""MI355X (gfx950) reduced-space Gauss-Newton-Krylov registration library (Python binding).

The compute path is the C-ABI library ``libregnk.so`` (hand-written HIP kernels); this package only
marshals arguments to it.  ``ffi`` holds the raw C functions with the names of ``include/regnk.h``;
``Problem`` is a convenience wrapper that keeps the workspace and device vectors in torch tensors.
There is no CPU fallback: if the library is not built, importing ``ffi.lib()`` raises.
"""
from .ffi import (  # noqa: F401
    RegParams, RegSolveOpts, RegSolveStats, RegStepRecord, RegError, lib, library_path,
    REG_H1, REG_H2, REG_UNCONSTRAINED, REG_DIVFREE, REG_MASS_SOURCE, REG_FP64, REG_FP32_TRANSPORT,
    REG_ADJ_DISCRETE, REG_ADJ_PAPER,
    reg_workspace_bytes, reg_create, reg_destroy, reg_set_stream, reg_state_forward, reg_objective,
    reg_gradient, reg_hessian_matvec, reg_precond_apply, reg_pcg, reg_solve, reg_time_pass, reg_time_phases,
    reg_autotune, reg_set_pass_variants, reg_batch_solve, reg_set_images, reg_deformation,
    reg_deformation_workspace_bytes, reg_cfl, REG_H3,
    reg_fno_param_count, reg_fno_workspace_bytes, reg_fno_create, reg_fno_destroy, reg_fno_features, reg_fno_target,
    reg_fno_gather, reg_fno_forward, reg_fno_backward, reg_fno_adam, reg_fno_train_step, reg_fno_predict,
    REG_FNO_PARAMS,
    reg_last_error,
)
from .problem import Problem, batch_solve, paper_nt  # noqa: F401
from .warmstart import Network, WarmStart  # noqa: F401
