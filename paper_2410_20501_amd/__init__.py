"""MI355X (gfx950) particle-mesh force-and-step library (arXiv:2410.20501, PySCo method).

The compute lives in libhippm.so (hand-written HIP kernels behind include/hippm.h);
this package is its Python binding. Importing fails loudly if the library has
not been built: `python paper_2410_20501_amd/build.py`.
"""
from .hippm import *  # noqa: F401,F403
from .hippm import (  # noqa: F401
    Context, PMError, PMWarning, MGParams, MGStats, StepParams, StepStats, EXPORTED,
    default_step_params, pm_create, pm_destroy, pm_deposit, pm_solve_mg, pm_solve_fft,
    pm_gradient, pm_interp, pm_accel, pm_kdk, pm_kdk_chain, pm_reorder,
    pm_kernel_timer, pm_kernel_timer_read,
    pm_deposit_vjp, pm_interp_vjp, pm_gradient_vjp, pm_accel_vjp, pm_kdk_adjoint,
    pm_density_loss, pm_ic_state, pm_ic_vjp,
    Batch, pm_batch_create, pm_batch_accel, pm_batch_kdk, pm_graph_capture_step, pm_tune,
)
