"""MI355X-native FCG-NO: flexible conjugate gradients preconditioned by a
Fourier neural operator, as hand-written HIP kernels for gfx950 behind the C
ABI in include/fcgno.h.  This package is the thin Python binding."""
from ._binding import (OP, SYS_BREAKDOWN, SYS_NONFINITE, SYS_NOT_CONVERGED, SYS_OK,  # noqa: F401
                       FcgnoError, Model, lib, precond_apply, precond_apply_noalloc, solve, solve_workspace_bytes,
                       weight_count, profile_enable, profile_reset, profile_read, PROFILE_KERNELS,
                       Optim, train_workspace, op_forward, op_backward, energy_loss, train_step,
                       OperatorFunction, krylov_samples, residual_samples, Engine, LOSS)
