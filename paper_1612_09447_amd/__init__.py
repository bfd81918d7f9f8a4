"""MI355X (gfx950) explicit Runge-Kutta-Chebyshev time integration for nonlinear
electro-quasistatic fields (Richter, Schoeps, Clemens, arXiv 1612.09447).

The compute path is the HIP library ``libeqs.so`` (C ABI in ``include/eqs.h``);
``binding`` marshals arguments to it. PyTorch is used only for device memory
and streams.
"""

from .binding import (  # noqa: F401
    Batch,
    Context,
    EqsError,
    Mlp,
    EQS_GUESS_GALERKIN,
    EQS_GUESS_MLP,
    EQS_GUESS_MOR,
    EQS_GUESS_PREVIOUS,
    EQS_GUESS_ZERO,
    EQS_MLP_NPARAM,
    EQS_OK,
    EQS_ERR_INVALID_ARG,
    EQS_ERR_STATE,
    EQS_ERR_HIP,
    EQS_ERR_NOT_CONVERGED,
    EQS_ERR_BREAKDOWN,
    EQS_ERR_NONFINITE,
    EQS_ERR_ALLOC,
    EQS_PREC_FP32,
    EQS_PREC_FP64,
    LIB_PATH,
    lib,
)
