"""MI355X-native randomized small-block Lanczos null-space solver.

The numerical work runs in ``libnullspace.so`` (hand-written HIP for gfx950,
C ABI in ``include/nullspace.h``); this package only marshals arguments.
"""
from ._lib import (  # noqa: F401
    Context,
    NspError,
    Params,
    Stats,
    default_params,
    load,
    locality_order,
    PREC_FP64,
    PREC_MIXED,
    OP_NORMAL,
    OP_SYM,
    PRECOND_NONE,
    PRECOND_JACOBI,
    PRECOND_IC,
)
from .autograd import NullSpaceFunction, null_space  # noqa: F401
