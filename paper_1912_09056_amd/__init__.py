"""MI355X-native block-AMG preconditioned FGMRES for mortar-contact
saddle-point systems (Wiesner, Mayr, Popp, Gee, Wall: algebraic multigrid
for saddle point systems from mortar contact formulations).

The solver lives in the HIP library libcamg.so (C-ABI in include/camg.h);
this package is its Python binding plus a differentiable wrapper.
"""
from .camg import AMGOptions, AMGSolver, CamgError, PREC_FP64, PREC_MIXED, PREC_MIXED_BF16, load_library
from .autograd import ContactSolve, contact_solve

__all__ = [
    "AMGOptions",
    "AMGSolver",
    "CamgError",
    "PREC_FP64",
    "PREC_MIXED",
    "PREC_MIXED_BF16",
    "load_library",
    "ContactSolve",
    "contact_solve",
]
