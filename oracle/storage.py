"""Oracle: reduced-precision storage of the fine-level stiffness block in the
V-cycle (FP64 arithmetic on the rounded values, CPU).

Test infrastructure only (see the package docstring).

Not a step of the paper: the solver's mixed-precision option that keeps the
fine level's K for the V-cycle (smoothing sweeps and the residual before
restriction) in bfloat16 while the outer FGMRES operator keeps K in FP64.
The V-cycle then applies exactly the operator whose K entries are rounded,
so the oracle's reference is the same V-cycle on a hierarchy whose level-0 K
holds the rounded values; the smoother data (Jacobi diagonal, lumping, Schur
diagonal) stay those of the FP64 K, as the library computes them at setup.

Rounding: FP64 -> FP32 to nearest (ties to even), then FP32 -> bfloat16
(sign, 8 exponent bits, 7 mantissa bits: the upper half of the FP32 word) to
nearest, ties to even.
"""
from __future__ import annotations

import copy

import numpy as np


def round_bf16(a):
    """FP64 values rounded to FP32 and then to bfloat16, returned as FP64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32)).view(np.uint32).astype(np.uint64)
    lower = f & 0xFFFF
    upper = f >> 16
    # nearest, ties to the even upper half
    up = (lower > 0x8000) | ((lower == 0x8000) & ((upper & 1) == 1))
    r = (upper + up.astype(np.uint64)) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def fine_k_bf16_levels(levels):
    """The hierarchy with the fine level's K rounded by round_bf16 (every
    other block and level, and all smoother data, unchanged)."""
    L0 = copy.copy(levels[0])
    K = L0.K.copy()
    K.data = round_bf16(K.data)
    L0.K = K
    return [L0] + list(levels[1:])
