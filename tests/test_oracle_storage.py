"""Pins of the oracle's bfloat16 storage rounding (the mixed-precision option
that stores the fine-level K of the V-cycle in bfloat16)."""
import numpy as np
import pytest

from oracle.storage import fine_k_bf16_levels, round_bf16


def test_bf16_rounding_hand_values():
    # bfloat16 keeps 7 mantissa bits: spacing 2^-7 on [1, 2)
    e = 2.0 ** -8
    cases = {
        1.0: 1.0,
        1.0 + e: 1.0,  # half-way, ties to the even neighbour 1.0
        1.0 + 3 * e: 1.0 + 4 * e,  # half-way between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
        1.0 + e + 2.0 ** -20: 1.0 + 2 * e,  # just above half-way
        1.0 + e - 2.0 ** -20: 1.0,  # just below
        -(1.0 + 3 * e): -(1.0 + 4 * e),
        0.0: 0.0,
        2.0 ** 100 * (1.0 + e): 2.0 ** 100,
        3.0: 3.0,
        1.0 / 3.0: 0.333984375,  # 0x3EAB: 0.0101010110 (binary) after rounding up
    }
    got = round_bf16(np.array(list(cases)))
    assert np.array_equal(got, np.array(list(cases.values())))


def test_bf16_rounding_bound_and_idempotence():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(100000) * np.exp(rng.uniform(-40, 40, 100000))
    r = round_bf16(x)
    # nearest rounding to 8 significant bits: relative error <= 2^-8 (plus the
    # FP32 step, far below)
    assert np.all(np.abs(r - x) <= (2.0 ** -8 + 2.0 ** -23) * np.abs(x))
    assert np.array_equal(round_bf16(r), r)
    # the representable values are exactly the FP32 words with a zero low half
    bits = r.astype(np.float32).view(np.uint32)
    assert np.all((bits & 0xFFFF) == 0)


def test_fine_k_rounding_touches_only_level0_k():
    from contactgen import make_workload
    from oracle.hierarchy import AMGOptions, build_hierarchy

    lv = build_hierarchy(make_workload("contact3d_6"), AMGOptions(max_levels=2))
    lb = fine_k_bf16_levels(lv)
    assert np.array_equal(lb[0].K.data, round_bf16(lv[0].K.data))
    assert np.array_equal(lb[0].K.indices, lv[0].K.indices)
    assert lb[0].G is lv[0].G and lb[0].atilde_inv is lv[0].atilde_inv and lb[1] is lv[1]
    assert not np.array_equal(lb[0].K.data, lv[0].K.data)
