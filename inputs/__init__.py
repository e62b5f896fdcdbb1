"""Seeded synthetic input generators shared by the oracle tests, the GPU tests and the bench.

This package only draws and assembles test matrices; it performs no step of the
factorization itself, so that the oracle and the HIP path stay independent.
"""
from .matrices import (  # noqa: F401
    spd_bbt,
    uniform01,
    tri_operand,
    wilkinson_growth,
    known_answer,
    zero_column,
    leader_perm,
    random_schedule,
    small_int_matrix,
    haar_spectrum,
    gaussian_rhs,
)
