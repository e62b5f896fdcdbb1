"""CPU oracle for the blocked LU variants: TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may import
or execute anything in this package.  The product library never does; it shares
no code, header, table or helper with it.
"""
from .lu import (  # noqa: F401
    RL, LL, LA, VARIANTS, Flops,
    lu_unb, lu_blk_rl, lu_blk_la, lu_blk_ll, getrf, getrs, trsm,
    trsm_unit_lower, unpack, permutation_of, apply_interchanges, schedule_from,
    flops_lu_exact, iamax_first,
)
from . import invariants, refine  # noqa: F401
