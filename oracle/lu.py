"""Plain CPU oracle for the LU factorization with partial pivoting.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg
of the benchmark may import this module.  It shares no code with the HIP library.

What it computes (Catalan, Herrero, Quintana-Orti, Rodriguez-Sanchez and van de
Geijn, "A Case for Malleable Thread-Level Linear Algebra Libraries: The LU
Factorization with Partial Pivoting"):  for A in R^{m x n}, P A = L U with L unit
lower trapezoidal, U upper trapezoidal and P a row permutation chosen by partial
pivoting; the result overwrites A as {L\\U} (Section 3, opening paragraph).

The algorithms are the paper's loop-based variants, each step in the paper's
order and notation:
  * lu_unb     -- unblocked right-looking (Fig. "LU", left: rl1, rl2),
  * lu_blk_rl  -- blocked right-looking (Fig. "LU", right: RL1, RL2, RL3),
  * lu_blk_la  -- blocked right-looking with look-ahead (Fig. "LU_la_blk":
                  initial panel factorization, PF1-PF3 and RU1-RU2),
  * lu_blk_ll  -- blocked left-looking (Section 4.2: LL1, LL2, LL3).

Readings where the paper is silent (each also listed in the design notes):
  * Pivoting is left out of every figure (Section 3.1) but used in every code.
    It is taken as the standard rule: at column c pick the row with the largest
    |value| in the current column from the diagonal down, taking the FIRST such
    row on ties, and interchange ENTIRE rows (the L part on the left and the
    not-yet-factored part on the right).  Interchanges are recorded LAPACK-style:
    ipiv[c] = row swapped with row c at step c (0-based here).
  * A pivot that is exactly zero is recorded as info = c + 1 (first occurrence,
    1-based); the division rl1 is skipped and the factorization continues.
  * rl1 is a true division a21 / alpha11 (not a multiplication by a reciprocal).
  * The loop guard n(A_TL) < n(A) becomes n(A_TL) < min(m, n) so that wide
    matrices are handled; the last block is b = min(nb, min(m, n) - j).
  * In the look-ahead variant the interchanges found by the panel factorization
    (init or PF3) are applied to the columns outside that panel at the start of
    the next loop body ("row permutations" between iterations, Section 3.2).
  * In the left-looking variant the panel's columns are brought up to date with
    all earlier interchanges just before LL1 ("lazy"), or the interchanges are
    applied to the whole right part as they are found ("eager").  Both give the
    same factorization; the loop invariant differs and the checker takes a flag.
  * The inner (panel) factorization is LU_unb, or a blocked RL / LL with the
    inner block size b_i (Section 4.2); b_i = 1 or b_i >= b means LU_unb.

Arrays may be float64 (IEEE double, the paper's arithmetic) or numpy object
arrays of fractions.Fraction for exact arithmetic on tiny inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

RL, LL, LA = "rl", "ll", "la"
VARIANTS = (RL, LL, LA)


@dataclass
class Flops:
    """Operation counts by kind (one division, multiply or subtraction = 1 flop)."""

    panel: int = 0      # everything done inside panel factorizations (RL1/PF3/LL3)
    trsm: int = 0       # RL2 / PF1 / RU1 / LL1 outside panels
    gemm: int = 0       # RL3 / PF2 / RU2 / LL2 outside panels
    _in_panel: int = field(default=0, repr=False)

    @property
    def total(self) -> int:
        return self.panel + self.trsm + self.gemm

    def add(self, kind: str, n: int) -> None:
        if self._in_panel:
            self.panel += n
        else:
            setattr(self, kind, getattr(self, kind) + n)


def _is_exact(A) -> bool:
    return A.dtype == object


def iamax_first(x) -> int:
    """Index of the first entry of largest magnitude (ties -> smallest index)."""
    if not _is_exact(x):
        # numpy documents that argmax returns the first occurrence of the maximum
        return int(np.argmax(np.abs(x)))
    best, bestv = 0, abs(x[0])
    for i in range(1, len(x)):
        v = abs(x[i])
        if v > bestv:
            best, bestv = i, v
    return best


def swap_rows(A, r: int, p: int) -> None:
    """Interchange rows r and p of the 2-D view A (all of its columns)."""
    if r != p and A.shape[1] > 0:
        tmp = A[r, :].copy()
        A[r, :] = A[p, :]
        A[p, :] = tmp


def apply_interchanges(A, piv, row0: int = 0) -> None:
    """Apply interchanges in order: step c swaps rows row0+c and row0+piv[c]."""
    for c, p in enumerate(piv):
        swap_rows(A, row0 + c, row0 + p)


def trsm_unit_lower(L, B, fl: Flops | None = None):
    """Return trilu(L)^{-1} B by forward substitution.

    trilu(L) is the strictly lower part of L with ones on the diagonal (notation
    of Fig. "LU").  Row r of the result is B[r] - sum_{c<r} L[r, c] X[c].
    """
    b = L.shape[0]
    X = B.copy()
    for r in range(1, b):
        X[r, :] = X[r, :] - L[r, :r] @ X[:r, :]
    if fl is not None:
        fl.add("trsm", b * (b - 1) * B.shape[1])
    return X


def gemm_update(C, A, B, fl: Flops | None = None) -> None:
    """C := C - A B (in place)."""
    if C.size == 0 or A.shape[1] == 0:
        return
    C[...] = C - A @ B
    if fl is not None:
        fl.add("gemm", 2 * C.shape[0] * C.shape[1] * A.shape[1])


def lu_unb(A, fl: Flops | None = None, info: list | None = None, col0: int = 0):
    """Unblocked right-looking LU with partial pivoting, in place on A (m x n).

    Per column c (alpha11 = A[c, c]):  pivot search and interchange of entire rows,
    rl1  a21 := a21 / alpha11,  rl2  A22 := A22 - a21 a12^T.
    Returns the relative interchanges (list of ints).
    """
    m, n = A.shape
    piv = []
    for c in range(min(m, n)):
        p = c + iamax_first(A[c:, c])
        piv.append(p)
        swap_rows(A, c, p)
        alpha = A[c, c]
        a21 = A[c + 1:, c]
        a12 = A[c, c + 1:]
        if alpha != 0:
            A[c + 1:, c] = a21 / alpha                               # rl1
            if fl is not None:
                fl.add("panel", m - c - 1)
        elif info is not None and info[0] == 0:
            info[0] = col0 + c + 1
        if m - c - 1 > 0 and n - c - 1 > 0:
            A[c + 1:, c + 1:] = A[c + 1:, c + 1:] - np.outer(A[c + 1:, c], a12)  # rl2
            if fl is not None:
                fl.add("panel", 2 * (m - c - 1) * (n - c - 1))
    return piv


def schedule_from(mn: int, nb: int | None = None, schedule=None) -> list[int]:
    """Block sizes b_0, b_1, ... covering min(m, n) columns.

    With a constant nb the last block is min(nb, min(m,n) - j).  An explicit
    schedule (any positive sizes, e.g. ones an early-terminated panel produced)
    is truncated/trimmed so that it covers exactly min(m, n) columns.
    """
    out, j = [], 0
    if schedule is not None:
        for b in schedule:
            if j >= mn:
                break
            b = min(int(b), mn - j)
            if b <= 0:
                raise ValueError("block sizes must be positive")
            out.append(b)
            j += b
        if j < mn:
            raise ValueError("schedule does not cover min(m, n) columns")
        return out
    if nb is None or nb < 1:
        raise ValueError("nb must be >= 1")
    while j < mn:
        b = min(nb, mn - j)
        out.append(b)
        j += b
    return out


def factor_panel(P, inner=None, fl: Flops | None = None, info=None, col0: int = 0):
    """Factor a panel [A11; A21] in place: LU_unb, or a blocked inner LU.

    inner: None | ("unb",) | ("rl", b_i) | ("ll", b_i).  b_i = 1 or b_i >= the
    panel width selects LU_unb (Section 4.2).
    """
    if fl is not None:
        fl._in_panel += 1
    try:
        width = P.shape[1]
        if inner is None or inner[0] == "unb" or inner[1] <= 1 or inner[1] >= width:
            return lu_unb(P, fl, info, col0)
        kind, bi = inner[0], int(inner[1])
        if kind == RL:
            return lu_blk_rl(P, nb=bi, fl=fl, info=info, col0=col0)[0]
        if kind == LL:
            return lu_blk_ll(P, nb=bi, fl=fl, info=info, col0=col0)[0]
        raise ValueError(f"unknown inner variant {kind!r}")
    finally:
        if fl is not None:
            fl._in_panel -= 1


def lu_blk_rl(A, nb=None, schedule=None, inner=None, fl=None, info=None,
              on_iter=None, iters_limit=None, col0: int = 0):
    """Blocked right-looking LU (Fig. "LU", right), in place.

    Per iteration with A11 b x b:
      RL1  [A11; A21] := LU([A11; A21])   (+ its interchanges applied to the
                                            rows j.. of every other column)
      RL2  A12 := trilu(A11)^{-1} A12
      RL3  A22 := A22 - A21 A12
    Returns (ipiv, info) with ipiv 0-based and relative to A's first row.
    """
    m, n = A.shape
    mn = min(m, n)
    info = [0] if info is None else info
    ipiv: list[int] = []
    j = 0
    for it, b in enumerate(schedule_from(mn, nb, schedule)):
        if iters_limit is not None and it >= iters_limit:
            break
        pv = factor_panel(A[j:, j:j + b], inner, fl, info, col0 + j)        # RL1
        apply_interchanges(A[j:, :j], pv)
        apply_interchanges(A[j:, j + b:], pv)
        ipiv += [j + p for p in pv]
        A[j:j + b, j + b:] = trsm_unit_lower(A[j:j + b, j:j + b],
                                             A[j:j + b, j + b:], fl)          # RL2
        gemm_update(A[j + b:, j + b:], A[j + b:, j:j + b], A[j:j + b, j + b:], fl)  # RL3
        j += b
        if on_iter is not None:
            on_iter(it, j, A, list(ipiv))
    return ipiv, info[0]


def lu_blk_la(A, nb=None, schedule=None, inner=None, fl=None, info=None,
              on_iter=None, iters_limit=None, col0: int = 0):
    """Blocked right-looking LU with look-ahead of depth one (Fig. "LU_la_blk").

    Before the loop the first panel A_BR^P is factored.  Each loop body, with
    A11 the already factored panel's diagonal block, first applies that panel's
    interchanges to the columns outside it, then splits (A12; A22) into the
    next b columns (P) and the remainder (R):
      PF1  A12^P := trilu(A11)^{-1} A12^P        RU1  A12^R := trilu(A11)^{-1} A12^R
      PF2  A22^P := A22^P - A21 A12^P            RU2  A22^R := A22^R - A21 A12^R
      PF3  A22^P := LU(A22^P)
    The two columns of operations touch disjoint columns, so their order here
    does not matter.  on_iter(k, j, A, ipiv, pending) is called at the top of
    each following loop test, when the next panel is factored but its
    interchanges are still pending.
    """
    m, n = A.shape
    mn = min(m, n)
    info = [0] if info is None else info
    sched = schedule_from(mn, nb, schedule) if mn > 0 else []
    if not sched:
        return [], info[0]
    b = sched[0]
    pend = factor_panel(A[0:, 0:b], inner, fl, info, col0)                   # init
    ipiv: list[int] = []
    j, k = 0, 0
    while j < mn:
        if iters_limit is not None and k >= iters_limit:
            break
        apply_interchanges(A[j:, :j], pend)
        apply_interchanges(A[j:, j + b:], pend)
        ipiv += [j + p for p in pend]
        jn = j + b
        bp = sched[k + 1] if k + 1 < len(sched) else 0
        A11, A21 = A[j:jn, j:jn], A[jn:, j:jn]
        nxt = []
        if bp > 0:
            A[j:jn, jn:jn + bp] = trsm_unit_lower(A11, A[j:jn, jn:jn + bp], fl)        # PF1
            gemm_update(A[jn:, jn:jn + bp], A21, A[j:jn, jn:jn + bp], fl)                # PF2
            nxt = factor_panel(A[jn:, jn:jn + bp], inner, fl, info, col0 + jn)          # PF3
        A[j:jn, jn + bp:] = trsm_unit_lower(A11, A[j:jn, jn + bp:], fl)                 # RU1
        gemm_update(A[jn:, jn + bp:], A21, A[j:jn, jn + bp:], fl)                        # RU2
        j, b, pend, k = jn, bp, nxt, k + 1
        if on_iter is not None:
            on_iter(k - 1, j, A, list(ipiv), list(pend))
    if iters_limit is not None and j < mn:
        # stopped early: the factored-but-pending panel's interchanges are
        # reported (relative to row j) after the completed ones
        ipiv += [j + p for p in pend]
    return ipiv, info[0]


def lu_blk_ll(A, nb=None, schedule=None, inner=None, fl=None, info=None,
              on_iter=None, iters_limit=None, lazy: bool = True, col0: int = 0):
    """Blocked left-looking LU (Section 4.2), in place.

    Per iteration with the current panel [A01; A11; A21] of b columns:
      (its columns first receive every earlier interchange when lazy)
      LL1  A01 := trilu(A00)^{-1} A01
      LL2  [A11; A21] := [A11; A21] - [A10; A20] A01
      LL3  [A11; A21] := LU([A11; A21])   (+ interchanges applied to the left
                                            columns, and to the right columns
                                            too when not lazy)
    Nothing to the right of the panel is read or written when lazy.  For a wide
    matrix (n > m) the columns past min(m, n) are brought up to date at the end
    (interchanges, then LL1 with the full trilu(A00)).
    """
    m, n = A.shape
    mn = min(m, n)
    info = [0] if info is None else info
    ipiv: list[int] = []
    j = 0
    completed = True
    for it, b in enumerate(schedule_from(mn, nb, schedule) if mn > 0 else []):
        if iters_limit is not None and it >= iters_limit:
            completed = False
            break
        if lazy:
            apply_interchanges(A[:, j:j + b], ipiv)
        A[0:j, j:j + b] = trsm_unit_lower(A[0:j, 0:j], A[0:j, j:j + b], fl)          # LL1
        gemm_update(A[j:, j:j + b], A[j:, 0:j], A[0:j, j:j + b], fl)                # LL2
        pv = factor_panel(A[j:, j:j + b], inner, fl, info, col0 + j)                # LL3
        apply_interchanges(A[j:, :j], pv)
        if not lazy:
            apply_interchanges(A[j:, j + b:], pv)
        ipiv += [j + p for p in pv]
        j += b
        if on_iter is not None:
            on_iter(it, j, A, list(ipiv))
    if completed and n > mn:
        if lazy:
            apply_interchanges(A[:, mn:], ipiv)
        A[0:mn, mn:] = trsm_unit_lower(A[0:mn, 0:mn], A[0:mn, mn:], fl)
    return ipiv, info[0]


def getrf(A, variant: str = RL, nb=None, schedule=None, inner=None, fl=None,
          on_iter=None, iters_limit=None, lazy: bool = True):
    """Dispatch to a variant.  Returns (ipiv, info); A is overwritten by {L\\U}."""
    if variant == RL:
        return lu_blk_rl(A, nb, schedule, inner, fl, None, on_iter, iters_limit)
    if variant == LA:
        return lu_blk_la(A, nb, schedule, inner, fl, None, on_iter, iters_limit)
    if variant == LL:
        return lu_blk_ll(A, nb, schedule, inner, fl, None, on_iter, iters_limit, lazy)
    raise ValueError(f"unknown variant {variant!r}")


def unpack(F):
    """Split a packed {L\\U} (m x n) into L (m x k, unit lower) and U (k x n)."""
    m, n = F.shape
    k = min(m, n)
    one = F.dtype.type(1) if not _is_exact(F) else 1
    L = np.tril(F[:, :k], -1)
    for i in range(k):
        L[i, i] = one
    U = np.triu(F[:k, :])
    return L, U


def permutation_of(ipiv, m: int) -> np.ndarray:
    """Row order produced by the sequential interchanges: (P A)[i] = A[perm[i]]."""
    perm = np.arange(m)
    for c, p in enumerate(ipiv):
        perm[c], perm[p] = perm[p], perm[c]
    return perm


def trsm(T, B, uplo: str = "L", diag: str = "U"):
    """Return op(T)^{-1} B for a triangular T (left side, no transpose).

    uplo 'L': forward substitution with the lower triangle of T;
    uplo 'U': back substitution with the upper triangle.
    diag 'U': unit diagonal assumed (the stored diagonal is not read);
    diag 'N': divide by the stored diagonal.
    """
    nrow = T.shape[0]
    X = B.copy()
    order = range(nrow) if uplo == "L" else range(nrow - 1, -1, -1)
    for r in order:
        if uplo == "L":
            if r > 0:
                X[r, :] = X[r, :] - T[r, :r] @ X[:r, :]
        else:
            if r < nrow - 1:
                X[r, :] = X[r, :] - T[r, r + 1:] @ X[r + 1:, :]
        if diag == "N":
            X[r, :] = X[r, :] / T[r, r]
    return X


def getrs(F, ipiv, B):
    """Solve A X = B from the factorization P A = L U held in F (square).

    X = U^{-1} L^{-1} (P B): apply the interchanges to B, then the unit lower
    and the upper triangular solves.
    """
    X = B.copy()
    apply_interchanges(X, ipiv)
    X = trsm(F, X, "L", "U")
    X = trsm(F, X, "U", "N")
    return X


def flops_lu_exact(m: int, n: int) -> int:
    """Exact operation count of LU_unb on an m x n matrix (no zero pivots):
    sum over columns c < min(m, n) of (m-c-1) divisions plus 2(m-c-1)(n-c-1)
    for the rank-1 update.  Its leading terms are m n^2 - n^3 / 3 (Section 3.1).
    """
    return sum((m - c - 1) + 2 * (m - c - 1) * (n - c - 1) for c in range(min(m, n)))
