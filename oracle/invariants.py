"""Loop-invariant and postcondition checks for the LU variants.

TEST INFRASTRUCTURE ONLY (see oracle/lu.py).

The paper's worksheet leaves the precondition, postcondition and invariant
slots blank for LU (Section 3.1, FLAME worksheet).  They are derived here and
checked only through products of the current state, never by solving:

  Precondition   A = A_hat (m x n).
  Postcondition  A = {L\\U} with P A_hat = L U.

  With A_hat' = (interchanges recorded so far) applied to A_hat, and the 2x2
  partition of the state at n(A_TL) = j:

  RL (after an iteration):
      L_TL U_TL = A_hat'_TL,   L_TL A_TR = A_hat'_TR,   A_BL U_TL = A_hat'_BL,
      A_BR + A_BL A_TR = A_hat'_BR.
  LA (top of the loop, next panel of b' columns factored, its interchanges
      P_P still pending):  the RL relations for TL, TR and BL, and with
      S = A_hat'_BR - A_BL A_TR:  P_P S^P = L_P U_P  ({L_P\\U_P} stored in
      A_BR^P)  and  A_BR^R = S^R.
  LL (after an iteration; lazy: nothing right of the panel has been touched):
      L_TL U_TL = A_hat'_TL,   A_BL U_TL = A_hat'_BL,
      [A_TR; A_BR] = A_hat[:, j:]      (lazy)   or   A_hat'[:, j:]   (eager).

Every check returns the largest normwise relative discrepancy found (0 when
exact); exact (Fraction) arrays must give exactly 0.
"""
from __future__ import annotations

import numpy as np

from .lu import apply_interchanges, unpack


def _rel(X, Y, scale):
    if X.size == 0:
        return 0.0
    D = X - Y
    if D.dtype == object:
        return 0.0 if all(d == 0 for d in D.ravel()) else float("inf")
    num = np.linalg.norm(D)
    return float(num / scale) if scale > 0 else float(num)


def _permuted(Ahat, ipiv):
    Ap = Ahat.copy()
    apply_interchanges(Ap, ipiv)
    return Ap


def _tl_factors(A, j):
    T = A[:j, :j]
    L, U = unpack(T) if j > 0 else (T, T)
    return L, U


def check_rl(Ahat, A, ipiv, j) -> float:
    scale = float(np.linalg.norm(np.asarray(Ahat, dtype=float))) or 1.0
    Ap = _permuted(Ahat, ipiv)
    L, U = _tl_factors(A, j)
    errs = [
        _rel(L @ U, Ap[:j, :j], scale),
        _rel(L @ A[:j, j:], Ap[:j, j:], scale),
        _rel(A[j:, :j] @ U, Ap[j:, :j], scale),
        _rel(A[j:, j:] + A[j:, :j] @ A[:j, j:], Ap[j:, j:], scale),
    ]
    return max(errs)


def check_la(Ahat, A, ipiv, pend, j, bp) -> float:
    scale = float(np.linalg.norm(np.asarray(Ahat, dtype=float))) or 1.0
    Ap = _permuted(Ahat, ipiv)
    L, U = _tl_factors(A, j)
    errs = [
        _rel(L @ U, Ap[:j, :j], scale),
        _rel(L @ A[:j, j:], Ap[:j, j:], scale),
        _rel(A[j:, :j] @ U, Ap[j:, :j], scale),
    ]
    S = Ap[j:, j:] - A[j:, :j] @ A[:j, j:]
    if bp > 0:
        SP = S[:, :bp].copy()
        apply_interchanges(SP, pend)
        LP, UP = unpack(A[j:, j:j + bp])
        errs.append(_rel(LP @ UP, SP, scale))
    errs.append(_rel(A[j:, j + bp:], S[:, bp:], scale))
    return max(errs)


def check_ll(Ahat, A, ipiv, j, lazy=True) -> float:
    scale = float(np.linalg.norm(np.asarray(Ahat, dtype=float))) or 1.0
    Ap = _permuted(Ahat, ipiv)
    L, U = _tl_factors(A, j)
    right = Ahat[:, j:] if lazy else Ap[:, j:]
    errs = [
        _rel(L @ U, Ap[:j, :j], scale),
        _rel(A[j:, :j] @ U, Ap[j:, :j], scale),
        _rel(A[:, j:], right, scale),
    ]
    return max(errs)


def postcondition(Ahat, F, ipiv) -> dict:
    """Residual and structure of a finished factorization F = {L\\U}."""
    m, n = Ahat.shape
    L, U = unpack(F)
    PA = _permuted(Ahat, ipiv)
    R = PA - L @ U
    if R.dtype == object:
        exact = all(r == 0 for r in R.ravel())
        lmax = max((abs(x) for x in np.tril(F[:, :min(m, n)], -1).ravel()), default=0)
        return {"exact": exact, "l_max": lmax}
    Af = np.asarray(Ahat, dtype=float)
    eps = np.finfo(float).eps
    nrm_f = np.linalg.norm(Af)
    nrm_1 = np.linalg.norm(Af, 1) if Af.size else 0.0
    k = min(m, n)
    lmax = float(np.max(np.abs(np.tril(F[:, :k], -1)))) if k > 0 and m > 1 else 0.0
    return {
        "rel_frob": float(np.linalg.norm(R) / nrm_f) if nrm_f > 0 else 0.0,
        "scaled_1": float(np.linalg.norm(R, 1) / (max(m, n) * eps * nrm_1)) if nrm_1 > 0 else 0.0,
        "l_max": lmax,
    }
