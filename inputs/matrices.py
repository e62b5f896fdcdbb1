"""Seeded host-side matrix recipes (numpy PCG64).

Every function returns a C-ordered float64 array: element (i, j) of an m x n
matrix sits at offset i*n + j, i.e. the row-major layout the library's C ABI
takes.  Nothing here factors, solves or pivots.

Recipes
-------
spd_bbt(n, seed)        A = B B^T + n I, B ~ N(0, 1)  (the symmetric positive
                        definite workload; partial pivoting makes no interchange
                        on it in practice).
uniform01(m, n, seed)   entries uniform in (0, 1): the distribution of the paper's
                        experiments (Section "Experimental Evaluation"); it makes
                        an interchange at nearly every column.
tri_operand(n, seed)    lower triangle of spd_bbt(n, seed) with the diagonal
                        replaced by U[1, 2] draws (triangular-solve operand).
wilkinson_growth(n)     1 on the diagonal, -1 strictly below, 1 in the last
                        column: every pivot search is an exact tie.
known_answer(m, n, s)   A = Pi^T L U with dyadic L (|l| <= 7/8, entries k/8) and
                        small-integer U, so that every step of elimination is
                        exact in binary floating point and partial pivoting must
                        return exactly Pi, L and U.
zero_column(n, s, c)    known_answer with row c of U set to zero: the pivot
                        candidates of column c are all exactly zero (info = c+1)
                        and elimination stays exact.
haar_spectrum(n, k, s)  A = Q diag(sv) Q^T with Q Haar-distributed orthogonal (QR
                        of a Gaussian matrix, column signs fixed by diag(R)) and
                        sv log-spaced from 1 down to 1/k: 2-norm condition
                        number k (the mixed-precision workload).
gaussian_rhs(n, r, s)   right-hand sides ~ N(0, 1), n x r.
"""
from __future__ import annotations

import numpy as np


def _rng(seed, *salt):
    return np.random.default_rng([int(seed), *[int(x) for x in salt]])


def spd_bbt(n: int, seed: int = 0) -> np.ndarray:
    rng = _rng(seed)
    b = rng.standard_normal((n, n))
    a = b @ b.T
    a[np.diag_indices(n)] += float(n)
    return np.ascontiguousarray(a)


def uniform01(m: int, n: int | None = None, seed: int = 0) -> np.ndarray:
    n = m if n is None else n
    rng = _rng(seed, 7)
    a = rng.random((m, n))
    # default_rng().random draws from [0, 1); move an exact 0 (probability 2^-53)
    # into the open interval so the recipe matches "uniform in (0, 1)".
    a[a == 0.0] = np.nextafter(0.0, 1.0)
    return np.ascontiguousarray(a)


def tri_operand(n: int, seed: int = 0) -> np.ndarray:
    t = np.tril(spd_bbt(n, seed))
    rng = _rng(seed, 11)
    t[np.diag_indices(n)] = rng.uniform(1.0, 2.0, n)
    return np.ascontiguousarray(t)


def wilkinson_growth(n: int) -> np.ndarray:
    w = np.eye(n) - np.tril(np.ones((n, n)), -1)
    w[:, n - 1] = 1.0
    return np.ascontiguousarray(w)


def known_answer(m: int, n: int | None = None, seed: int = 0, perm=None):
    """Return (A, perm, L, U) with A[perm[i], :] = (L @ U)[i, :].

    `perm` (optional) fixes where each row of L U lands; by default it is a
    seeded random permutation.

    L is m x k unit lower trapezoidal (k = min(m, n)) with off-diagonal entries
    in {-7/8, ..., 7/8}; U is k x n upper trapezoidal with integer entries in
    [-8, 8] and a nonzero diagonal.  Products and sums of such numbers stay
    dyadic and small, so elimination in any order is exact in binary64.
    """
    n = m if n is None else n
    k = min(m, n)
    rng = _rng(seed, 3)
    L = np.zeros((m, k))
    for j in range(k):
        L[j, j] = 1.0
        L[j + 1:, j] = rng.integers(-7, 8, m - j - 1) / 8.0
    U = np.triu(rng.integers(-8, 9, (k, n)).astype(np.float64))
    d = rng.integers(1, 9, k) * rng.choice([-1.0, 1.0], k)
    U[np.arange(k), np.arange(k)] = d
    perm = rng.permutation(m) if perm is None else np.asarray(perm, dtype=np.int64)
    LU = L @ U
    A = np.empty((m, n))
    A[perm, :] = LU
    return np.ascontiguousarray(A), perm, L, U


def zero_column(n: int, seed: int = 0, col: int = 0):
    """known_answer(n, n, seed) with row `col` of U zeroed (an exactly zero pivot)."""
    k = n
    rng = _rng(seed, 3)
    L = np.zeros((n, k))
    for j in range(k):
        L[j, j] = 1.0
        L[j + 1:, j] = rng.integers(-7, 8, n - j - 1) / 8.0
    U = np.triu(rng.integers(-8, 9, (k, n)).astype(np.float64))
    d = rng.integers(1, 9, k) * rng.choice([-1.0, 1.0], k)
    U[np.arange(k), np.arange(k)] = d
    U[col, :] = 0.0
    perm = rng.permutation(n)
    # keep row `col` of A where the all-zero pivot search leaves it (first index
    # on ties), so that every later step still follows perm exactly
    at = int(np.flatnonzero(perm == col)[0])
    perm[at], perm[col] = perm[col], perm[at]
    A = np.empty((n, n))
    A[perm, :] = L @ U
    return np.ascontiguousarray(A)


def leader_perm(m: int, k: int, split: int, fail_at, seed: int = 0):
    """A permutation whose first k entries lie below `split`, except entry
    `fail_at` (if not None), which lies at or above it."""
    rng = _rng(seed, 17)
    low = rng.permutation(split)
    high = split + rng.permutation(m - split)
    head = list(low[:k])
    if fail_at is not None:
        head[fail_at] = high[0]
        rest = list(low[k:]) + list(high[1:]) + [low[fail_at]]
    else:
        rest = list(low[k:]) + list(high)
    rest = list(rng.permutation(np.array(rest)))
    return np.array(head + rest, dtype=np.int64)


def small_int_matrix(m: int, n: int, seed: int = 0, lo: int = -3, hi: int = 3) -> np.ndarray:
    """Small-integer entries: frequent exact ties among pivot candidates."""
    rng = _rng(seed, 5)
    return np.ascontiguousarray(rng.integers(lo, hi + 1, (m, n)).astype(np.float64))


def random_schedule(total: int, seed: int = 0, max_b: int = 8) -> list[int]:
    """A random sequence of positive block sizes that sums to `total`."""
    rng = _rng(seed, 13)
    out, left = [], total
    while left > 0:
        b = int(rng.integers(1, max_b + 1))
        b = min(b, left)
        out.append(b)
        left -= b
    return out


def haar_spectrum(n: int, cond: float, seed: int = 0) -> np.ndarray:
    rng = _rng(seed, 11)
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    sv = np.logspace(0.0, -np.log10(float(cond)), n)
    return np.ascontiguousarray((q * sv[None, :]) @ q.T)


def gaussian_rhs(n: int, nrhs: int = 1, seed: int = 1) -> np.ndarray:
    return np.ascontiguousarray(_rng(seed, 13).standard_normal((n, nrhs)))
