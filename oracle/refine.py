"""Plain CPU oracle for iterative refinement: LU-IR and GMRES-IR.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg
of the benchmark may import this module.  It shares no code with the HIP library.

The precision ladder refines a solution of A x = b whose LU factors were computed
with low-precision trailing products.  The paper's factorization (Section 3) is
the preconditioner; the refinement itself is taken from the literature:

  * LU-IR (classical iterative refinement, Wilkinson; in the mixed-precision
    form of Langou et al. 2006):  r_i = b - A x_i,  solve (LU) d_i = P r_i,
    x_{i+1} = x_i + d_i.
  * GMRES-IR (Carson and Higham, SIAM J. Sci. Comput. 39(6), 2017, and
    40(2), 2018):  the correction equation A d_i = r_i is solved by GMRES on
    the left-preconditioned system  M^{-1} A d = M^{-1} r_i,  M = P^T L U the
    low-precision factors, applied in FP64.  GMRES (Saad and Schultz 1986):
    Arnoldi with modified Gram-Schmidt builds an orthonormal basis V of the
    Krylov space K_k(M^{-1} A, z), z = M^{-1} r_i, with the Hessenberg matrix
    H; Givens rotations reduce H to triangular form as it grows, so that
    |g_{k+1}| is the residual norm || z - M^{-1} A d_k ||_2 of the minimizer
    d_k = V_k y_k over K_k, and the iteration stops when it falls below
    gmres_tol * ||z||_2 or at the Krylov dimension limit m.

Stopping rule of both (the same as the library's):
    berr_i = ||r_i||_inf / (||A||_inf ||x_i||_inf + ||b||_inf) <= tol.
Everything is FP64 (numpy); the low-precision factors enter through
`solve_low`, a callable r -> M^{-1} r.
"""
from __future__ import annotations

import numpy as np

from .lu import getrs


def backward_error(A, x, b) -> float:
    """||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf) (componentwise max norms)."""
    r = b - A @ x
    den = np.abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()
    rn = np.abs(r).max()
    return float(rn / den) if den > 0 else (0.0 if rn == 0 else float("inf"))


def givens(a: float, b: float):
    """(c, s, rho) with [c s; -s c] [a; b] = [rho; 0], rho = sqrt(a^2 + b^2) >= 0."""
    rho = float(np.hypot(a, b))
    if rho == 0.0:
        return 1.0, 0.0, 0.0
    return a / rho, b / rho, rho


def orthogonalize(V, k: int, w, H):
    """Modified Gram-Schmidt: w := w - sum_j (v_j . w) v_j over j = 0..k, one
    basis vector at a time, the coefficients into column k of H."""
    for j in range(k + 1):
        H[j, k] = V[j] @ w
        w = w - H[j, k] * V[j]
    return w


def rotate_column(H, k: int, cs, sn) -> None:
    """Apply the rotations of steps 0..k-1 to column k of H, in order."""
    for j in range(k):
        a, b = H[j, k], H[j + 1, k]
        H[j, k] = cs[j] * a + sn[j] * b
        H[j + 1, k] = -sn[j] * a + cs[j] * b


def back_substitute(H, g, steps: int):
    """y with H[:steps, :steps] y = g[:steps] (H upper triangular there)."""
    y = np.zeros(steps)
    for i in range(steps - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:steps] @ y[i + 1:]) / H[i, i]
    return y


def gmres(apply_op, z, m: int, tol: float):
    """GMRES from d_0 = 0 for Op d = z, at most m steps.

    Returns (d, steps, history) where history[k] = |g_{k+1}| after step k+1,
    the residual norm of the minimizer over the Krylov space of dimension k+1.
    Stops when |g_{k+1}| <= tol * ||z||_2, at m steps, or at a breakdown
    (h_{k+1,k} = 0: the Krylov space is invariant and d_k is exact).
    """
    n = z.shape[0]
    beta = float(np.sqrt(z @ z))
    if beta == 0.0 or m == 0:
        return np.zeros(n), 0, []
    V = np.zeros((m + 1, n))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    V[0] = z / beta
    hist = []
    steps = 0
    for k in range(m):
        w = orthogonalize(V, k, apply_op(V[k]), H)
        hnext = float(np.sqrt(w @ w))
        H[k + 1, k] = hnext
        if hnext != 0.0:
            V[k + 1] = w / hnext
        rotate_column(H, k, cs, sn)
        cs[k], sn[k], H[k, k] = givens(H[k, k], H[k + 1, k])
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        hist.append(abs(g[k + 1]))
        steps = k + 1
        if abs(g[k + 1]) <= tol * beta or hnext == 0.0:
            break
    return V[:steps].T @ back_substitute(H, g, steps), steps, hist


def refine(A, b, solve_low, tol: float = 1e-13, max_outer: int = 10, solver: str = "gmres",
           m: int = 64, gmres_tol: float = 1e-6, switch_ratio: float = 0.5):
    """Iterative refinement of A x = b from x_0 = solve_low(b).

    solver = "lu":     LU-IR corrections d = solve_low(r);
             "gmres":  GMRES-IR corrections (GMRES on solve_low(A v) = solve_low(r));
             "auto":   LU-IR while each correction shrinks the backward error by
                       at least switch_ratio, GMRES-IR from the first step that
                       does not (and for the rest of the solve).
    Returns (x, outer, inner, berrs): outer = corrections made before berr <= tol
    (-1 if max_outer corrections did not reach it), inner = total GMRES steps,
    berrs = the backward error of every iterate.
    """
    x = solve_low(b)
    mode = "gmres" if solver == "gmres" else "lu"
    inner = 0
    berrs = []
    for i in range(max_outer + 1):
        berr = backward_error(A, x, b)
        berrs.append(berr)
        if berr <= tol:
            return x, i, inner, berrs
        if i == max_outer:
            break
        if solver == "auto" and mode == "lu" and i > 0 and not (berr <= switch_ratio * berrs[-2]):
            mode = "gmres"
        r = b - A @ x
        z = solve_low(r)
        if mode == "lu":
            d = z
        else:
            d, k, _ = gmres(lambda v: solve_low(A @ v), z, m, gmres_tol)
            inner += k
        x = x + d
    return x, -1, inner, berrs


def lu_solver(F, ipiv):
    """r -> (P^T L U)^{-1} r from packed factors F (any float dtype), in FP64."""
    F64 = np.asarray(F, dtype=np.float64)

    def solve(r):
        return getrs(F64, ipiv, np.asarray(r, dtype=np.float64).reshape(-1, 1))[:, 0]

    return solve
