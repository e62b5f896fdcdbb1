"""Pins of the refinement oracle (oracle/refine.py) against what the mathematics
fixes, and planted mistakes that the pins must catch (on the CPU).

* GMRES after k steps is the minimizer of ||z - Op d||_2 over the Krylov space
  span{z, Op z, ..., Op^{k-1} z}: checked against a brute-force least-squares
  solve over an explicit Krylov basis (Saad and Schultz 1986, the defining
  property).
* An operator with d distinct eigenvalues (diagonalizable) is solved exactly by
  step d; any nonsingular n x n operator by step n; the residual history never
  increases; the identity takes one step.
* Givens and the backward error: closed forms.
* Carson and Higham (2017): with FP32 factors and kappa = 1e8 (kappa u_32 > 1),
  LU-IR does not reach an FP64 backward error while GMRES-IR does, and its
  solution agrees with the FP64 solve.
"""
import numpy as np
import pytest

import inputs as G
import oracle as O
import oracle.refine as R


def _krylov_minimizer(Op, z, k):
    K = np.empty((z.shape[0], k))
    v = z.copy()
    for j in range(k):
        K[:, j] = v
        v = Op @ v
    Q, _ = np.linalg.qr(K)
    c, *_ = np.linalg.lstsq(Op @ Q, z, rcond=None)
    d = Q @ c
    return d, float(np.linalg.norm(z - Op @ d))


def krylov_pin_ok(seed=0, n=9, kmax=6) -> bool:
    rng = np.random.default_rng(seed)
    Op = np.eye(n) + 0.6 * rng.standard_normal((n, n)) / np.sqrt(n)
    z = rng.standard_normal(n)
    for k in range(1, kmax + 1):
        d, steps, hist = R.gmres(lambda v: Op @ v, z, k, 0.0)
        dref, res = _krylov_minimizer(Op, z, k)
        if steps != k:
            return False
        if np.abs(d - dref).max() > 1e-10 * np.abs(dref).max():
            return False
        if abs(hist[-1] - res) > 1e-10 * np.linalg.norm(z):
            return False
        if abs(hist[-1] - np.linalg.norm(z - Op @ d)) > 1e-10 * np.linalg.norm(z):
            return False
    return True


def distinct_eigenvalues_pin_ok(seed=1, n=12) -> bool:
    rng = np.random.default_rng(seed)
    S = rng.standard_normal((n, n))
    lam = np.array([2.0, -1.5, 3.0])[np.arange(n) % 3]   # three distinct eigenvalues
    Op = S @ np.diag(lam) @ np.linalg.inv(S)
    z = rng.standard_normal(n)
    d, steps, hist = R.gmres(lambda v: Op @ v, z, n, 1e-12)
    return steps <= 3 and np.linalg.norm(z - Op @ d) <= 1e-9 * np.linalg.norm(z)


def pins_pass() -> bool:
    try:
        if not krylov_pin_ok():
            return False
        if not distinct_eigenvalues_pin_ok():
            return False
        c, s, rho = R.givens(3.0, 4.0)
        if (c, s, rho) != (0.6, 0.8, 5.0):
            return False
        if R.backward_error(np.array([[2.0, 1.0], [0.0, 3.0]]), np.array([1.0, 1.0]),
                            np.array([3.0, 2.0])) != 1.0 / (3.0 * 1.0 + 3.0):
            return False
        return True
    except Exception:
        return False


def test_gmres_iterates_are_krylov_minimizers():
    assert krylov_pin_ok()
    assert krylov_pin_ok(seed=5, n=7, kmax=7)


def test_gmres_exact_at_number_of_distinct_eigenvalues():
    assert distinct_eigenvalues_pin_ok()


def test_gmres_exact_by_step_n_and_monotone_history():
    rng = np.random.default_rng(3)
    n = 6
    Op = rng.standard_normal((n, n)) + 3 * np.eye(n)
    z = rng.standard_normal(n)
    d, steps, hist = R.gmres(lambda v: Op @ v, z, n, 0.0)
    assert steps <= n
    assert np.linalg.norm(z - Op @ d) <= 1e-12 * np.linalg.norm(z)
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))


def test_gmres_identity_one_step_and_zero_rhs():
    z = np.arange(1.0, 6.0)
    d, steps, hist = R.gmres(lambda v: v, z, 10, 1e-14)
    assert steps == 1 and np.allclose(d, z, rtol=1e-15, atol=0)
    d, steps, hist = R.gmres(lambda v: v, np.zeros(4), 10, 1e-14)
    assert steps == 0 and not d.any()


def test_givens_and_backward_error_closed_forms():
    assert R.givens(3.0, 4.0) == (0.6, 0.8, 5.0)
    assert R.givens(0.0, 0.0) == (1.0, 0.0, 0.0)
    c, s, rho = R.givens(0.0, -2.0)
    assert (c, s, rho) == (0.0, -1.0, 2.0)
    A = np.array([[2.0, 1.0], [0.0, 3.0]])
    # r = b - A x = (3, 2) - (3, 3) = (0, -1); ||A||_inf = 3, ||x||_inf = 1, ||b||_inf = 3
    assert R.backward_error(A, np.array([1.0, 1.0]), np.array([3.0, 2.0])) == 1.0 / 6.0
    assert R.backward_error(np.zeros((2, 2)), np.zeros(2), np.zeros(2)) == 0.0


def test_refine_with_exact_factors_needs_at_most_one_correction():
    A = G.haar_spectrum(60, 1e3, seed=2)
    b = G.gaussian_rhs(60, 1, seed=3)[:, 0]
    F = A.copy()
    ipiv, info = O.getrf(F, "rl", nb=16)
    for solver in ("lu", "gmres", "auto"):
        x, outer, inner, berrs = R.refine(A, b, R.lu_solver(F, ipiv), tol=1e-14, solver=solver)
        assert outer in (0, 1) and berrs[-1] <= 1e-14


@pytest.mark.parametrize("n", [200, 300])
def test_gmres_ir_converges_where_lu_ir_does_not(n):
    A = G.haar_spectrum(n, 1e8, seed=0)
    b = G.gaussian_rhs(n, 1, seed=1)[:, 0]
    F32 = A.astype(np.float32)
    ipiv, info = O.getrf(F32, "rl", nb=32)
    assert info == 0 and F32.dtype == np.float32
    solve = R.lu_solver(F32, ipiv)
    _, outer_lu, _, berrs_lu = R.refine(A, b, solve, tol=1e-13, max_outer=10, solver="lu")
    x, outer, inner, berrs = R.refine(A, b, solve, tol=1e-13, max_outer=10, solver="gmres")
    assert outer_lu == -1 and min(berrs_lu) > 1e-13
    assert outer >= 1 and inner >= 2 and berrs[-1] <= 1e-13
    F = A.copy()
    ipiv64, _ = O.getrf(F, "rl", nb=32)
    x64 = O.getrs(F, ipiv64, b.reshape(-1, 1))[:, 0]
    assert np.abs(x - x64).max() <= 1e8 * 1e-14 * np.abs(x64).max()
    xa, outer_a, inner_a, berrs_a = R.refine(A, b, solve, tol=1e-13, max_outer=10, solver="auto")
    assert outer_a >= 1 and inner_a >= 1 and berrs_a[-1] <= 1e-13


def test_unmutated_refine_oracle_passes():
    assert pins_pass()


def _mgs_skips_last(V, k, w, H):
    for j in range(k):
        H[j, k] = V[j] @ w
        w = w - H[j, k] * V[j]
    return w


def _rotate_transposed(H, k, cs, sn):
    for j in range(k):
        a, b = H[j, k], H[j + 1, k]
        H[j, k] = cs[j] * a - sn[j] * b
        H[j + 1, k] = sn[j] * a + cs[j] * b


def _givens_wrong_sign(a, b):
    rho = float(np.hypot(a, b))
    return (1.0, 0.0, 0.0) if rho == 0.0 else (a / rho, -b / rho, rho)


def _back_sub_drops_coupling(H, g, steps):
    return np.array([g[i] / H[i, i] for i in range(steps)])


def _berr_without_b(A, x, b):
    r = b - A @ x
    return float(np.abs(r).max() / (np.abs(A).sum(axis=1).max() * np.abs(x).max()))


MUTATIONS = {
    "mgs_skips_last_vector": ("orthogonalize", _mgs_skips_last),
    "rotation_transposed": ("rotate_column", _rotate_transposed),
    "givens_wrong_sign": ("givens", _givens_wrong_sign),
    "back_substitution_drops_coupling": ("back_substitute", _back_sub_drops_coupling),
    "berr_without_b_norm": ("backward_error", _berr_without_b),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_refine_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(R, attr, fn)
    assert not pins_pass()
